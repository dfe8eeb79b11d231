"""Build and bind the atomic-throughput probe (measure/atomic_probe.hip) for profiling."""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "atomic_probe.hip")
LIB = os.path.join(HERE, "libperf_probe.so")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

_lib = None


def build() -> str:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    tmp = LIB + ".tmp"
    proc = subprocess.run([hipcc] + FLAGS + ["-o", tmp, SRC], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                          text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{proc.stdout}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with measure.probe.build()")
        lib = ctypes.CDLL(LIB)
        lib.probe_atomic_add.restype = ctypes.c_int32
        lib.probe_atomic_add.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p]
        _lib = lib
    return _lib


def atomic_add(y_ptr: int, n: int, reps: int, stride: int, stream) -> None:
    rc = load().probe_atomic_add(ctypes.c_void_p(y_ptr), n, reps, stride, stream)
    if rc != 0:
        raise RuntimeError(f"probe_atomic_add failed ({rc})")
