"""ctypes binding of include/perf_gn.h: the same names, argument marshalling only.

Every computation happens in libperf_gn.so (HIP kernels for gfx950).  If the
library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libperf_gn.so")

PERF_MAX_LAYERS = 8
PERF_MAX_PCG = 256
PERF_MLP_NW = 64 * 16 + 64 + 64 * 64 + 64 + 16 * 64 + 16
PERF_MLP_NNORM = 32
PERF_MLP_NFEAT = 6

PERF_OK, PERF_EINVAL, PERF_ENOMEM, PERF_EDEVICE, PERF_ENUMERIC, PERF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PERF_F32, PERF_BF16 = 0, 1
PERF_PRECOND_NONE, PERF_PRECOND_JACOBI, PERF_PRECOND_BLOCK4, PERF_PRECOND_LEARNED = 0, 1, 2, 3
PERF_FLAG_BREAKDOWN, PERF_FLAG_STALL, PERF_FLAG_CONVERGED, PERF_FLAG_LS_CAPPED, PERF_FLAG_NO_DESCENT = 1, 2, 4, 8, 16
PERF_FLAG_FALLBACK = 32


class perf_scene_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3),
        ("n_layers", ctypes.c_int32), ("env_w", ctypes.c_int32), ("env_h", ctypes.c_int32),
        ("layer_radius", ctypes.c_float * PERF_MAX_LAYERS),
        ("step_vox", ctypes.c_float),
        ("param_dtype", ctypes.c_int32),
        ("background", ctypes.c_float * 3),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("checks", ctypes.c_int32),
        ("learned", ctypes.c_int32),
        ("aux_lambda", ctypes.c_float),
        ("render_threshold", ctypes.c_float),
    ]


class perf_camera(ctypes.Structure):
    _fields_ = [
        ("origin", ctypes.c_float * 3),
        ("rot", ctypes.c_float * 9),
        ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
    ]


class perf_pcg_opts(ctypes.Structure):
    _fields_ = [
        ("max_iters", ctypes.c_int32),
        ("rel_tol", ctypes.c_double),
        ("abs_eps", ctypes.c_double),
        ("stall_ratio", ctypes.c_double),
        ("precond", ctypes.c_int32),
        ("line_search", ctypes.c_int32),
        ("ls_factor", ctypes.c_float),
        ("ls_max", ctypes.c_int32),
    ]


class perf_gn_stats(ctypes.Structure):
    _fields_ = [
        ("F_before", ctypes.c_double), ("F_after", ctypes.c_double), ("gamma", ctypes.c_double),
        ("pcg_iters", ctypes.c_int32), ("ls_trials", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("fallback_iters", ctypes.c_int32),
        ("R0", ctypes.c_double),
        ("R", ctypes.c_double * PERF_MAX_PCG),
        ("alpha", ctypes.c_double * PERF_MAX_PCG),
        ("beta", ctypes.c_double * PERF_MAX_PCG),
        ("pAp", ctypes.c_double * PERF_MAX_PCG),
        ("ms_phase", ctypes.c_float * 8),
    ]


# (name, restype, argtypes) for every function the header declares
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = [
    ("perf_workspace_bytes", ctypes.c_size_t, [_P, _I32]),
    ("perf_init_scene", _I32, [_P, _P, _I32, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    ("perf_set_targets", _I32, [_P, _P]),
    ("perf_set_stream", _I32, [_P, _P]),
    ("perf_scene_sizes", _I32, [_P, _P, _P, _P]),
    ("perf_destroy_scene", _I32, [_P]),
    ("perf_last_error", ctypes.c_char_p, []),
    ("perf_render_residuals", _I32, [_P, _P, _P, _P]),
    ("perf_apply_J", _I32, [_P, _P, _P, _P]),
    ("perf_apply_Jt", _I32, [_P, _P, _P, _P]),
    ("perf_apply_JtJ", _I32, [_P, _P, _P, _P]),
    ("perf_build_precond", _I32, [_P, _P, _I32, _P, _P, _P, _P]),
    ("perf_gn_step", _I32, [_P, _P, _P, _P]),
    ("perf_objective", _I32, [_P, _P, _P, ctypes.c_float, _P]),
    ("perf_footprint", _I32, [_P, _P, _P]),
    ("perf_upsample", _I32, [_P, _P, _P, _P, _P]),
    ("perf_set_jitter", _I32, [_P, ctypes.c_uint32]),
    ("perf_invert_blocks", _I32, [_P, _I64, _I32, _P, _P]),
    ("perf_pack_bf16", _I32, [_P, _P, _I64, _P]),
    ("perf_precond_features", _I32, [_P, _P, _P, _P]),
    ("perf_mlp_set_weights", _I32, [_P, _P, _I32, _P, ctypes.c_float]),
    ("perf_mlp_infer", _I32, [_P, _P, _P, _P]),
    ("perf_mlp_train_step", _I32, [_P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float, _P, _P, _P, _I32, _P, _P,
                                   _P]),
    ("perf_mlp_train_step_noalloc", _I32, [_P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float, _P, _P, _P, _I32,
                                           _P, _P]),
    ("perf_mlp_feature_stats", _I32, [_P, _I64, _P, _P]),
    ("perf_mlp_training_rows", _I32, [_P, _P, _P, ctypes.c_uint32, ctypes.c_float, _P, _P, _I64,
                                      ctypes.POINTER(_I64)]),
]

_lib = None


class PerfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def load():
    """Load libperf_gn.so; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2112_05598_amd.build_lib.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int):
    if rc != PERF_OK:
        msg = load().perf_last_error()
        raise PerfError(rc, msg.decode() if msg else "error")
    return rc


def __getattr__(name):
    # perf_* names resolve to the library's functions
    if name.startswith("perf_"):
        return getattr(load(), name)
    raise AttributeError(name)
