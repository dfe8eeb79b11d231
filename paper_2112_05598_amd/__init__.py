"""MI355X-native matrix-free Gauss-Newton / PCG for explicit radiance fields.

The computation lives in libperf_gn.so (hand-written HIP for gfx950) behind the
C ABI of include/perf_gn.h; this package only marshals arguments.
"""
from . import abi  # noqa: F401


def __getattr__(name):
    if name == "Scene":
        from .scene import Scene
        return Scene
    if name == "RenderResiduals":
        from .autograd import RenderResiduals
        return RenderResiduals
    raise AttributeError(name)
