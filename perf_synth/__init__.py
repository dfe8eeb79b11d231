"""Seeded synthetic inputs for the PERF Gauss-Newton path.

This package only *generates inputs*: ground-truth voxel grids rasterised from
primitives, smooth environment-layer textures, camera poses and intrinsics,
initial guesses and random vectors.  It holds none of the method's arithmetic
(no ray generation, no sampling, no compositing, no derivatives), so both the
FP64 oracle and the HIP path can consume it without sharing any of the method.
"""
from .scenes import (  # noqa: F401
    SceneSpec,
    Cameras,
    Workload,
    make_cameras,
    cameras_from_origins,
    rasterize_primitives,
    random_primitives,
    smooth_env_layers,
    pack_params,
    unpack_params,
    init_params,
    random_vector,
    workload,
    WORKLOADS,
    crop_workload,
    n_params,
    n_units,
)
