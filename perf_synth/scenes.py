"""Seeded scene, camera and vector generators.

Parameter layout (shared convention of every consumer):
  voxels  : x[((z*ny + y)*nx + xi)*4 + {r,g,b,sigma}]
  texels  : after the voxels, x[Nvox*4 + ((l*He + j)*We + i)*4 + {r,g,b,alpha}]
Cameras : origin (n,3); rot (n,3,3) camera-to-world with columns
          (right, down, forward); fx, fy, cx, cy per camera; one shared
          image size width x height.

Everything here is input generation.  Workload shapes follow the configs the
method is evaluated on (an object in a box seen from a hemisphere, a 360-degree
ring of cameras); the paper's datasets are not available, so these seeded
synthetic scenes stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def _f32(v):
    """The nearest single-precision values, kept as float64: the library reads scene and camera
    parameters in single precision, so the generators hand every consumer exactly those values."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass
class SceneSpec:
    nx: int
    ny: int
    nz: int
    bbox_min: Tuple[float, float, float] = (-1.0, -1.0, -1.0)
    bbox_max: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    layer_radii: Tuple[float, ...] = (1.8,)
    env_w: int = 64
    env_h: int = 32
    step_vox: float = 0.5
    background: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def __post_init__(self):
        self.bbox_min = tuple(float(v) for v in _f32(self.bbox_min))
        self.bbox_max = tuple(float(v) for v in _f32(self.bbox_max))
        self.layer_radii = tuple(float(v) for v in _f32(self.layer_radii))
        self.step_vox = float(_f32(self.step_vox))
        self.background = tuple(float(v) for v in _f32(self.background))

    @property
    def n_layers(self) -> int:
        return len(self.layer_radii)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_texels(self) -> int:
        return self.n_layers * self.env_w * self.env_h

    @property
    def n_units(self) -> int:
        return self.n_vox + self.n_texels

    @property
    def n_params(self) -> int:
        return 4 * self.n_units


def n_units(spec: SceneSpec) -> int:
    return spec.n_units


def n_params(spec: SceneSpec) -> int:
    return spec.n_params


@dataclasses.dataclass
class Cameras:
    origin: np.ndarray  # (n,3) float64
    rot: np.ndarray     # (n,3,3) float64, columns right/down/forward
    fx: np.ndarray
    fy: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    width: int
    height: int

    def __post_init__(self):
        self.origin = _f32(self.origin)
        self.rot = _f32(self.rot)
        self.fx, self.fy, self.cx, self.cy = _f32(self.fx), _f32(self.fy), _f32(self.cx), _f32(self.cy)

    @property
    def n(self) -> int:
        return int(self.origin.shape[0])

    @property
    def n_rays(self) -> int:
        return self.n * self.width * self.height

    def subset(self, idx: Sequence[int]) -> "Cameras":
        idx = np.asarray(idx, dtype=np.int64)
        return Cameras(self.origin[idx].copy(), self.rot[idx].copy(), self.fx[idx].copy(),
                       self.fy[idx].copy(), self.cx[idx].copy(), self.cy[idx].copy(),
                       self.width, self.height)

    def with_image(self, width: int, height: int, fov_deg: float) -> "Cameras":
        """Same poses, new image size and horizontal field of view."""
        f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
        n = self.n
        return Cameras(self.origin.copy(), self.rot.copy(), np.full(n, f), np.full(n, f),
                       np.full(n, width / 2.0), np.full(n, height / 2.0), width, height)


def _look_at_origin(origin: np.ndarray) -> np.ndarray:
    fwd = -origin / np.linalg.norm(origin)
    up = np.array([0.0, 0.0, 1.0])
    if np.linalg.norm(np.cross(fwd, up)) < 1e-3:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    down /= np.linalg.norm(down)
    return np.stack([right, down, fwd], axis=1)  # columns


def cameras_from_origins(origins, width: int, height: int, fov_deg: float) -> Cameras:
    """Pinhole cameras at the given positions, each looking at the origin."""
    origins = np.asarray(origins, dtype=np.float64).reshape(-1, 3)
    rot = np.stack([_look_at_origin(o) for o in origins], axis=0)
    n = origins.shape[0]
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Cameras(origins.copy(), rot, np.full(n, f), np.full(n, f), np.full(n, width / 2.0),
                   np.full(n, height / 2.0), width, height)


def make_cameras(kind: str, n: int, width: int, height: int, fov_deg: float,
                 radius, rng: np.random.Generator, z_range=(-0.5, 0.5)) -> Cameras:
    """Pinhole cameras looking at the origin.

    kind: 'sphere'      uniform directions on the sphere, fixed radius
          'hemisphere'  uniform directions with z >= 0, fixed radius
          'ring'        azimuth evenly spaced (+ jitter), radius U(r0, r1), z in z_range
    fov_deg is the horizontal field of view; pixels are square.
    """
    origins = np.zeros((n, 3))
    if kind in ("sphere", "hemisphere"):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        if kind == "hemisphere":
            v[:, 2] = np.abs(v[:, 2])
        origins = v * float(radius)
    elif kind == "ring":
        r0, r1 = radius
        phi = 2.0 * np.pi * (np.arange(n) + rng.uniform(-0.5, 0.5, size=n)) / n
        r = rng.uniform(r0, r1, size=n)
        z = rng.uniform(z_range[0], z_range[1], size=n)
        origins = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    else:
        raise ValueError(kind)
    rot = np.stack([_look_at_origin(o) for o in origins], axis=0)
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Cameras(origins, rot, np.full(n, f), np.full(n, f), np.full(n, width / 2.0),
                   np.full(n, height / 2.0), width, height)


# ----------------------------------------------------------------------------- ground truth

@dataclasses.dataclass
class Primitive:
    kind: str            # 'sphere' | 'box'
    centre: np.ndarray   # (3,)
    size: np.ndarray     # radius (1,) or half extents (3,)
    rgb: np.ndarray      # (3,)
    sigma: float


def random_primitives(rng: np.random.Generator, n: int, kinds="mixed",
                      r_range=(0.05, 0.25), centre_range=0.7, sigma_range=(0.5, 1.0)) -> List[Primitive]:
    prims = []
    for _ in range(n):
        if kinds == "spheres":
            kind = "sphere"
        else:
            kind = "sphere" if rng.uniform() < 0.5 else "box"
        centre = rng.uniform(-centre_range, centre_range, size=3)
        if kind == "sphere":
            size = np.array([rng.uniform(*r_range)])
        else:
            size = rng.uniform(*r_range, size=3)
        rgb = rng.uniform(0.0, 1.0, size=3)
        sigma = float(rng.uniform(*sigma_range)) if sigma_range[0] != sigma_range[1] else float(sigma_range[0])
        prims.append(Primitive(kind, centre, size, rgb, sigma))
    return prims


def rasterize_primitives(spec: SceneSpec, prims: Sequence[Primitive]) -> np.ndarray:
    """Voxel grid (nz, ny, nx, 4) float32 sampled at voxel centres; later primitives overwrite."""
    grid = np.zeros((spec.nz, spec.ny, spec.nx, 4), dtype=np.float32)
    bmin = np.asarray(spec.bbox_min, dtype=np.float64)
    bmax = np.asarray(spec.bbox_max, dtype=np.float64)
    dims = np.array([spec.nx, spec.ny, spec.nz])
    h = (bmax - bmin) / dims
    for p in prims:
        ext = p.size if p.kind == "box" else np.repeat(p.size, 3)
        lo = np.floor((p.centre - ext - bmin) / h - 0.5).astype(np.int64)
        hi = np.ceil((p.centre + ext - bmin) / h - 0.5).astype(np.int64) + 1
        lo = np.clip(lo, 0, dims)
        hi = np.clip(hi, 0, dims)
        if np.any(hi <= lo):
            continue
        xs = bmin[0] + (np.arange(lo[0], hi[0]) + 0.5) * h[0]
        ys = bmin[1] + (np.arange(lo[1], hi[1]) + 0.5) * h[1]
        zs = bmin[2] + (np.arange(lo[2], hi[2]) + 0.5) * h[2]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        dx, dy, dz = X - p.centre[0], Y - p.centre[1], Z - p.centre[2]
        if p.kind == "sphere":
            m = dx * dx + dy * dy + dz * dz <= p.size[0] ** 2
        else:
            m = (np.abs(dx) <= p.size[0]) & (np.abs(dy) <= p.size[1]) & (np.abs(dz) <= p.size[2])
        sub = grid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[m, 0:3] = p.rgb.astype(np.float32)
        sub[m, 3] = np.float32(p.sigma)
    return grid


def _texel_dirs(w: int, h: int) -> np.ndarray:
    """Unit directions at equirectangular texel centres, (h, w, 3)."""
    phi = ((np.arange(w) + 0.5) / w - 0.5) * 2.0 * np.pi
    theta = (np.arange(h) + 0.5) / h * np.pi
    T, P = np.meshgrid(theta, phi, indexing="ij")
    return np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1)


def _smooth_field(rng: np.random.Generator, dirs: np.ndarray, n_terms=6, freq=1.5) -> np.ndarray:
    k = rng.normal(scale=freq, size=(n_terms, 3))
    a = rng.uniform(-1.0, 1.0, size=n_terms)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_terms)
    b = rng.uniform(-0.5, 0.5)
    out = np.full(dirs.shape[:-1], b)
    for i in range(n_terms):
        out = out + a[i] * np.sin(dirs @ k[i] + ph[i])
    return out


def _sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def smooth_env_layers(spec: SceneSpec, rng: np.random.Generator, alphas: Sequence) -> np.ndarray:
    """(L, He, We, 4) float32. alphas[l] is a constant opacity or 'blobs' (smooth partial opacity)."""
    dirs = _texel_dirs(spec.env_w, spec.env_h)
    env = np.zeros((spec.n_layers, spec.env_h, spec.env_w, 4), dtype=np.float32)
    for l in range(spec.n_layers):
        for ch in range(3):
            env[l, :, :, ch] = _sigmoid(_smooth_field(rng, dirs)).astype(np.float32)
        a = alphas[l]
        if isinstance(a, str):
            env[l, :, :, 3] = (0.8 * _sigmoid(4.0 * _smooth_field(rng, dirs) - 2.0)).astype(np.float32)
        else:
            env[l, :, :, 3] = np.float32(a)
    return env


def pack_params(grid: np.ndarray, env: np.ndarray) -> np.ndarray:
    return np.concatenate([grid.reshape(-1), env.reshape(-1)]).astype(np.float32)


def unpack_params(spec: SceneSpec, x: np.ndarray):
    nv = spec.n_vox * 4
    grid = x[:nv].reshape(spec.nz, spec.ny, spec.nx, 4)
    env = x[nv:].reshape(spec.n_layers, spec.env_h, spec.env_w, 4)
    return grid, env


def init_params(spec: SceneSpec, colour=0.5, sigma=0.01, alpha=0.01) -> np.ndarray:
    grid = np.empty((spec.nz, spec.ny, spec.nx, 4), dtype=np.float32)
    grid[..., 0:3] = colour
    grid[..., 3] = sigma
    env = np.empty((spec.n_layers, spec.env_h, spec.env_w, 4), dtype=np.float32)
    env[..., 0:3] = colour
    env[..., 3] = alpha
    return pack_params(grid, env)


def random_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return (np.random.default_rng(seed).normal(size=n) * scale).astype(np.float32)


# ----------------------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    spec: SceneSpec
    cams: Cameras
    x_gt: np.ndarray
    x_init: np.ndarray
    seed: int


def _scene(name, spec, cams, grid, env, seed) -> Workload:
    return Workload(name, spec, cams, pack_params(grid, env), init_params(spec), seed)


def _primitive_scene(spec: SceneSpec, rng, n_prims, layer_alphas) -> Tuple[np.ndarray, np.ndarray]:
    prims = random_primitives(rng, n_prims)
    grid = rasterize_primitives(spec, prims)
    env = smooth_env_layers(spec, rng, layer_alphas)
    return grid, env


def workload(name: str, seed: Optional[int] = None, grid_n: Optional[int] = None) -> Workload:
    """Named synthetic workloads.

    tiny / small / ragged : parity cases (several tiles and a ragged image tail)
    cfg1 : 32^3, 1 layer 64x32 @1.8, 8 cams 64x64 FOV40 on a sphere r=3, 3 spheres sigma 0.9
    cfg2 : 128^3, 3 layers 256x128 @1.8/3/6, 100 cams 400x400 on the upper hemisphere r=4,
           40 spheres/boxes, RGB U(0,1), opacity U(0.5,1)
    cfg3 : cfg2 kind at 256^3, 3 layers 512x256, 200 cams 800x800
    cfg5 : 256^3, 4 layers 1024x512 @1.8/3/6/12, 150 cams 1008x756 on a ring r U(2.5,4)

    grid_n re-rasterises the same primitives (same seed, same env and cameras) at another
    cubic resolution, e.g. the 16^3 copy of cfg5 used for finite differences.
    """
    if name == "tiny":
        s = 11 if seed is None else seed
        rng = np.random.default_rng(s)
        spec = SceneSpec(8, 8, 8, layer_radii=(1.8,), env_w=16, env_h=8)
        cams = make_cameras("sphere", 2, 13, 11, 40.0, 3.0, rng)
        grid = rasterize_primitives(spec, random_primitives(rng, 2, kinds="spheres", r_range=(0.3, 0.6),
                                                            centre_range=0.4, sigma_range=(0.9, 0.9)))
        env = smooth_env_layers(spec, rng, [1.0])
        return _scene(name, spec, cams, grid, env, s)
    if name == "small":
        s = 12 if seed is None else seed
        rng = np.random.default_rng(s)
        spec = SceneSpec(16, 12, 10, bbox_min=(-1.0, -0.75, -0.625), bbox_max=(1.0, 0.75, 0.625),
                         layer_radii=(1.8, 3.0), env_w=32, env_h=16)
        cams = make_cameras("sphere", 3, 37, 29, 40.0, 3.5, rng)
        grid, env = _primitive_scene(spec, rng, 6, [0.4, 1.0])
        return _scene(name, spec, cams, grid, env, s)
    if name == "ragged":
        s = 13 if seed is None else seed
        rng = np.random.default_rng(s)
        spec = SceneSpec(24, 24, 24, layer_radii=(1.8, 3.0, 6.0), env_w=48, env_h=24)
        cams = make_cameras("hemisphere", 3, 45, 38, 40.0, 4.0, rng)
        grid, env = _primitive_scene(spec, rng, 10, [0.0, "blobs", 1.0])
        return _scene(name, spec, cams, grid, env, s)
    if name == "cfg1":
        s = 1 if seed is None else seed
        rng = np.random.default_rng(s)
        n = 32 if grid_n is None else grid_n
        spec = SceneSpec(n, n, n, layer_radii=(1.8,), env_w=64, env_h=32)
        prims = random_primitives(rng, 3, kinds="spheres", r_range=(0.15, 0.4), centre_range=0.5,
                                  sigma_range=(0.9, 0.9))
        grid = rasterize_primitives(spec, prims)
        env = smooth_env_layers(spec, rng, [1.0])
        cams = make_cameras("sphere", 8, 64, 64, 40.0, 3.0, rng)
        return _scene(name, spec, cams, grid, env, s)
    if name in ("cfg2", "cfg4"):
        s = 2 if seed is None else seed
        rng = np.random.default_rng(s)
        n = 128 if grid_n is None else grid_n
        spec = SceneSpec(n, n, n, layer_radii=(1.8, 3.0, 6.0), env_w=256, env_h=128)
        grid, env = _primitive_scene(spec, rng, 40, [0.0, 0.0, 1.0])
        cams = make_cameras("hemisphere", 100, 400, 400, 40.0, 4.0, rng)
        return _scene(name, spec, cams, grid, env, s)
    if name == "cfg3":
        s = 3 if seed is None else seed
        rng = np.random.default_rng(s)
        n = 256 if grid_n is None else grid_n
        spec = SceneSpec(n, n, n, layer_radii=(1.8, 3.0, 6.0), env_w=512, env_h=256)
        grid, env = _primitive_scene(spec, rng, 40, [0.0, 0.0, 1.0])
        cams = make_cameras("hemisphere", 200, 800, 800, 40.0, 4.0, rng)
        return _scene(name, spec, cams, grid, env, s)
    if name == "cfg5":
        s = 5 if seed is None else seed
        rng = np.random.default_rng(s)
        n = 256 if grid_n is None else grid_n
        spec = SceneSpec(n, n, n, layer_radii=(1.8, 3.0, 6.0, 12.0), env_w=1024, env_h=512)
        grid, env = _primitive_scene(spec, rng, 40, ["blobs", "blobs", "blobs", 1.0])
        cams = make_cameras("ring", 150, 1008, 756, 60.0, (2.5, 4.0), rng)
        return _scene(name, spec, cams, grid, env, s)
    raise KeyError(name)


WORKLOADS = ("tiny", "small", "ragged", "cfg1", "cfg2", "cfg3", "cfg5")


def crop_workload(full: Workload, lo: int, size: int, n_cams: int, width: int, height: int,
                  fov_deg: float, name: str) -> Workload:
    """A standalone sub-grid voxels [lo, lo+size)^3 of `full` with the same voxel size and env layers.

    Used for the 64^3 crop of the 256^3 workload and the 16^3 copy for finite differences.
    """
    spec = full.spec
    h = (np.asarray(spec.bbox_max) - np.asarray(spec.bbox_min)) / np.array([spec.nx, spec.ny, spec.nz])
    bmin = np.asarray(spec.bbox_min) + lo * h
    bmax = bmin + size * h
    cspec = dataclasses.replace(spec, nx=size, ny=size, nz=size, bbox_min=tuple(bmin), bbox_max=tuple(bmax))
    g_full, env = unpack_params(spec, full.x_gt)
    grid = g_full[lo:lo + size, lo:lo + size, lo:lo + size].copy()
    cams = full.cams.subset(range(min(n_cams, full.cams.n))).with_image(width, height, fov_deg)
    return Workload(name, cspec, cams, pack_params(grid, env), init_params(cspec), full.seed)
