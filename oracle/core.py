"""FP64 oracle: ctypes binding of perf_oracle.c plus the solver layer in numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Callable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perf_oracle.c")
_LIB = os.path.join(_HERE, "_perf_oracle.so")
MAX_LAYERS = 8


def library_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile perf_oracle.c with gcc (IEEE double, OpenMP over rays)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bmin", ctypes.c_double * 3), ("bmax", ctypes.c_double * 3),
        ("n_layers", ctypes.c_int32), ("env_w", ctypes.c_int32), ("env_h", ctypes.c_int32),
        ("radius", ctypes.c_double * MAX_LAYERS),
        ("step", ctypes.c_double),
        ("bg", ctypes.c_double * 3),
        ("n_cams", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("cam_origin", ctypes.c_void_p), ("cam_rot", ctypes.c_void_p), ("cam_intr", ctypes.c_void_p),
        ("aux_lambda", ctypes.c_double),
        ("jitter_seed", ctypes.c_uint32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.orc_n_units.restype = i64
        lib.orc_n_units.argtypes = [P]
        lib.orc_n_rays.restype = i64
        lib.orc_n_rays.argtypes = [P]
        lib.orc_entry_capacity.restype = i64
        lib.orc_entry_capacity.argtypes = [P]
        lib.orc_render.argtypes = [P, P, P, P, i64, P, P, P, P, P]
        lib.orc_apply_J.argtypes = [P, P, P, P, i64, P]
        lib.orc_apply_Jt.argtypes = [P, P, P, P, i64, P]
        lib.orc_apply_JtJ.argtypes = [P, P, P, P, i64, P]
        lib.orc_grad_blocks.argtypes = [P, P, P, P, i64, P, P, P]
        lib.orc_footprint.argtypes = [P, P, i64, P, P, P]
        lib.orc_ray_row.restype = i64
        lib.orc_ray_row.argtypes = [P, P, i64, ctypes.c_int, i64, P, P, P, P]
        lib.orc_ray_samples.restype = i64
        lib.orc_ray_samples.argtypes = [P, P, i64, ctypes.c_int, i64, P, P, P, P, P, P, P, P, P]
        lib.orc_sample_field.restype = ctypes.c_double
        lib.orc_sample_field.argtypes = [P, P, P, ctypes.c_int]
        lib.orc_ray.argtypes = [P, i64, P, P]
        lib.orc_render_image.argtypes = [P, P, ctypes.c_double, P, P, i64, P, P, P]
        lib.orc_jitter_u.restype = ctypes.c_double
        lib.orc_jitter_u.argtypes = [ctypes.c_uint32, i64, ctypes.c_uint32]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleScene:
    """A scene description (grid, environment layers, cameras) for the oracle.

    aux_lambda > 0 adds the auxiliary opacity residual of Sec. III-I (Eq. 10) as a fourth
    residual per ray: residual and J v arrays then have 4 columns, and J^T u takes 4.
    jitter_seed != 0 jitters ray origins within pixels and samples within steps (Sec. IV)."""

    def __init__(self, spec, cams, aux_lambda: float = 0.0, jitter_seed: int = 0):
        self.lib = _load()
        self.spec = spec
        self.cams = cams
        if spec.n_layers > MAX_LAYERS:
            raise ValueError("too many layers")
        self._origin = _f64(cams.origin).reshape(-1, 3).copy()
        self._rot = _f64(cams.rot).reshape(-1, 9).copy()
        self._intr = _f64(np.stack([cams.fx, cams.fy, cams.cx, cams.cy], axis=1)).copy()
        s = _Scene()
        s.nx, s.ny, s.nz = spec.nx, spec.ny, spec.nz
        for i in range(3):
            s.bmin[i] = spec.bbox_min[i]
            s.bmax[i] = spec.bbox_max[i]
            s.bg[i] = spec.background[i]
        s.n_layers, s.env_w, s.env_h = spec.n_layers, spec.env_w, spec.env_h
        for i, r in enumerate(spec.layer_radii):
            s.radius[i] = r
        s.step = spec.step_vox
        s.n_cams, s.width, s.height = cams.n, cams.width, cams.height
        s.cam_origin = self._origin.ctypes.data
        s.cam_rot = self._rot.ctypes.data
        s.cam_intr = self._intr.ctypes.data
        s.aux_lambda = float(aux_lambda)
        s.jitter_seed = int(jitter_seed) & 0xFFFFFFFF
        self.aux_lambda = float(aux_lambda)
        self.n_res = 4 if aux_lambda > 0 else 3
        self._s = s
        self.p = ctypes.addressof(s)
        self.n_units = int(self.lib.orc_n_units(self.p))
        self.n_params = 4 * self.n_units
        self.n_rays = int(self.lib.orc_n_rays(self.p))
        self.n_vox = spec.n_vox

    def set_jitter(self, seed: int):
        """Jitter seed for every later call (0 = off)."""
        self._s.jitter_seed = int(seed) & 0xFFFFFFFF

    def jitter_u(self, seed: int, ray: int, stream: int) -> float:
        return float(self.lib.orc_jitter_u(int(seed) & 0xFFFFFFFF, int(ray), int(stream)))

    # ---------------------------------------------------------------- helpers
    def _rays(self, rays):
        if rays is None:
            return None, self.n_rays
        r = np.ascontiguousarray(rays, dtype=np.int64)
        if r.size and (r.min() < 0 or r.max() >= self.n_rays):
            raise IndexError("ray id out of range")
        return r, int(r.size)

    def ray(self, ray_id: int):
        o = np.zeros(3)
        d = np.zeros(3)
        self.lib.orc_ray(self.p, int(ray_id), o.ctypes.data, d.ctypes.data)
        return o, d

    # ---------------------------------------------------------------- operators
    def render(self, x, targets=None, rays=None):
        """Eq. 3 per ray: returns (H [n,3], r [n,n_res] or None, F, T_exit [n]); with the
        auxiliary residual on, r[:, 3] is r_4 and F includes it."""
        x = _f64(x)
        r_ids, n = self._rays(rays)
        H = np.zeros((n, 3))
        Te = np.zeros(n)
        aux = np.zeros(n)
        r = np.zeros((n, 3)) if targets is not None else None
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.float32).reshape(-1)
        F = ctypes.c_double(0.0)
        self.lib.orc_render(self.p, _ptr(x), _ptr(t), _ptr(r_ids), n, _ptr(H), _ptr(r), ctypes.addressof(F),
                            _ptr(Te), _ptr(aux))
        if r is not None and self.n_res == 4:
            r = np.concatenate([r, aux[:, None]], axis=1)
        return H, r, F.value, Te

    def render_image(self, x, threshold=0.0, targets=None, rays=None):
        """Rendering of Sec. IV: (H [n,3] with the opacity-threshold rule, T_exit [n], mean
        squared colour error against targets or None)."""
        x = _f64(x)
        r_ids, n = self._rays(rays)
        H = np.zeros((n, 3))
        Te = np.zeros(n)
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.float32).reshape(-1)
        mse = ctypes.c_double(0.0)
        self.lib.orc_render_image(self.p, _ptr(x), float(threshold), _ptr(t), _ptr(r_ids), n, _ptr(H), _ptr(Te),
                                  ctypes.addressof(mse))
        return H, Te, (mse.value if targets is not None else None)

    def apply_J(self, x, v, rays=None):
        x, v = _f64(x), _f64(v)
        r_ids, n = self._rays(rays)
        u = np.zeros((n, self.n_res))
        self.lib.orc_apply_J(self.p, _ptr(x), _ptr(v), _ptr(r_ids), n, _ptr(u))
        return u

    def apply_Jt(self, x, u, rays=None):
        x, u = _f64(x), _f64(u).reshape(-1)
        r_ids, n = self._rays(rays)
        if u.size != self.n_res * n:
            raise ValueError(f"u must have {self.n_res} entries per ray")
        y = np.zeros(self.n_params)
        self.lib.orc_apply_Jt(self.p, _ptr(x), _ptr(u), _ptr(r_ids), n, _ptr(y))
        return y

    def apply_JtJ(self, x, v, rays=None):
        x, v = _f64(x), _f64(v)
        r_ids, n = self._rays(rays)
        y = np.zeros(self.n_params)
        self.lib.orc_apply_JtJ(self.p, _ptr(x), _ptr(v), _ptr(r_ids), n, _ptr(y))
        return y

    def grad_blocks(self, x, targets, rays=None):
        """(grad = -J^T r [P], blocks [units,5] = (d, e_r, e_g, e_b, f), F)."""
        x = _f64(x)
        t = np.ascontiguousarray(targets, dtype=np.float32).reshape(-1)
        r_ids, n = self._rays(rays)
        g = np.zeros(self.n_params)
        b = np.zeros((self.n_units, 5))
        F = ctypes.c_double(0.0)
        self.lib.orc_grad_blocks(self.p, _ptr(x), _ptr(t), _ptr(r_ids), n, _ptr(g), _ptr(b), ctypes.addressof(F))
        return g, b, F.value

    def footprint(self, rays=None):
        """(U unique voxels per ray, layers hit per ray, samples per ray)."""
        r_ids, n = self._rays(rays)
        U = np.zeros(n, dtype=np.int64)
        L = np.zeros(n, dtype=np.int32)
        K = np.zeros(n, dtype=np.int64)
        self.lib.orc_footprint(self.p, _ptr(r_ids), n, _ptr(U), _ptr(L), _ptr(K))
        return U, L, K

    def ray_row(self, x, ray_id, mode=0):
        x = _f64(x)
        cap = int(self.lib.orc_entry_capacity(self.p))
        unit = np.zeros(cap, dtype=np.int64)
        a = np.zeros(cap)
        s = np.zeros((cap, 3))
        H = np.zeros(3)
        m = int(self.lib.orc_ray_row(self.p, _ptr(x), int(ray_id), int(mode), cap, _ptr(unit), _ptr(a), _ptr(s),
                                     _ptr(H)))
        return unit[:m].copy(), a[:m].copy(), s[:m].copy(), H

    def ray_samples(self, x, ray_id, mode=0):
        x = _f64(x)
        cap = int(self.lib.orc_entry_capacity(self.p))
        arrs = {k: np.zeros(cap) for k in ("delta", "sigma", "T", "alpha", "dHdc")}
        c = np.zeros((cap, 3))
        dHds = np.zeros((cap, 3))
        H = np.zeros(3)
        Tend = np.zeros(1)
        K = int(self.lib.orc_ray_samples(self.p, _ptr(x), int(ray_id), int(mode), cap, _ptr(arrs["delta"]),
                                         _ptr(arrs["sigma"]), _ptr(arrs["T"]), _ptr(arrs["alpha"]), _ptr(c),
                                         _ptr(arrs["dHdc"]), _ptr(dHds), _ptr(H), _ptr(Tend)))
        out = {k: v[:K].copy() for k, v in arrs.items()}
        out["c"] = c[:K].copy()
        out["dHds"] = dHds[:K].copy()
        out["H"] = H
        out["T_end"] = float(Tend[0])
        return out

    def sample_field(self, x, p, ch):
        x = _f64(x)
        p = _f64(p)
        return float(self.lib.orc_sample_field(self.p, _ptr(x), _ptr(p), int(ch)))

    def num_threads(self) -> int:
        return int(self.lib.orc_num_threads())


# ------------------------------------------------------------------ preconditioners (Sec. III-G)

def psnr(mse: float, peak: float = 1.0) -> float:
    """Peak signal-to-noise ratio in dB of a mean squared error, colours in [0, peak]."""
    return float(10.0 * np.log10(peak * peak / mse)) if mse > 0 else float("inf")


def jacobi_diag(blocks: np.ndarray) -> np.ndarray:
    """diag(J^T J) per parameter from the (d, e, f) blocks: (d, d, d, f) per unit."""
    b = np.asarray(blocks, dtype=np.float64)
    return np.stack([b[:, 0], b[:, 0], b[:, 0], b[:, 4]], axis=1).reshape(-1)


def jacobi_inverse(blocks: np.ndarray) -> np.ndarray:
    """M^{-1} = 1/diag(J^T J) per parameter (Sec. III-G), 0 where the diagonal is 0."""
    d = jacobi_diag(blocks)
    out = np.zeros_like(d)
    nz = d > 0
    out[nz] = 1.0 / d[nz]
    return out


def block_matrix(blocks: np.ndarray) -> np.ndarray:
    """[units,4,4] matrices [[d I, e], [e^T, f]]."""
    b = np.asarray(blocks, dtype=np.float64)
    n = b.shape[0]
    B = np.zeros((n, 4, 4))
    for i in range(3):
        B[:, i, i] = b[:, 0]
        B[:, i, 3] = b[:, 1 + i]
        B[:, 3, i] = b[:, 1 + i]
    B[:, 3, 3] = b[:, 4]
    return B


RIDGE = 1e-6


def block_inverse(blocks: np.ndarray, ridge: float = RIDGE) -> np.ndarray:
    """Inverse of each 4x4 block after adding ridge*max(d, f) to the diagonal; 0 for empty units
    (no ray: max(d, f) = 0; or a non-finite block).

    Returned as [units,4,4] (the plain matrix inverse, numpy.linalg.inv).
    """
    b = np.asarray(blocks, dtype=np.float64)
    B = block_matrix(b)
    m = np.maximum(b[:, 0], b[:, 4])
    live = (m > 0) & np.all(np.isfinite(b), axis=1)  # a non-finite block counts as an empty unit
    out = np.zeros_like(B)
    if np.any(live):
        Bl = B[live] + (ridge * m[live])[:, None, None] * np.eye(4)[None]
        out[live] = np.linalg.inv(Bl)
    return out


def apply_block_inverse(Binv: np.ndarray, r: np.ndarray) -> np.ndarray:
    return np.einsum("nij,nj->ni", Binv, np.asarray(r, dtype=np.float64).reshape(-1, 4)).reshape(-1)


def apply_precond(kind: str, data, r: np.ndarray) -> np.ndarray:
    if kind == "none":
        return np.array(r, dtype=np.float64)
    if kind == "jacobi":
        return data * r
    if kind in ("block", "learned"):
        return apply_block_inverse(data, r)
    raise ValueError(kind)


# ------------------------------------------------------------------ Alg. 2

@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    alpha: list
    beta: list
    R: list
    pAp: list
    R0: float
    flags: set


def pcg(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, apply_Minv: Callable[[np.ndarray], np.ndarray],
        max_iters: int = 20, rel_tol: float = 0.0, abs_eps: float = 0.0, stall_ratio: float = 0.0) -> PCGResult:
    """Preconditioned conjugate gradient as in Alg. 2, started at x0 = 0.

    Stops after max_iters products with A, when R = r^T r < abs_eps, when
    sqrt(R / R0) <= rel_tol, or when R / R_prev > stall_ratio (the early exit of
    Alg. 2; the paper uses 0.85; <= 0 disables it).  A non-positive or
    non-finite p^T A p stops the iteration before the update ('breakdown').
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    R0 = float(r @ r)
    R_prev = R0
    z = apply_Minv(r)
    p = z.copy()
    rz = float(r @ z)
    res = PCGResult(x, 0, [], [], [], [], R0, set())
    if max_iters <= 0:
        return res
    if R0 == 0.0:
        res.flags.add("converged")
        return res
    k = 0
    while True:
        Ap = apply_A(p)
        pAp = float(p @ Ap)
        res.pAp.append(pAp)
        if not (pAp > 0.0) or not math.isfinite(pAp):
            res.flags.add("breakdown")
            break
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        R = float(r @ r)
        res.alpha.append(alpha)
        res.R.append(R)
        k += 1
        if abs_eps > 0 and R < abs_eps:
            res.flags.add("converged")
            break
        if rel_tol > 0 and math.sqrt(R / R0) <= rel_tol:
            res.flags.add("converged")
            break
        if stall_ratio > 0 and R / R_prev > stall_ratio:
            res.flags.add("stall")
            break
        if k >= max_iters:
            break
        R_prev = R
        z = apply_Minv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        res.beta.append(beta)
        rz = rz_new
        p = z + beta * p
    res.x = x
    res.iters = k
    return res


# ------------------------------------------------------------------ Alg. 3

def line_search(objective: Callable[[float], float], F0: float, factor: float = 0.7, ls_max: int = 20):
    """Backtracking of Alg. 3 with a trial cap.

    gamma starts at 1 and shrinks by `factor` while the error keeps falling; at
    the first strict increase the previous gamma is returned.  With the cap hit,
    or when no trial beats F0, the trial with the smallest error is returned if
    it beats F0, else gamma = 0.  Returns (gamma, mu, n_trials, capped).
    """
    gamma = 1.0
    mu_prev = math.inf
    best_mu, best_gamma = math.inf, 0.0
    n = 0
    while n < ls_max:
        mu = float(objective(gamma))
        n += 1
        if mu < best_mu:
            best_mu, best_gamma = mu, gamma
        if mu > mu_prev:
            g = gamma / factor
            if mu_prev < F0:
                return g, mu_prev, n, False
            return 0.0, F0, n, False
        gamma = factor * gamma
        mu_prev = mu
    if best_mu < F0:
        return best_gamma, best_mu, n, True
    return 0.0, F0, n, True


def project(spec, x: np.ndarray) -> np.ndarray:
    """sigma >= 0 on voxels, alpha in [0, 1] on texels; colours unconstrained."""
    y = np.array(x, dtype=np.float64).reshape(-1, 4)
    nv = spec.n_vox
    y[:nv, 3] = np.maximum(y[:nv, 3], 0.0)
    y[nv:, 3] = np.clip(y[nv:, 3], 0.0, 1.0)
    return y.reshape(-1)


# ------------------------------------------------------------------ hierarchy (Sec. IV, hierarchical formulation)

def _shortest_side(spec) -> float:
    return min((spec.bbox_max[a] - spec.bbox_min[a]) / n for a, n in enumerate((spec.nx, spec.ny, spec.nz)))


def _lerp_axis(n_src: int, n_dst: int, periodic: bool):
    """For every destination cell centre along one axis: the two source indices and the weight
    of the upper one, cell-centred coordinates (source coordinate g = (j + 0.5) n_src / n_dst
    - 0.5); clamped to [0, n_src - 1] (lower index at most n_src - 2), or wrapped if periodic."""
    j = np.arange(n_dst, dtype=np.float64)
    g = (j + 0.5) * n_src / n_dst - 0.5
    if periodic:
        i0 = np.floor(g)
        f = g - i0
        i0 = i0.astype(np.int64) % n_src
        i1 = (i0 + 1) % n_src
    else:
        g = np.clip(g, 0.0, n_src - 1.0)
        i0 = np.minimum(np.floor(g).astype(np.int64), n_src - 2)
        f = g - i0
        i1 = i0 + 1
    return i0, i1, f


def upsample(spec_from, x_from: np.ndarray, spec_to) -> np.ndarray:
    """Parameters of the next hierarchical level from the current one by linear interpolation
    (Sec. IV): trilinear over the voxel grid, bilinear over each environment layer (periodic
    in azimuth, clamped in polar angle), at the new cell / texel centres.  sigma is an optical
    depth per shortest voxel side (the reading of delta), so it is scaled by the ratio of the
    new side to the old one; colours and texel opacities are interpolated as they are.
    Requires the same bounding box and environment layers."""
    xf = np.asarray(x_from, dtype=np.float64)
    nv = spec_from.n_vox
    grid = xf[:4 * nv].reshape(spec_from.nz, spec_from.ny, spec_from.nx, 4)
    env = xf[4 * nv:].reshape(spec_from.n_layers, spec_from.env_h, spec_from.env_w, 4)
    ix0, ix1, fx = _lerp_axis(spec_from.nx, spec_to.nx, False)
    iy0, iy1, fy = _lerp_axis(spec_from.ny, spec_to.ny, False)
    iz0, iz1, fz = _lerp_axis(spec_from.nz, spec_to.nz, False)
    out = np.zeros((spec_to.nz, spec_to.ny, spec_to.nx, 4))
    for bz, (iz, wz) in enumerate(((iz0, 1.0 - fz), (iz1, fz))):
        for by, (iy, wy) in enumerate(((iy0, 1.0 - fy), (iy1, fy))):
            for bx, (ix, wx) in enumerate(((ix0, 1.0 - fx), (ix1, fx))):
                w = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                out += w[..., None] * grid[np.ix_(iz, iy, ix)]
    out[..., 3] *= _shortest_side(spec_to) / _shortest_side(spec_from)
    iu0, iu1, fu = _lerp_axis(spec_from.env_w, spec_to.env_w, True)
    iv0, iv1, fv = _lerp_axis(spec_from.env_h, spec_to.env_h, False)
    eout = np.zeros((spec_to.n_layers, spec_to.env_h, spec_to.env_w, 4))
    for (iv, wv) in ((iv0, 1.0 - fv), (iv1, fv)):
        for (iu, wu) in ((iu0, 1.0 - fu), (iu1, fu)):
            w = wv[:, None] * wu[None, :]
            eout += w[None, :, :, None] * env[:, iv][:, :, iu]
    return np.concatenate([out.reshape(-1), eout.reshape(-1)])


def gn_step(scene: OracleScene, x: np.ndarray, targets: np.ndarray, precond: str = "jacobi", max_iters: int = 20,
            rel_tol: float = 0.0, abs_eps: float = 0.0, stall_ratio: float = 0.0, line_search_on: bool = True,
            ls_factor: float = 0.7, ls_max: int = 20, learned_minv=None):
    """One Gauss-Newton step (Eq. 7): b = -J^T r, PCG on J^T J Delta = b, Alg. 3, projected update.

    With precond='learned' (learned_minv: the predicted inverses), a solve that breaks down,
    stalls or whose line search finds no descent is discarded and the step solved again with
    the exact block inverse; fallback_iters then holds the discarded solve's iterations."""
    x = np.asarray(x, dtype=np.float64)
    grad, blocks, F0 = scene.grad_blocks(x, targets)
    if precond == "jacobi":
        data = jacobi_inverse(blocks)
    elif precond == "block":
        data = block_inverse(blocks)
    elif precond == "learned":
        data = learned_minv
    else:
        data = None
    spec = scene.spec

    def solve(kind, minv):
        res = pcg(lambda p: scene.apply_JtJ(x, p), grad, lambda r: apply_precond(kind, minv, r),
                  max_iters=max_iters, rel_tol=rel_tol, abs_eps=abs_eps, stall_ratio=stall_ratio)

        def objective(g):
            return scene.render(project(spec, x + g * res.x), targets)[2]

        if line_search_on:
            return (res,) + tuple(line_search(objective, F0, ls_factor, ls_max))
        return res, 1.0, objective(1.0), 1, False

    res, gamma, mu, n_ls, capped = solve(precond, data)
    fallback_iters = None
    if precond == "learned" and (res.flags & {"breakdown", "stall"} or gamma == 0.0):
        # a failed learned solve is replaced by the exact block-Jacobi solve (reading of this library)
        fallback_iters = res.iters
        res, gamma, mu, n_ls, capped = solve("block", block_inverse(blocks))
    delta = res.x
    x_new = project(spec, x + gamma * delta)
    return dict(x=x_new, delta=delta, gamma=gamma, F_before=F0, F_after=mu, pcg=res, blocks=blocks, grad=grad,
                n_ls=n_ls, ls_capped=capped, fallback_iters=fallback_iters)
