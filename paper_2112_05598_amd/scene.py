"""Python handle over the C ABI: device memory and streams come from PyTorch,
every step of the computation runs in libperf_gn.so."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import abi

_PRECOND = {"none": abi.PERF_PRECOND_NONE, "jacobi": abi.PERF_PRECOND_JACOBI, "block": abi.PERF_PRECOND_BLOCK4,
            "learned": abi.PERF_PRECOND_LEARNED}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_desc(spec, width: int, height: int, param_dtype: str = "f32", checks: bool = False,
              learned: bool = False, aux_lambda: float = 0.0, render_threshold: float = 0.0) -> abi.perf_scene_desc:
    d = abi.perf_scene_desc()
    d.nx, d.ny, d.nz = spec.nx, spec.ny, spec.nz
    for i in range(3):
        d.bbox_min[i] = spec.bbox_min[i]
        d.bbox_max[i] = spec.bbox_max[i]
        d.background[i] = spec.background[i]
    d.n_layers = len(spec.layer_radii)
    d.env_w, d.env_h = spec.env_w, spec.env_h
    for i, r in enumerate(spec.layer_radii):
        d.layer_radius[i] = r
    d.step_vox = spec.step_vox
    d.param_dtype = abi.PERF_BF16 if param_dtype == "bf16" else abi.PERF_F32
    d.width, d.height = width, height
    d.checks = 1 if checks else 0
    d.learned = 1 if learned else 0
    d.aux_lambda = aux_lambda
    d.render_threshold = render_threshold
    return d


def make_cameras(cams) -> ctypes.Array:
    arr = (abi.perf_camera * cams.n)()
    for c in range(cams.n):
        for i in range(3):
            arr[c].origin[i] = float(cams.origin[c][i])
        rot = np.asarray(cams.rot[c], dtype=np.float64).reshape(3, 3)
        for i in range(9):
            arr[c].rot[i] = float(rot.reshape(-1)[i])
        arr[c].fx, arr[c].fy = float(cams.fx[c]), float(cams.fy[c])
        arr[c].cx, arr[c].cy = float(cams.cx[c]), float(cams.cy[c])
    return arr


class Scene:
    """A grid + environment layers + posed images living on one GPU.

    aux_lambda > 0 turns on the per-ray opacity residual of Sec. III-I (Eq. 10): residual, J v and
    J^T u vectors then hold n_res = 4 values per ray instead of 3.  render_threshold > 0 applies
    the rendering rule of Sec. IV in render_residuals (a volume with opacity below it is dropped)."""

    def __init__(self, spec, cams, targets: Optional[torch.Tensor] = None, param_dtype: str = "f32",
                 checks: bool = False, learned: bool = False, device: str = "cuda", aux_lambda: float = 0.0,
                 render_threshold: float = 0.0):
        self.lib = abi.load()
        self.spec = spec
        self.device = torch.device(device)
        self.param_dtype = param_dtype
        self.desc = make_desc(spec, cams.width, cams.height, param_dtype, checks, learned, aux_lambda,
                              render_threshold)
        self.aux_lambda = float(aux_lambda)
        self.n_res = 4 if aux_lambda > 0 else 3
        self._cams = make_cameras(cams)
        n = cams.n
        nbytes = int(self.lib.perf_workspace_bytes(ctypes.byref(self.desc), n))
        if nbytes == 0:
            abi.check(abi.PERF_EINVAL)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self._ws_bytes = nbytes
        self._targets = targets
        h = ctypes.c_void_p()
        abi.check(self.lib.perf_init_scene(ctypes.byref(self.desc), self._cams, n, _ptr(targets),
                                           ctypes.c_void_p(self._ws_ptr), nbytes, self._stream(), ctypes.byref(h)))
        self.handle = h
        nr, nu, npar = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        abi.check(self.lib.perf_scene_sizes(h, ctypes.byref(nr), ctypes.byref(nu), ctypes.byref(npar)))
        self.n_rays, self.n_units, self.n_params = nr.value, nu.value, npar.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.perf_destroy_scene(h)
            self.handle = None

    # ------------------------------------------------------------ plumbing
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _bind(self):
        abi.check(self.lib.perf_set_stream(self.handle, self._stream()))

    def _check_params(self, x: torch.Tensor):
        want = torch.float32 if self.param_dtype == "f32" else torch.bfloat16
        if x.dtype != want or x.numel() != self.n_params or not x.is_contiguous() or x.device != self.device:
            raise ValueError(f"parameters must be a contiguous {self.n_params}-element {want} tensor on {self.device}")

    def _vec(self, t: torch.Tensor, n: int, name: str):
        if t.dtype != torch.float32 or t.numel() != n or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements on {self.device}")

    def set_jitter(self, seed: int):
        """Jittered ray origins and sample positions (Sec. IV) for every later call; 0 = off.
        Keep one seed per Gauss-Newton step."""
        abi.check(self.lib.perf_set_jitter(self.handle, ctypes.c_uint32(int(seed) & 0xFFFFFFFF)))

    def set_targets(self, targets: torch.Tensor):
        self._vec(targets, 3 * self.n_rays, "targets")
        self._targets = targets
        abi.check(self.lib.perf_set_targets(self.handle, _ptr(targets)))

    def pack_bf16(self, x: torch.Tensor) -> torch.Tensor:
        self._vec(x, x.numel(), "x")
        out = torch.empty(x.numel(), dtype=torch.bfloat16, device=self.device)
        abi.check(self.lib.perf_pack_bf16(_ptr(x), _ptr(out), x.numel(), self._stream()))
        return out

    # ------------------------------------------------------------ operators
    def render_residuals(self, x: torch.Tensor, want_r: bool = True):
        self._check_params(x)
        self._bind()
        per = self.n_res if self._targets is not None else 3
        r = torch.empty(self.n_rays * per, dtype=torch.float32, device=self.device) if want_r else None
        F = torch.zeros(1, dtype=torch.float64, device=self.device)
        abi.check(self.lib.perf_render_residuals(self.handle, _ptr(x), _ptr(r), _ptr(F)))
        return r, F

    def apply_J(self, x, v, out=None):
        self._check_params(x)
        self._vec(v, self.n_params, "v")
        self._bind()
        if out is not None:
            self._vec(out, self.n_res * self.n_rays, "out")
        u = out if out is not None else torch.empty(self.n_rays * self.n_res, dtype=torch.float32, device=self.device)
        abi.check(self.lib.perf_apply_J(self.handle, _ptr(x), _ptr(v), _ptr(u)))
        return u

    def apply_Jt(self, x, u, out=None):
        self._check_params(x)
        self._vec(u, self.n_res * self.n_rays, "u")
        self._bind()
        y = out if out is not None else torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        abi.check(self.lib.perf_apply_Jt(self.handle, _ptr(x), _ptr(u), _ptr(y)))
        return y

    def apply_JtJ(self, x, v, out=None):
        self._check_params(x)
        self._vec(v, self.n_params, "v")
        self._bind()
        y = out if out is not None else torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        abi.check(self.lib.perf_apply_JtJ(self.handle, _ptr(x), _ptr(v), _ptr(y)))
        return y

    def build_precond(self, x, kind: str = "jacobi"):
        """(grad = -J^T r [P], blocks [units,5], M^-1 in scaled form ([units,4] Jacobi D^-1/2 or
        [units,8] block (t_d, t_f, e~, 1/s, 0, 0)), F)."""
        self._check_params(x)
        self._bind()
        k = _PRECOND[kind]
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        blocks = torch.empty(self.n_units * 5, dtype=torch.float32, device=self.device)
        out = None
        if k == abi.PERF_PRECOND_JACOBI:
            out = torch.empty(self.n_units, 4, dtype=torch.float32, device=self.device)
        elif k == abi.PERF_PRECOND_BLOCK4:
            out = torch.empty(self.n_units, 8, dtype=torch.float32, device=self.device)
        F = torch.zeros(1, dtype=torch.float64, device=self.device)
        abi.check(self.lib.perf_build_precond(self.handle, _ptr(x), k, _ptr(grad), _ptr(blocks), _ptr(out), _ptr(F)))
        return grad, blocks.view(-1, 5), out, F

    def objective(self, x, delta=None, gamma: float = 1.0) -> float:
        self._vec(x, self.n_params, "x")
        self._bind()
        F = ctypes.c_double()
        abi.check(self.lib.perf_objective(self.handle, _ptr(x), _ptr(delta), ctypes.c_float(gamma), ctypes.byref(F)))
        return F.value

    def footprint(self, per_ray: bool = True):
        self._bind()
        pr = torch.empty(self.n_rays * 2, dtype=torch.int32, device=self.device) if per_ray else None
        tot = torch.zeros(3, dtype=torch.int64, device=self.device)
        abi.check(self.lib.perf_footprint(self.handle, _ptr(pr), _ptr(tot)))
        return (pr.view(-1, 2) if pr is not None else None), tot

    # ------------------------------------------------------------ learned preconditioner
    def features(self, x):
        """(features [units, PERF_MLP_NFEAT], exact blocks [units, 5]) at x: one gradient/block
        traversal; the features come from x and the blocks."""
        self._check_params(x)
        self._bind()
        feat = torch.empty(self.n_units * abi.PERF_MLP_NFEAT, dtype=torch.float32, device=self.device)
        blocks = torch.empty(self.n_units * 5, dtype=torch.float32, device=self.device)
        abi.check(self.lib.perf_precond_features(self.handle, _ptr(x), _ptr(feat), _ptr(blocks)))
        return feat.view(-1, abi.PERF_MLP_NFEAT), blocks.view(-1, 5)

    def mlp_set_weights(self, w_bf16: torch.Tensor, norm: torch.Tensor, q_fallback: float = float("inf")):
        """Network weights (bfloat16 [PERF_MLP_NW]), standardisation (float32 [PERF_MLP_NNORM]) and
        the per-unit fallback threshold on q = ||L L^T B~ - I||_F^2 (inf: never)."""
        if w_bf16.dtype != torch.bfloat16 or w_bf16.numel() != abi.PERF_MLP_NW or w_bf16.device != self.device:
            raise ValueError("weights must be a bfloat16 tensor of PERF_MLP_NW elements on the scene's device")
        if norm.dtype != torch.float32 or norm.numel() != abi.PERF_MLP_NNORM or norm.device != self.device:
            raise ValueError("norm must be a float32 tensor of PERF_MLP_NNORM elements on the scene's device")
        self._bind()
        self._mlp_w = w_bf16.contiguous()
        self._mlp_norm = norm.contiguous()
        abi.check(self.lib.perf_mlp_set_weights(self.handle, _ptr(self._mlp_w), abi.PERF_MLP_NW, _ptr(self._mlp_norm),
                                                ctypes.c_float(q_fallback)))

    def training_rows(self, feat: torch.Tensor, blocks: torch.Tensor, seed: int, keep: float, cap: int):
        """(features [k, PERF_MLP_NFEAT], blocks [k, 5], n_kept) for a random subset of the touched units
        (library-side sampling: each kept with probability keep; at most cap rows written, unit
        order; cap = 0 only counts)."""
        self._bind()
        fo = torch.empty(max(cap, 1) * abi.PERF_MLP_NFEAT, dtype=torch.float32, device=self.device)
        bo = torch.empty(max(cap, 1) * 5, dtype=torch.float32, device=self.device)
        n = ctypes.c_int64()
        abi.check(self.lib.perf_mlp_training_rows(self.handle, _ptr(feat.contiguous()), _ptr(blocks.contiguous()),
                                                  ctypes.c_uint32(int(seed) & 0xFFFFFFFF), ctypes.c_float(keep),
                                                  _ptr(fo) if cap else None, _ptr(bo) if cap else None, cap,
                                                  ctypes.byref(n)))
        k = min(n.value, cap)
        return fo.view(-1, abi.PERF_MLP_NFEAT)[:k], bo.view(-1, 5)[:k], n.value

    def mlp_infer(self, feat: torch.Tensor, blocks: torch.Tensor):
        """[units, 12] predicted block inverses in scaled form (t_d, t_f, L row by row)."""
        self._bind()
        out = torch.empty(self.n_units * 12, dtype=torch.float32, device=self.device)
        abi.check(self.lib.perf_mlp_infer(self.handle, _ptr(feat.contiguous()), _ptr(blocks.contiguous()),
                                          _ptr(out)))
        return out.view(-1, 12)

    def gn_step(self, x: torch.Tensor, max_iters: int = 20, precond: str = "jacobi", rel_tol: float = 0.0,
                abs_eps: float = 0.0, stall_ratio: float = 0.0, line_search: bool = True, ls_factor: float = 0.7,
                ls_max: int = 20) -> dict:
        self._vec(x, self.n_params, "x")
        self._bind()
        o = abi.perf_pcg_opts()
        o.max_iters, o.rel_tol, o.abs_eps, o.stall_ratio = max_iters, rel_tol, abs_eps, stall_ratio
        o.precond = _PRECOND[precond]
        o.line_search = 1 if line_search else 0
        o.ls_factor, o.ls_max = ls_factor, ls_max
        st = abi.perf_gn_stats()
        abi.check(self.lib.perf_gn_step(self.handle, _ptr(x), ctypes.byref(o), ctypes.byref(st)))
        k = st.pcg_iters
        return dict(F_before=st.F_before, F_after=st.F_after, gamma=st.gamma, pcg_iters=k, ls_trials=st.ls_trials,
                    flags=st.flags, fallback_iters=st.fallback_iters, R0=st.R0, R=list(st.R[:k]), alpha=list(st.alpha[:k]),
                    beta=list(st.beta[:max(k - 1, 0)]), pAp=list(st.pAp[:k + 1]), ms_phase=list(st.ms_phase[:6]), ms_jtj=st.ms_phase[6], n_jtj=int(st.ms_phase[7]))


def mlp_train_step(w32, wbf16, m, v, t: int, lr: float, norm, feat, blocks, loss, grad, stream=None,
                   damp: float = 0.0):
    """One Adam step of the learned preconditioner on a batch (feat [n, PERF_MLP_NFEAT], blocks [n, 5]) with the
    fixed standardisation norm [32]; the target is the damped normalised inverse (B~ + damp I)^-1."""
    lib = abi.load()
    n = int(feat.shape[0])
    st = ctypes.c_void_p(torch.cuda.current_stream(feat.device).cuda_stream) if stream is None else stream
    abi.check(lib.perf_mlp_train_step(_ptr(w32), _ptr(wbf16), _ptr(m), _ptr(v), int(t), ctypes.c_float(lr),
                                      ctypes.c_float(damp), _ptr(norm), _ptr(feat), _ptr(blocks), n, _ptr(loss),
                                      _ptr(grad), st))


def mlp_feature_stats(feat: torch.Tensor, stream=None) -> torch.Tensor:
    """Standardisation [32] = (mu[16], s[16]) of a training set of features [n, PERF_MLP_NFEAT]
    (library-side)."""
    lib = abi.load()
    if feat.dtype != torch.float32 or not feat.is_cuda or feat.dim() != 2 or feat.shape[1] != abi.PERF_MLP_NFEAT:
        raise ValueError(f"features must be a float32 device tensor of shape [n, {abi.PERF_MLP_NFEAT}]")
    out = torch.empty(abi.PERF_MLP_NNORM, dtype=torch.float32, device=feat.device)
    st = ctypes.c_void_p(torch.cuda.current_stream(feat.device).cuda_stream) if stream is None else stream
    abi.check(lib.perf_mlp_feature_stats(_ptr(feat.contiguous()), feat.shape[0], _ptr(out), st))
    return out


def upsample(spec_from, x_from: torch.Tensor, spec_to, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Parameters of the next hierarchical level from those of the current one (perf_upsample):
    linear interpolation at the new cell / texel centres, sigma scaled by the voxel-side ratio."""
    lib = abi.load()
    n_from = 4 * (spec_from.n_vox + spec_from.n_texels)
    n_to = 4 * (spec_to.n_vox + spec_to.n_texels)
    if x_from.dtype != torch.float32 or not x_from.is_cuda or not x_from.is_contiguous() or x_from.numel() != n_from:
        raise ValueError(f"x_from must be a contiguous float32 device tensor of {n_from} values")
    if out is None:
        out = torch.empty(n_to, dtype=torch.float32, device=x_from.device)
    elif out.dtype != torch.float32 or out.numel() != n_to or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float32 tensor of {n_to} values")
    d_from = make_desc(spec_from, 1, 1)
    d_to = make_desc(spec_to, 1, 1)
    st = ctypes.c_void_p(torch.cuda.current_stream(x_from.device).cuda_stream) if stream is None else stream
    abi.check(lib.perf_upsample(ctypes.byref(d_from), _ptr(x_from), ctypes.byref(d_to), _ptr(out), st))
    return out


def invert_blocks(blocks: torch.Tensor, kind: str = "jacobi", stream=None) -> torch.Tensor:
    """Preconditioner of given (d, e_r, e_g, e_b, f) blocks [units, 5] in scaled form
    (perf_invert_blocks): [units, 4] Jacobi D^-1/2 or [units, 8] (t_d, t_f, e~, 1/s, 0, 0)."""
    lib = abi.load()
    if blocks.dtype != torch.float32 or not blocks.is_cuda or not blocks.is_contiguous() or blocks.dim() != 2 \
            or blocks.shape[1] != 5:
        raise ValueError("blocks must be a contiguous float32 device tensor of shape [units, 5]")
    k = _PRECOND[kind]
    width = {abi.PERF_PRECOND_JACOBI: 4, abi.PERF_PRECOND_BLOCK4: 8}.get(k)
    if width is None:
        raise ValueError("kind must be 'jacobi' or 'block'")
    out = torch.empty(blocks.shape[0], width, dtype=torch.float32, device=blocks.device)
    st = ctypes.c_void_p(torch.cuda.current_stream(blocks.device).cuda_stream) if stream is None else stream
    abi.check(lib.perf_invert_blocks(_ptr(blocks), blocks.shape[0], k, _ptr(out), st))
    return out
