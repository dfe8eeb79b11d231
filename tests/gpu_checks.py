"""Helpers of the GPU parity tests: dense FP64 forms of the library's scaled preconditioner
outputs, and the check of PCG scalars against an FP64 run.

Jacobi: [units][4] t = D^-1/2 per parameter, M^-1 = t^2.
Block: [units][8] = (t_d, t_f, e~, 1/s, 0, 0), M^-1 = D^-1/2 [[I, e~], [e~^T, 1]]^-1 D^-1/2.
Learned: [units][12] = (t_d, t_f, L row by row), M^-1 = D^-1/2 L L^T D^-1/2.
D^-1/2 = diag(t_d, t_d, t_d, t_f).
"""
import numpy as np

TRIL = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3)]


def jacobi_minv(t):
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    return t * t


def _scale(q):
    return np.stack([q[:, 0], q[:, 0], q[:, 0], q[:, 1]], axis=1)


def block_inner(q):
    """[units, 4, 4] inverse of the normalised block, from a [units][8] form, in FP64."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 8)
    e, inv_s = q[:, 2:5], q[:, 5]
    N = np.zeros((q.shape[0], 4, 4))
    N[:, :3, :3] = np.eye(3)[None] * (inv_s != 0)[:, None, None] + e[:, :, None] * e[:, None, :] * inv_s[:, None, None]
    N[:, :3, 3] = -e * inv_s[:, None]
    N[:, 3, :3] = -e * inv_s[:, None]
    N[:, 3, 3] = inv_s
    return N


def block_minv(q):
    """[units, 4, 4] M^-1 of a [units][8] block form, formed in FP64."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 8)
    s = _scale(q)
    return s[:, :, None] * block_inner(q) * s[:, None, :]


def learned_factor(q):
    """[units, 4, 4] lower-triangular L of a [units][12] learned form."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 12)
    L = np.zeros((q.shape[0], 4, 4))
    for k, (i, j) in enumerate(TRIL):
        L[:, i, j] = q[:, 2 + k]
    return L


def learned_minv(q):
    """[units, 4, 4] M^-1 of a [units][12] learned form, formed in FP64."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 12)
    L = learned_factor(q)
    s = _scale(q)
    return s[:, :, None] * (L @ np.transpose(L, (0, 2, 1))) * s[:, None, :]


def check_pcg_history(st, pcg, n, tol=1e-4):
    """PCG scalars alpha_k and beta_k of the first n iterations against the FP64 run, each within
    tol relative (the J^T J v bound); R_k = |r_k|^2 carries the FP32 error of r_k, about
    tol |r_0| absolute, so its relative bound grows as 2 tol sqrt(R_0 / R_k) while CG converges."""
    R0 = pcg.R0
    ea, eb, er = [], [], []
    for k in range(n):
        Rk = pcg.R[k]
        ea.append(abs(st["alpha"][k] - pcg.alpha[k]) / abs(pcg.alpha[k]))
        er.append(abs(st["R"][k] - Rk) / Rk / (2 * np.sqrt(R0 / Rk)))
        if k < n - 1:
            eb.append(abs(st["beta"][k] - pcg.beta[k]) / abs(pcg.beta[k]))
    print(f"[pcg] alpha rel err {['%.1e' % e for e in ea]} beta {['%.1e' % e for e in eb]}", flush=True)
    assert not ea or max(ea) <= tol, ea
    assert not eb or max(eb) <= tol, eb
    assert not er or max(er) <= tol, er
