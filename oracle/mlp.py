"""FP64 reference of the learned block preconditioner (test infrastructure only).

Not part of the paper: the learned part replaces the exact inverse of each unit's
4x4 block of J^T J (Sec. III-G uses only its diagonal) with a prediction from cheap
per-unit features.  Conventions, identical to the product's:

  features:        6 per unit, from x and the unit's block alone: sigma/alpha, colour (3),
                   log d, log f
  weights, packed: W1[64][16] b1[64] W2[64][64] b2[64] W3[16][64] b3[16]
                   (inputs padded 10 -> 16, outputs 10 -> 16 with zeros)
  standardisation: norm = (mu[16], s[16]) from the training features: mu the mean and
                   s = 1 / max(std, 1e-3) per feature (0 for the other slots)
  inputs:          x[0:6] = clamp((feature - mu) s, -CLAMP, CLAMP) for the 6 features,
                   x[6:9] = e~, the normalised colour-density coupling of the unit's block
                   (the off-diagonal column of B~ below; |e~| < 1, used as is),
                   x[9] = -1/2 log(1 - |e~|^2) (the Schur complement's log; 8 where the
                   complement is at most exp(-16)), x[10:16] = 0
  network:         h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3
  factor:          L lower triangular from o[0:10] row by row, softplus on the diagonal
  ridge:           rho = 1e-6 max(d, f); D = diag(d, d, d, f) + rho I
  normalised block B~ = D^-1/2 (B + rho I) D^-1/2,  M^-1 = D^-1/2 L L^T D^-1/2
  fallback:        a unit whose prediction misses its own normalised block by
                   q = ||L L^T B~ - I||_F^2 > q_fallback takes the exact block inverse
                   (B + rho I)^-1 instead (plain block-Jacobi)
  loss per unit:   q = || L L^T (B~ + damp I) - I ||_F^2 (damp = 0: the exact inverse is the
                   target; larger damp moves it towards plain Jacobi), made robust above KAPPA:
                   q if q <= KAPPA, else 2 sqrt(KAPPA q) - KAPPA (linear in the norm), averaged
                   over all n units given (a unit no ray touches contributes zero)
"""
from __future__ import annotations

import numpy as np

N_IN, N_IN_PAD, N_HID, N_OUT, N_OUT_PAD = 6, 16, 64, 10, 16
N_CPL = 4               # network inputs taken from the block: e~ (3) and its Schur log
N_NET = N_IN + N_CPL    # network inputs in use
SCHUR_CAP = 8.0         # cap on the Schur log input
SHAPES = [("W1", (N_HID, N_IN_PAD)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT_PAD, N_HID)), ("b3", (N_OUT_PAD,))]
NW = sum(int(np.prod(s)) for _, s in SHAPES)
TRIL = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3)]
DIAG = [0, 2, 5, 9]
RIDGE = 1e-6
KAPPA = 4.0
CLAMP = 8.0
STD_FLOOR = 1e-3


def bf16_round(w: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (nearest even) and return them as float64."""
    f = np.asarray(w, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(w: np.ndarray) -> np.ndarray:
    f = np.asarray(w, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(w: np.ndarray) -> dict:
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == NW
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_weights(seed: int = 0) -> np.ndarray:
    """He-style initialisation; padded input columns and output rows are zero."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2.0 / N_NET), (N_HID, N_IN_PAD)), "b1": np.zeros(N_HID),
         "W2": rng.normal(0, np.sqrt(2.0 / N_HID), (N_HID, N_HID)), "b2": np.zeros(N_HID),
         "W3": rng.normal(0, np.sqrt(1.0 / N_HID), (N_OUT_PAD, N_HID)), "b3": np.zeros(N_OUT_PAD)}
    p["W1"][:, N_NET:] = 0.0
    p["W3"][N_OUT:, :] = 0.0
    p["W3"] *= 0.1
    p["b3"][DIAG] = 0.5413  # softplus(0.5413) = 1: start at L = I, i.e. plain Jacobi
    return pack(p)


def features(x: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """[units, 6]: sigma/alpha, colour (3), log d, log f."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 4)
    b = np.asarray(blocks, dtype=np.float64)
    f = np.zeros((x.shape[0], N_IN))
    f[:, 0] = x[:, 3]
    f[:, 1:4] = x[:, 0:3]
    f[:, 4] = np.log(np.maximum(b[:, 0], 0.0) + 1e-12)
    f[:, 5] = np.log(np.maximum(b[:, 4], 0.0) + 1e-12)
    return f


def feature_stats(feat: np.ndarray) -> np.ndarray:
    """norm [32] = (mu[16], s[16]) of a training set: per-feature mean and 1 / max(std, 1e-3),
    std the population standard deviation; zeros for the other slots."""
    f = np.asarray(feat, dtype=np.float64).reshape(-1, N_IN)
    mu = f.mean(axis=0)
    sd = np.sqrt(np.maximum((f * f).mean(axis=0) - mu * mu, 0.0))
    norm = np.zeros(2 * N_IN_PAD)
    norm[:N_IN] = mu
    norm[N_IN_PAD:N_IN_PAD + N_IN] = 1.0 / np.maximum(sd, STD_FLOOR)
    return norm


def standardise(norm: np.ndarray, feat: np.ndarray) -> np.ndarray:
    """[n, 16] network inputs: clamp((feature - mu) s, -CLAMP, CLAMP), zero padding."""
    norm = np.asarray(norm, dtype=np.float64).reshape(-1)
    f = np.asarray(feat, dtype=np.float64).reshape(-1, N_IN)
    x = np.zeros((f.shape[0], N_IN_PAD))
    x[:, :N_IN] = np.clip((f - norm[:N_IN]) * norm[N_IN_PAD:N_IN_PAD + N_IN], -CLAMP, CLAMP)
    return x


def inputs(norm: np.ndarray, feat: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """[n, 16] network inputs: the standardised stored features, then e~ of each unit's block and
    -1/2 log(s) with s = 1 - |e~|^2 the Schur complement of B~ (the inverse's entries grow as 1/s),
    SCHUR_CAP where s <= exp(-2 SCHUR_CAP); all zero for a unit with no rays or a non-finite block;
    then zeros."""
    x = standardise(norm, feat)
    Bn, _, live = normalised_block(blocks)
    e = Bn[:, 0:3, 3]
    x[:, N_IN:N_IN + 3] = e
    s = 1.0 - (e * e).sum(axis=1)
    ok = live & (s > np.exp(-2.0 * SCHUR_CAP))  # else the cap (also for a block that rounding left indefinite)
    x[:, N_IN + 3] = np.where(ok, -0.5 * np.log(np.where(ok, s, 1.0)), np.where(live, SCHUR_CAP, 0.0))
    return x


def forward(w: np.ndarray, norm: np.ndarray, feat: np.ndarray, blocks: np.ndarray, emulate_bf16: bool = False):
    """Raw outputs [n, 10] and the activations needed for the backward pass.

    emulate_bf16 rounds the input and both hidden activations to bfloat16 before the
    next product, as a bfloat16 matrix-core implementation does (products and sums
    stay exact here)."""
    p = unpack(w)
    rnd = bf16_round if emulate_bf16 else (lambda a: a)
    x = rnd(inputs(norm, feat, blocks))
    z1 = x @ p["W1"].T + p["b1"]
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = rnd(np.maximum(z2, 0.0))
    o = h2 @ p["W3"].T + p["b3"]
    return o[:, :N_OUT], (x, z1, h1, z2, h2)


def softplus(v):
    return np.logaddexp(0.0, v)


def factor(raw: np.ndarray) -> np.ndarray:
    """[n, 4, 4] lower-triangular L with softplus on the diagonal."""
    L = np.zeros((raw.shape[0], 4, 4))
    for k, (i, j) in enumerate(TRIL):
        L[:, i, j] = softplus(raw[:, k]) if k in DIAG else raw[:, k]
    return L


def normalised_block(blocks: np.ndarray):
    """(B~ [n,4,4], D^-1/2 [n,4], live mask)."""
    b = np.asarray(blocks, dtype=np.float64)
    d, e, f = b[:, 0], b[:, 1:4], b[:, 4]
    m = np.maximum(d, f)
    live = (m > 0) & np.all(np.isfinite(b), axis=1)  # a non-finite block counts as an empty unit
    rho = RIDGE * np.where(live, m, 0.0)
    dd, ff = d + rho, f + rho
    sd = np.where(live, 1.0 / np.sqrt(np.where(live, dd, 1.0)), 0.0)
    sf = np.where(live, 1.0 / np.sqrt(np.where(live, ff, 1.0)), 0.0)
    Bn = np.zeros((b.shape[0], 4, 4))
    for i in range(3):
        Bn[:, i, i] = np.where(live, 1.0, 0.0)
        Bn[:, i, 3] = np.where(live, e[:, i] * sd * sf, 0.0)
        Bn[:, 3, i] = np.where(live, e[:, i] * sd * sf, 0.0)
    Bn[:, 3, 3] = np.where(live, 1.0, 0.0)
    dis = np.stack([sd, sd, sd, sf], axis=1)
    return Bn, dis, live


def prediction_error(L: np.ndarray, Bn: np.ndarray) -> np.ndarray:
    """q = ||L L^T B~ - I||_F^2 per unit."""
    E = (L @ np.transpose(L, (0, 2, 1))) @ Bn - np.eye(4)[None]
    return (E * E).sum(axis=(1, 2))


def minv(w: np.ndarray, norm: np.ndarray, feat: np.ndarray, blocks: np.ndarray, emulate_bf16: bool = False,
         q_fallback: float = np.inf, return_fallback: bool = False):
    """[n, 4, 4] M^-1 = D^-1/2 L L^T D^-1/2, zero for units with no rays; units whose q exceeds
    q_fallback get the exact block inverse (B + rho I)^-1.  With return_fallback, also the
    [n] mask of those units and their q."""
    raw, _ = forward(w, norm, feat, blocks, emulate_bf16)
    L = factor(raw)
    Bn, dis, live = normalised_block(blocks)
    q = prediction_error(L, Bn)
    fb = live & ~(q <= q_fallback)  # (a non-finite prediction falls back too)
    N = L @ np.transpose(L, (0, 2, 1))
    if np.any(fb):
        N[fb] = np.linalg.inv(Bn[fb])
    M = dis[:, :, None] * N * dis[:, None, :]
    M[~live] = 0.0
    return (M, fb, q) if return_fallback else M


def loss_and_grad(w: np.ndarray, norm: np.ndarray, feat: np.ndarray, blocks: np.ndarray, damp: float = 0.0):
    """Mean over the n given units of the robust ||L L^T (B~ + damp I) - I||_F^2 (zero for
    units no ray touches) and its gradient w.r.t. the packed weights (the standardisation is
    fixed, not trained)."""
    p = unpack(w)
    raw, (x, z1, h1, z2, h2) = forward(w, norm, feat, blocks)
    L = factor(raw)
    Bn, _, live = normalised_block(blocks)
    Bn = Bn + damp * np.where(live, 1.0, 0.0)[:, None, None] * np.eye(4)[None]
    n_live = max(int(raw.shape[0]), 1)
    P = L @ np.transpose(L, (0, 2, 1))
    E = P @ Bn - np.eye(4)[None]
    E[~live] = 0.0
    q = (E * E).sum(axis=(1, 2))
    big = q > KAPPA
    lu = np.where(big, 2.0 * np.sqrt(KAPPA * np.where(big, q, 1.0)) - KAPPA, q)
    scale = np.where(big, np.sqrt(KAPPA / np.where(big, q, 1.0)), 1.0)  # d lu / d q
    loss = float(lu.sum()) / n_live
    G = 2.0 * (scale[:, None, None] * E) @ Bn / n_live   # d loss / d P
    dL = (G + np.transpose(G, (0, 2, 1))) @ L      # d loss / d L
    draw = np.zeros_like(raw)
    for k, (i, j) in enumerate(TRIL):
        draw[:, k] = dL[:, i, j] * (1.0 / (1.0 + np.exp(-raw[:, k])) if k in DIAG else 1.0)
    do = np.zeros((raw.shape[0], N_OUT_PAD))
    do[:, :N_OUT] = draw
    g = {"W3": do.T @ h2, "b3": do.sum(0)}
    dh2 = do @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def raw_from_factor(L: np.ndarray) -> np.ndarray:
    """Inverse of `factor`: raw outputs that reproduce a given L (positive diagonal)."""
    raw = np.zeros((L.shape[0], N_OUT))
    for k, (i, j) in enumerate(TRIL):
        v = L[:, i, j]
        raw[:, k] = np.log(np.expm1(v)) if k in DIAG else v
    return raw
