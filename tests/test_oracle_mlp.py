"""Pins of the FP64 learned-preconditioner reference (CPU only)."""
import numpy as np
import pytest

import perf_synth as ps


@pytest.fixture(scope="module")
def mlp(oracle_mod):
    from oracle import mlp
    return mlp


def unit_norm(mlp):
    """Standardisation that leaves features within the clamp unchanged (mu = 0, s = 1)."""
    norm = np.zeros(2 * mlp.N_IN_PAD)
    norm[mlp.N_IN_PAD:mlp.N_IN_PAD + mlp.N_IN] = 1.0
    return norm


def random_blocks(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.1, 5.0, n)
    f = rng.uniform(0.1, 5.0, n)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rho = rng.uniform(0.0, 0.95, n)  # |e~| < 1: the block is positive definite
    e = dirs * (rho * np.sqrt(d * f))[:, None]
    b = np.concatenate([d[:, None], e, f[:, None]], axis=1)
    b[:3] = 0.0  # units no ray touches
    return b


def unit_errors(mlp, w, feat, blocks, damp):
    """||L L^T (B~ + damp I) - I||_F^2 per unit, assembled independently of loss_and_grad."""
    L = mlp.factor(mlp.forward(w, unit_norm(mlp), feat, blocks)[0])
    Bn, _, live = mlp.normalised_block(blocks)
    E = L @ np.transpose(L, (0, 2, 1)) @ (Bn + damp * np.eye(4)) - np.eye(4)
    q = (E * E).sum(axis=(1, 2))
    q[~live] = 0.0
    return q


@pytest.mark.parametrize("damp", [0.0, 0.3])
def test_loss_gradient_matches_finite_differences(mlp, damp):
    rng = np.random.default_rng(0)
    w = mlp.init_weights(1) + 0.05 * rng.normal(size=mlp.NW)
    feat = rng.normal(size=(40, mlp.N_IN))
    blocks = random_blocks(40, 2)
    q = unit_errors(mlp, w, feat, blocks, damp)
    # both branches of the robust loss are exercised
    assert np.any(q > mlp.KAPPA) and np.any((q > 0) & (q < mlp.KAPPA))
    norm = unit_norm(mlp)
    loss, g = mlp.loss_and_grad(w, norm, feat, blocks, damp)
    expect = np.where(q > mlp.KAPPA, 4.0 * np.sqrt(q) - 4.0, q).sum() / 40
    assert abs(loss - expect) <= 1e-12 * expect
    idx = rng.choice(mlp.NW, 60, replace=False)
    eps = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd = (mlp.loss_and_grad(wp, norm, feat, blocks, damp)[0]
              - mlp.loss_and_grad(wm, norm, feat, blocks, damp)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_robust_loss_is_continuous_at_kappa(mlp):
    """Quadratic below KAPPA, 2 sqrt(KAPPA q) - KAPPA above: value and slope agree at KAPPA."""
    k = mlp.KAPPA
    above = lambda q: 2.0 * np.sqrt(k * q) - k  # noqa: E731
    assert abs(above(k) - k) < 1e-12
    h = 1e-6
    assert abs((above(k + h) - above(k)) / h - 1.0) < 1e-5


@pytest.mark.parametrize("damp", [0.0, 0.5])
def test_damped_inverse_is_a_zero_of_the_loss(mlp, damp):
    """Raw outputs from the Cholesky factor of (B~ + damp I)^-1 give zero loss and zero
    gradient through the last layer's bias (the network reproduces them when W3 = 0)."""
    blocks = random_blocks(30, 8)
    Bn, dis, live = mlp.normalised_block(blocks)
    L = np.zeros_like(Bn)
    L[live] = np.linalg.cholesky(np.linalg.inv(Bn[live] + damp * np.eye(4)))
    L[~live] = np.eye(4)
    # one unit at a time: a network with W3 = 0 outputs b3 for every input
    for u in np.nonzero(live)[0][:5]:
        p = mlp.unpack(mlp.init_weights(3))
        p["W3"][:] = 0.0
        p["b3"][:] = 0.0
        p["b3"][:10] = mlp.raw_from_factor(L[u:u + 1])[0]
        loss, g = mlp.loss_and_grad(mlp.pack(p), unit_norm(mlp), np.zeros((1, mlp.N_IN)), blocks[u:u + 1], damp)
        assert loss < 1e-20
        assert np.abs(g).max() < 1e-9


def test_exact_factor_reproduces_block_inverse(mlp, oracle_mod):
    """Plugging in the Cholesky factor of the exact normalised inverse gives back the
    ridge-regularised block inverse, through the same assembly as the network output."""
    blocks = random_blocks(50, 3)
    Bn, dis, live = mlp.normalised_block(blocks)
    L = np.zeros_like(Bn)
    L[live] = np.linalg.cholesky(np.linalg.inv(Bn[live]))
    L[~live] = np.eye(4)
    raw = mlp.raw_from_factor(L)
    L2 = mlp.factor(raw)
    np.testing.assert_allclose(L2[live], L[live], rtol=1e-10, atol=1e-12)
    P = L2 @ np.transpose(L2, (0, 2, 1))
    M = dis[:, :, None] * P * dis[:, None, :]
    M[~live] = 0.0
    ref = oracle_mod.block_inverse(blocks)
    np.testing.assert_allclose(M, ref, rtol=1e-8, atol=1e-12)


def test_initial_network_is_jacobi(mlp, oracle_mod):
    """The initial weights output L = I exactly, i.e. M^-1 = D^-1 (Jacobi with the ridge)."""
    w = mlp.init_weights(5)
    p = mlp.unpack(w)
    p["W3"][:] = 0.0
    w = mlp.pack(p)
    blocks = random_blocks(20, 6)
    feat = np.random.default_rng(1).normal(size=(20, mlp.N_IN))
    M = mlp.minv(w, unit_norm(mlp), feat, blocks)
    sp = np.logaddexp(0.0, 0.5413)
    b = blocks
    rho = 1e-6 * np.maximum(b[:, 0], b[:, 4])
    for u in range(3, 20):
        np.testing.assert_allclose(np.diag(M[u]), sp ** 2 / np.array([b[u, 0] + rho[u]] * 3 + [b[u, 4] + rho[u]]),
                                   rtol=1e-12)


def test_bf16_rounding(mlp):
    # bfloat16 keeps 8 significant bits: the spacing just above 1 is 2^-7
    v = np.array([1.0, 1.0078125, 1.00390625, 3.14159, -2.5e-3, 0.0, 1.01171875], dtype=np.float32)
    r = mlp.bf16_round(v)
    np.testing.assert_array_equal(r[[0, 1, 5]], [1.0, 1.0078125, 0.0])
    assert r[2] == 1.0  # a tie rounds to the even neighbour
    assert r[6] == 1.015625  # the other tie, 1 + 3 * 2^-8, rounds up to the even 1 + 2 * 2^-7
    assert abs(r[3] - 3.140625) < 1e-12
    np.testing.assert_array_equal(mlp.bits_to_f64(mlp.bf16_bits(v)), r)


def test_learned_inverse_scales_with_the_block(mlp):
    """M^-1 = D^-1/2 L L^T D^-1/2 with B~ = D^-1/2 B D^-1/2 scale-free: scaling a block by s scales
    the predicted inverse by 1/s exactly, at any s (no threshold on tiny diagonals)."""
    w = mlp.init_weights(5)
    blocks = random_blocks(6, 8)
    feat = np.random.default_rng(2).normal(size=(6, mlp.N_IN))
    M1 = mlp.minv(w, unit_norm(mlp), feat, blocks)
    for s in (1e-20, 1e-41):
        Ms = mlp.minv(w, unit_norm(mlp), feat, blocks * s)
        np.testing.assert_allclose(Ms * s, M1, rtol=1e-12, atol=0)
    # units no ray touches get 0; the others are symmetric positive definite
    assert np.all(M1[:3] == 0)
    assert np.all(np.linalg.eigvalsh(M1[3:]) > 0)


def test_feature_stats_closed_form(mlp):
    """Column i = a_i + b_i t with t = +-1 alternating: mean a_i, population std |b_i|; a
    constant column gets s = 1 / 1e-3; the padding stays 0."""
    a = np.linspace(-20.0, 5.0, 6)
    b = np.linspace(0.5, 3.0, 6)
    b[4] = 0.0
    t = np.tile([1.0, -1.0], 50)
    feat = a[None, :] + b[None, :] * t[:, None]
    norm = mlp.feature_stats(feat)
    np.testing.assert_allclose(norm[:6], a, rtol=1e-14, atol=1e-13)
    want = 1.0 / np.maximum(np.abs(b), 1e-3)
    np.testing.assert_allclose(norm[16:22], want, rtol=1e-12)
    assert np.all(norm[6:16] == 0) and np.all(norm[22:32] == 0)


def test_standardise_centres_scales_and_clamps(mlp):
    rng = np.random.default_rng(3)
    feat = rng.normal(size=(200, 6)) * 4.0 + 10.0
    norm = mlp.feature_stats(feat)
    x = mlp.standardise(norm, feat)
    inner = np.abs(x[:, :6]) < mlp.CLAMP
    z = (feat - feat.mean(0)) / feat.std(0)
    np.testing.assert_allclose(x[:, :6][inner], z[inner], rtol=1e-12)
    far = feat.copy(); far[0, 3] = 1e6; far[1, 5] = -1e6
    xf = mlp.standardise(norm, far)
    assert xf[0, 3] == mlp.CLAMP and xf[1, 5] == -mlp.CLAMP
    assert np.all(x[:, 6:] == 0)


def test_fallback_units_take_the_exact_block_inverse(mlp, oracle_mod):
    """Units whose prediction error q exceeds the threshold get (B + rho I)^-1 exactly, the
    others keep D^-1/2 L L^T D^-1/2; a threshold of 0 turns the whole preconditioner into
    plain block-Jacobi, an infinite one never falls back."""
    rng = np.random.default_rng(11)
    w = mlp.init_weights(4) + 0.2 * rng.normal(size=mlp.NW)
    blocks = random_blocks(60, 5)
    feat = rng.normal(size=(60, mlp.N_IN))
    norm = unit_norm(mlp)
    M_all, fb_all, q = mlp.minv(w, norm, feat, blocks, q_fallback=0.0, return_fallback=True)
    np.testing.assert_allclose(M_all, oracle_mod.block_inverse(blocks), rtol=1e-9, atol=1e-12)
    M_none, fb_none, _ = mlp.minv(w, norm, feat, blocks, return_fallback=True)
    assert not fb_none.any()
    thr = float(np.median(q[3:]))
    M, fb, _ = mlp.minv(w, norm, feat, blocks, q_fallback=thr, return_fallback=True)
    assert np.array_equal(fb, (q > thr) & (np.arange(60) >= 3))
    np.testing.assert_array_equal(M[~fb], M_none[~fb])
    np.testing.assert_allclose(M[fb], M_all[fb], rtol=1e-12)
    # the error measure: the exact inverse scores 0
    Bn, _, live = mlp.normalised_block(blocks)
    Lx = np.linalg.cholesky(np.linalg.inv(Bn[live]))
    assert mlp.prediction_error(Lx, Bn[live]).max() < 1e-18


def test_coupling_inputs_are_the_normalised_off_diagonal(mlp):
    """Network inputs 6..8 are the block's colour-density coupling scaled to a unit diagonal, input 9
    the log of 1 / sqrt of the normalised block's Schur complement:
    for blocks built as e = rho sqrt(d f) u with a unit vector u, that is rho u up to the ridge
    (1e-6 max(d, f) added to d and f: at most 2.5e-5 relative here, d/f within 50); zero for units
    no ray touches, and the remaining input slots stay zero."""
    rng = np.random.default_rng(8)
    n = 50
    d = rng.uniform(0.1, 5.0, n)
    f = rng.uniform(0.1, 5.0, n)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rho = rng.uniform(0.0, 0.95, n)
    blocks = np.concatenate([d[:, None], u * (rho * np.sqrt(d * f))[:, None], f[:, None]], axis=1)
    blocks[:2] = 0.0
    x = mlp.inputs(unit_norm(mlp), rng.normal(size=(n, mlp.N_IN)), blocks)
    want = u * rho[:, None]
    np.testing.assert_allclose(x[2:, 6:9], want[2:], rtol=3e-5, atol=1e-12)
    assert np.all(np.linalg.norm(x[:, 6:9], axis=1) < 1.0)
    # input 9: -1/2 log of the Schur complement 1 - rho^2 of the normalised block (the ridge moves
    # |e~|^2 by at most 5e-5 relative, 1 - rho^2 >= 0.0975 here)
    np.testing.assert_allclose(x[2:, 9], -0.5 * np.log1p(-rho[2:] ** 2), rtol=0, atol=1e-3)
    assert np.all(x[:2, 6:10] == 0) and np.all(x[:, 10:] == 0)
    # the ridge keeps a singular block's complement near 2e-6 (input about 6.6); a block that
    # rounding left indefinite (|e~| > 1) takes the cap rather than the log of a negative number
    sing = np.array([[1.0, 1.0, 0.0, 0.0, 1.0], [1.0, 1.5, 0.0, 0.0, 1.0]])
    xs = mlp.inputs(unit_norm(mlp), np.zeros((2, mlp.N_IN)), sing)[:, 9]
    assert abs(xs[0] + 0.5 * np.log(1.0 - 1.0 / (1.0 + 1e-6) ** 2)) < 1e-6 and xs[1] == mlp.SCHUR_CAP
