"""Pins of the FP64 learned-preconditioner reference (CPU only)."""
import numpy as np
import pytest

import perf_synth as ps


@pytest.fixture(scope="module")
def mlp(oracle_mod):
    from oracle import mlp
    return mlp


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
    L = mlp.factor(mlp.forward(w, feat)[0])
    Bn, _, live = mlp.normalised_block(blocks)
    E = L @ np.transpose(L, (0, 2, 1)) @ (Bn + damp * np.eye(4)) - np.eye(4)
    q = (E * E).sum(axis=(1, 2))
    q[~live] = 0.0
    return q


@pytest.mark.parametrize("damp", [0.0, 0.3])
def test_loss_gradient_matches_finite_differences(mlp, damp):
    rng = np.random.default_rng(0)
    w = mlp.init_weights(1) + 0.05 * rng.normal(size=mlp.NW)
    feat = rng.normal(size=(40, 12))
    blocks = random_blocks(40, 2)
    q = unit_errors(mlp, w, feat, blocks, damp)
    # both branches of the robust loss are exercised
    assert np.any(q > mlp.KAPPA) and np.any((q > 0) & (q < mlp.KAPPA))
    loss, g = mlp.loss_and_grad(w, feat, blocks, damp)
    expect = np.where(q > mlp.KAPPA, 4.0 * np.sqrt(q) - 4.0, q).sum() / 40
    assert abs(loss - expect) <= 1e-12 * expect
    idx = rng.choice(mlp.NW, 60, replace=False)
    eps = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd = (mlp.loss_and_grad(wp, feat, blocks, damp)[0] - mlp.loss_and_grad(wm, feat, blocks, damp)[0]) / (2 * eps)
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
        loss, g = mlp.loss_and_grad(mlp.pack(p), np.zeros((1, 12)), blocks[u:u + 1], damp)
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
    feat = np.random.default_rng(1).normal(size=(20, 12))
    M = mlp.minv(w, feat, blocks)
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


def test_feature_sums_identities(oracle_mod):
    """Sum over units of the weight channel = samples + layers hit (weights of a lookup sum
    to 1); of the transmittance channel = sum over rays of T at every sample and layer."""
    w = ps.workload("tiny")
    sc = oracle_mod.OracleScene(w.spec, w.cams)
    x = w.x_gt.astype(np.float64)
    sums = sc.feature_sums(x)
    U, L, K = sc.footprint()
    assert abs(sums[:, 0].sum() - (K.sum() + L.sum())) < 1e-9 * (K.sum() + L.sum())
    totT = 0.0
    for ray in range(sc.n_rays):
        s = sc.ray_samples(x, ray)
        totT += s["T"].sum()
    # layer transmittances: T in front of each used layer
    H, _, _, Te = sc.render(x)
    assert sums[:, 1].sum() >= totT - 1e-9
    assert np.all(sums[:, 0] >= 0) and np.all(sums[:, 1] <= sums[:, 0] + 1e-12)


def test_inverse_beyond_fp32_is_empty(mlp):
    """A unit whose learned inverse would exceed the FP32 range (subnormal diagonals) is taken as
    empty, as for the exact inverses; a unit with small but normal diagonals is kept."""
    w = mlp.init_weights(5)
    blocks = random_blocks(6, 8)
    blocks[3] = [1e-41, 0.0, 0.0, 0.0, 2e-41]   # D^-1/2 ~ 1e20: entries ~ 1e40
    blocks[4] = [1e-30, 0.0, 0.0, 0.0, 1e-30]   # entries ~ 1e30: in range
    feat = np.random.default_rng(2).normal(size=(6, 12))
    M = mlp.minv(w, feat, blocks)
    assert np.all(M[3] == 0)
    assert np.all(np.isfinite(M)) and np.abs(M).max() <= np.finfo(np.float32).max
    assert np.abs(M[4]).max() > 1e28
