"""Preconditioner inverses of given blocks (perf_invert_blocks) against the oracle, Sec. III-G.

Blocks [[d I3, e], [e^T, f]] drawn as SPD arrowheads over many scales, with empty units, units
with one zero diagonal, and diagonals in the FP32 subnormal range, whose exact inverses lie far
beyond the FP32 range: the library's scaled form (D^-1/2 and a normalised inverse) holds them
all, and multiplied out in FP64 it matches the oracle's exact inverse.  Jacobi entries: two FP32
roundings of t = D^-1/2; block inverses: 1e-6 relative per unit (FP64 arithmetic, FP32 storage
of order-one normalised entries).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def crafted_blocks(n=5000, seed=31):
    rng = np.random.default_rng(seed)
    scale = 10.0 ** rng.uniform(-30, 6, n)
    d = rng.uniform(0.5, 2.0, n)
    e = rng.normal(size=(n, 3)) * 0.3
    f = (e * e).sum(1) / d + rng.uniform(0.05, 1.0, n)
    b = np.stack([d, e[:, 0], e[:, 1], e[:, 2], f], axis=1) * scale[:, None]
    b[:50] = 0.0                                  # empty units
    b[50:80, 0] = 0.0                              # no colour partials
    b[50:80, 1:4] = 0.0
    b[80:110, 4] = 0.0                             # no opacity partial
    b[80:110, 1:4] = 0.0
    b[110:140] *= 1e-40 / scale[110:140, None]     # subnormal diagonals
    b[140:170, 0] = 1e-40                          # subnormal d beside a normal f
    b[140:170, 1:4] = 0.0
    return b.astype(np.float32)


def test_invert_blocks_matches_oracle():
    import oracle
    from gpu_checks import block_minv, jacobi_minv
    from paper_2112_05598_amd.scene import invert_blocks
    b = crafted_blocks()
    print(f"[invert] {b.shape[0]} crafted blocks", flush=True)
    tb = torch.from_numpy(b).to("cuda:0")
    jac = invert_blocks(tb, "jacobi").cpu().numpy()
    blk = invert_blocks(tb, "block").cpu().numpy()
    assert np.all(np.isfinite(jac)) and np.all(np.isfinite(blk))
    b64 = b.astype(np.float64)
    jac_or = oracle.jacobi_inverse(b64)
    mj = jacobi_minv(jac)
    assert np.all((mj == 0) == (jac_or == 0))
    np.testing.assert_allclose(mj, jac_or, rtol=3e-7, atol=0)
    assert jac_or[4 * 110:4 * 140].min() > 1e38  # far beyond FP32, held by the scaled form
    binv = oracle.block_inverse(b64)
    got = block_minv(blk)
    empty = np.all(binv == 0, axis=(1, 2))
    assert np.all(np.all(blk == 0, axis=1) == empty)
    assert empty[:50].all() and not empty[50:].any()
    live = ~empty
    err = np.linalg.norm(got[live] - binv[live], axis=(1, 2)) / np.linalg.norm(binv[live], axis=(1, 2))
    print(f"[invert] block max per-unit error {err.max():.3e}", flush=True)
    assert err.max() <= 1e-6, err.max()


def test_invert_blocks_rejects_bad_arguments():
    import ctypes
    from paper_2112_05598_amd import abi
    lib = abi.load()
    assert lib.perf_invert_blocks(None, 4, abi.PERF_PRECOND_JACOBI, None, None) == abi.PERF_EINVAL
    tb = torch.zeros(4, 5, device="cuda:0")
    out = torch.zeros(4, 4, device="cuda:0")
    assert lib.perf_invert_blocks(ctypes.c_void_p(tb.data_ptr()), 4, abi.PERF_PRECOND_NONE,
                                  ctypes.c_void_p(out.data_ptr()), None) == abi.PERF_EINVAL
    assert lib.perf_invert_blocks(ctypes.c_void_p(tb.data_ptr()), -1, abi.PERF_PRECOND_JACOBI,
                                  ctypes.c_void_p(out.data_ptr()), None) == abi.PERF_EINVAL
    assert lib.perf_invert_blocks(None, 0, abi.PERF_PRECOND_JACOBI, None, None) == abi.PERF_OK
