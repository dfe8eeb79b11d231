"""The variants together: BF16 parameter storage with the auxiliary opacity residual (Eq. 10,
lambda = 0.1) and jittered sampling on, on the ragged-tile workload, against the oracle
evaluated at the bf16-rounded parameters (the oracle's own rounding) with the same lambda and
jitter seed.  FP32-level bars: residuals and F 1e-5, J v, J^T u, J^T J v, gradient and blocks
1e-4.
"""
import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def setup():
    import oracle
    from oracle import mlp
    from paper_2112_05598_amd.scene import Scene
    w = ps.workload("ragged")
    print(f"[variants] ragged {w.cams.n} cameras {w.cams.width}x{w.cams.height}: bf16, aux 0.1, jitter 9",
          flush=True)
    orc = oracle.OracleScene(w.spec, w.cams, aux_lambda=0.1, jitter_seed=9)
    rng = np.random.default_rng(91)
    targets = rng.uniform(0.0, 1.0, size=(w.cams.n_rays, 3)).astype(np.float32)
    x = rng.uniform(0.0, 1.0, size=(w.spec.n_units, 4)).astype(np.float32)
    x[:w.spec.n_vox, 3] *= 1.5
    x = x.reshape(-1)
    dev = torch.device("cuda:0")
    sc = Scene(w.spec, w.cams, torch.from_numpy(targets.reshape(-1)).to(dev), param_dtype="bf16", device="cuda:0",
               aux_lambda=0.1)
    sc.set_jitter(9)
    tb = sc.pack_bf16(torch.from_numpy(x).to(dev))
    xb = mlp.bf16_round(x).astype(np.float64)
    return sc, orc, tb, xb, targets, dev


def test_residuals(setup):
    sc, orc, tb, xb, targets, dev = setup
    r, F = sc.render_residuals(tb)
    _, r_or, F_or, _ = orc.render(xb, targets)
    assert sc.n_res == 4
    assert rel(r.cpu().numpy().reshape(-1, 4), r_or) <= 1e-5
    assert abs(F.item() - F_or) <= 1e-5 * F_or


def test_products(setup):
    sc, orc, tb, xb, targets, dev = setup
    v = ps.random_vector(sc.n_params, 41)
    u = ps.random_vector(4 * sc.n_rays, 42)
    tv = torch.from_numpy(v).to(dev)
    assert rel(sc.apply_J(tb, tv).cpu().numpy(), orc.apply_J(xb, v.astype(np.float64))) <= 1e-4
    assert rel(sc.apply_Jt(tb, torch.from_numpy(u).to(dev)).cpu().numpy(), orc.apply_Jt(xb, u.astype(np.float64))) <= 1e-4
    assert rel(sc.apply_JtJ(tb, tv).cpu().numpy(), orc.apply_JtJ(xb, v.astype(np.float64))) <= 1e-4


def test_gradient_and_blocks(setup):
    sc, orc, tb, xb, targets, dev = setup
    grad, blocks, _, F = sc.build_precond(tb, "jacobi")
    g_or, b_or, F_or = orc.grad_blocks(xb, targets)
    assert rel(grad.cpu().numpy(), g_or) <= 1e-4
    assert rel(blocks.cpu().numpy(), b_or) <= 1e-4
    assert abs(F.item() - F_or) <= 1e-5 * F_or
