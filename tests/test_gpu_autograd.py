"""render_residuals as a torch.autograd.Function: its J^T backward against central finite
differences of the GPU forward and against the FP64 oracle gradient, on the 16^3
re-rasterisation of the 360-degree scene (4 environment layers of 1024x512, 4 cameras 64x48)."""
import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def problem():
    import oracle
    from paper_2112_05598_amd.scene import Scene
    print("[case] autograd cfg5 16^3 copy", flush=True)
    full = ps.workload("cfg5", grid_n=16)
    cams = full.cams.subset(range(4)).with_image(64, 48, 60.0)
    w = ps.Workload("cfg5_16", full.spec, cams, full.x_gt, full.x_init, full.seed)
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(targets.reshape(-1)).to(dev)
    sc = Scene(w.spec, w.cams, t, device="cuda:0")
    rng = np.random.default_rng(5)
    x = w.x_init.copy().reshape(-1, 4)
    x[:w.spec.n_vox, 3] = rng.uniform(0.05, 0.6, w.spec.n_vox).astype(np.float32)
    x[:w.spec.n_vox, :3] = rng.uniform(0, 1, (w.spec.n_vox, 3)).astype(np.float32)
    x[w.spec.n_vox:, 3] = 0.3
    x = x.reshape(-1).astype(np.float32)
    # pick parameters from the oracle's own diagonal of J^T J: touched voxels, touched texels,
    # and untouched ones (whose gradient is exactly zero)
    _, blocks, _ = orc.grad_blocks(x.astype(np.float64), targets)
    touched = np.maximum(blocks[:, 0], blocks[:, 4]) > 0
    vox = np.nonzero(touched[:w.spec.n_vox])[0]
    tex = w.spec.n_vox + np.nonzero(touched[w.spec.n_vox:])[0]
    cold = np.nonzero(~touched)[0]
    units = np.concatenate([rng.choice(vox, 11, replace=False), rng.choice(tex, 4, replace=False),
                            rng.choice(cold, 1, replace=False)])
    params = (4 * units[:, None] + np.arange(4)[None, :]).reshape(-1)  # 64 parameters
    g = rng.normal(size=(sc.n_rays, 3)).astype(np.float32)
    return w, orc, sc, targets, x, params, g


def test_backward_is_Jt_and_matches_finite_differences(problem):
    from paper_2112_05598_amd.autograd import RenderResiduals
    w, orc, sc, targets, x, params, g = problem
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev).requires_grad_(True)
    gt = torch.from_numpy(g).to(dev)
    r = RenderResiduals.apply(xt, sc)
    assert r.shape == (sc.n_rays, 3)
    (r * gt).sum().backward()
    grad = xt.grad.cpu().numpy()

    def ell(xv):
        rr, _ = sc.render_residuals(torch.from_numpy(xv).to(dev))
        return float(np.dot(rr.cpu().numpy().astype(np.float64), g.reshape(-1).astype(np.float64)))

    eps = 1e-3
    fd = np.zeros(len(params))
    for i, p in enumerate(params):
        xp = x.copy(); xp[p] += eps
        xm = x.copy(); xm[p] -= eps
        fd[i] = (ell(xp) - ell(xm)) / (2 * eps)
    cold = params[-4:]
    assert np.all(grad[cold] == 0.0) and np.all(fd[-4:] == 0.0)
    err = np.linalg.norm(grad[params] - fd) / np.linalg.norm(fd)
    assert err <= 1e-3, err
    # against the FP64 oracle gradient J^T g over every parameter, one bound (the J^T product's)
    y_or = orc.apply_Jt(x.astype(np.float64), g.astype(np.float64))
    nv = 4 * w.spec.n_vox
    e_all = np.linalg.norm(grad - y_or) / np.linalg.norm(y_or)
    e_vox = np.linalg.norm(grad[:nv] - y_or[:nv]) / np.linalg.norm(y_or[:nv])
    e_tex = np.linalg.norm(grad[nv:] - y_or[nv:]) / np.linalg.norm(y_or[nv:])
    print(f"[autograd] J^T g vs oracle: all {e_all:.3e} (voxels {e_vox:.3e}, texels {e_tex:.3e}), FD {err:.3e}",
          flush=True)
    assert e_all <= 1e-4, e_all
    assert e_vox <= 1e-4 and e_tex <= 1e-4, (e_vox, e_tex)
