"""Degenerate ray geometry against the FP64 oracle.

* every ray misses the grid and sees only environment layers (cameras outside the box,
  looking away from it, inside the layer spheres);
* a camera inside the grid box (the slab test's entry clipped to t = 0);
* rays exactly along an axis (zero direction components: IEEE infinities in the slab test);
* 1x1 images (one pixel per camera, a single lane of a 16x8 tile).

Same bars as the parity tests: residuals and F 1e-5, J v, J^T J v, gradient and blocks 1e-4
(norm-wise relative).
"""
import math

import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cams_looking(origins, forwards, width, height, fov_deg=60.0):
    """Pinhole cameras at the origins looking along the given forward directions."""
    rots = []
    for f in forwards:
        f = np.asarray(f, dtype=np.float64)
        f = f / np.linalg.norm(f)
        up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
        right = np.cross(f, up)
        right /= np.linalg.norm(right)
        down = np.cross(f, right)
        rots.append(np.stack([right, down, f], axis=1))
    n = len(rots)
    fpx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return ps.Cameras(np.asarray(origins, dtype=np.float64).reshape(-1, 3), np.stack(rots), np.full(n, fpx),
                      np.full(n, fpx), np.full(n, width / 2.0), np.full(n, height / 2.0), width, height)


SPEC = ps.SceneSpec(12, 10, 8, layer_radii=(1.8, 3.0), env_w=32, env_h=16, background=(0.1, 0.2, 0.3))

CASES = {
    "all rays miss the grid": cams_looking([(0.0, 0.0, 1.5), (1.5, 0.2, 0.0)], [(0, 0, 1), (1, 0.1, 0)], 9, 7),
    "camera inside the box": cams_looking([(0.2, -0.1, 0.3), (-0.5, 0.4, -0.2)], [(1, 0.2, 0.1), (0.1, -1, 0.3)],
                                          9, 7),
    "axis-aligned central rays": ps.cameras_from_origins([(0.0, 0.0, 3.0), (3.0, 0.0, 0.0), (0.0, -3.0, 0.0)],
                                                         9, 7, 40.0),
    "one-pixel images": ps.cameras_from_origins([(2.0, 1.0, 2.0), (-2.5, 0.5, 1.0), (0.3, -2.8, 0.9)], 1, 1, 40.0),
}


@pytest.fixture(scope="module", params=list(CASES), ids=lambda k: k.replace(" ", "-"))
def case(request):
    import oracle
    from paper_2112_05598_amd.scene import Scene
    cams = CASES[request.param]
    print(f"[degenerate] {request.param}: {cams.n} cameras {cams.width}x{cams.height}", flush=True)
    rng = np.random.default_rng(77)
    x = rng.uniform(0.0, 1.0, size=(SPEC.n_units, 4)).astype(np.float32)
    x[:SPEC.n_vox, 3] *= 1.5
    x = x.reshape(-1)
    targets = rng.uniform(0.0, 1.0, size=(cams.n_rays, 3)).astype(np.float32)
    dev = torch.device("cuda:0")
    sc = Scene(SPEC, cams, torch.from_numpy(targets.reshape(-1)).to(dev), device="cuda:0")
    orc = oracle.OracleScene(SPEC, cams)
    return dict(name=request.param, sc=sc, orc=orc, x=x, x64=x.astype(np.float64), tx=torch.from_numpy(x).to(dev),
                targets=targets, dev=dev)


def test_render(case):
    r, F = case["sc"].render_residuals(case["tx"])
    _, r_or, F_or, _ = case["orc"].render(case["x64"], case["targets"])
    assert rel(r.cpu().numpy(), r_or) <= 1e-5
    assert abs(F.item() - F_or) <= 1e-5 * F_or


def test_products(case):
    sc, orc = case["sc"], case["orc"]
    v = ps.random_vector(sc.n_params, 11)
    tv = torch.from_numpy(v).to(case["dev"])
    u_or = orc.apply_J(case["x64"], v.astype(np.float64))
    y_or = orc.apply_JtJ(case["x64"], v.astype(np.float64))
    if np.linalg.norm(u_or) == 0:  # nothing depends on the parameters for these rays
        assert np.all(sc.apply_J(case["tx"], tv).cpu().numpy() == 0)
        assert np.all(sc.apply_JtJ(case["tx"], tv).cpu().numpy() == 0)
        return
    assert rel(sc.apply_J(case["tx"], tv).cpu().numpy(), u_or) <= 1e-4
    assert rel(sc.apply_JtJ(case["tx"], tv).cpu().numpy(), y_or) <= 1e-4


def test_gradient_and_blocks(case):
    grad, blocks, _, F = case["sc"].build_precond(case["tx"], "jacobi")
    g_or, b_or, F_or = case["orc"].grad_blocks(case["x64"], case["targets"])
    assert rel(grad.cpu().numpy(), g_or) <= 1e-4
    assert rel(blocks.cpu().numpy(), b_or) <= 1e-4
    assert abs(F.item() - F_or) <= 1e-5 * F_or


def test_geometry_is_what_the_case_says(case):
    """The footprint pass confirms the degenerate geometry (no voxel touched when all rays miss)."""
    per_ray, tot = case["sc"].footprint()
    tot = tot.cpu().numpy()
    if case["name"] == "all rays miss the grid":
        assert tot[0] == 0 and tot[1] > 0
    else:
        assert tot[0] > 0
