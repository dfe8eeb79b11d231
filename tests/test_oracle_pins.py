"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Closed forms of the rendering sum (Sec. III-A, Eq. 3-4), the derivative of that
sum by central finite differences (Sec. III-E), brute-force dense J^T J for the
matrix-free identity (Eq. 9) and the Jacobi diagonal (Sec. III-G), textbook
conjugate gradients for Alg. 2, and scripted objectives for Alg. 3.
"""
import dataclasses
import math

import numpy as np
import pytest

import perf_synth as ps


# ----------------------------------------------------------------------------- helpers

def axis_scene(n=8, step=0.5, W=5, H=5, fov=20.0, radii=(1.8,), env=(16, 8), bg=(0.0, 0.0, 0.0)):
    spec = ps.SceneSpec(n, n, n, layer_radii=radii, env_w=env[0], env_h=env[1], step_vox=step, background=bg)
    cams = ps.cameras_from_origins([[3.0, 0.0, 0.0]], W, H, fov)
    return spec, cams


def params(spec, grid_rgbs, env_rgba):
    grid = np.zeros((spec.nz, spec.ny, spec.nx, 4))
    grid[...] = grid_rgbs
    env = np.zeros((spec.n_layers, spec.env_h, spec.env_w, 4))
    env[...] = env_rgba
    return pack64(grid, env)


def pack64(grid, env):
    return np.concatenate([np.asarray(grid, np.float64).reshape(-1), np.asarray(env, np.float64).reshape(-1)])


def random_x(spec, seed, sigma_max=2.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(spec.n_units, 4))
    x[:spec.n_vox, 3] *= sigma_max
    return x.reshape(-1)


def dense_jacobian_fd(sc, x, rays, eps=1e-6):
    """Central differences of H (3 per ray) with respect to every parameter."""
    P = sc.n_params
    J = np.zeros((3 * len(rays), P))
    for j in range(P):
        xp = x.copy(); xp[j] += eps
        xm = x.copy(); xm[j] -= eps
        Hp = sc.render(xp, rays=rays)[0].reshape(-1)
        Hm = sc.render(xm, rays=rays)[0].reshape(-1)
        J[:, j] = (Hp - Hm) / (2 * eps)
    return J


def dense_jacobian_rows(sc, x, rays, mode=0):
    P = sc.n_params
    J = np.zeros((3 * len(rays), P))
    for i, ray in enumerate(rays):
        unit, a, s, _ = sc.ray_row(x, ray, mode)
        for u, aa, ss in zip(unit, a, s):
            for ch in range(3):
                J[3 * i + ch, 4 * u + ch] += aa
                J[3 * i + ch, 4 * u + 3] += ss[ch]
    return J


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    w = ps.workload("tiny")
    spec = dataclasses.replace(w.spec, background=(0.2, 0.3, 0.1))
    sc = oracle_mod.OracleScene(spec, w.cams)
    x = random_x(spec, 5)
    rng = np.random.default_rng(3)
    U, L, K = sc.footprint()
    hit = np.nonzero(K > 0)[0]
    miss = np.nonzero(K == 0)[0]
    rays = np.concatenate([rng.choice(hit, 28, replace=False), miss[:4]]).astype(np.int64)
    return sc, spec, x, rays


@pytest.fixture(scope="module")
def tiny_fd(tiny):
    sc, spec, x, rays = tiny
    return dense_jacobian_fd(sc, x, rays)


# ----------------------------------------------------------------------------- cameras

def test_principal_ray_hits_origin(oracle_mod):
    w = ps.workload("tiny")  # 13 x 11: the centre pixel sits on the principal point
    sc = oracle_mod.OracleScene(w.spec, w.cams)
    for cam in range(w.cams.n):
        ray = cam * 13 * 11 + 5 * 13 + 6
        o, d = sc.ray(ray)
        np.testing.assert_allclose(d, -o / np.linalg.norm(o), atol=1e-14)


def test_pinhole_angles(oracle_mod):
    spec, cams = axis_scene(W=9, H=9, fov=40.0)
    sc = oracle_mod.OracleScene(spec, cams)
    f = cams.fx[0]
    _, d0 = sc.ray(4 * 9 + 4)
    for k in (1, 2, 4):
        _, d1 = sc.ray(4 * 9 + 4 + k)   # k pixels to the right
        _, d2 = sc.ray((4 + k) * 9 + 4)  # k pixels down
        assert math.isclose(math.acos(np.clip(d0 @ d1, -1, 1)), math.atan(k / f), rel_tol=1e-9)
        assert math.isclose(math.acos(np.clip(d0 @ d2, -1, 1)), math.atan(k / f), rel_tol=1e-9)
        # right is +y and down is -z for a camera on +x looking at the origin
        assert d1[1] > 0 and abs(d1[2]) < 1e-14
        assert d2[2] < 0 and abs(d2[1]) < 1e-14
    R = cams.rot[0]
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-14)


# ----------------------------------------------------------------------------- closed forms of Eq. 3-4

def test_trilinear_reproduces_affine_field(oracle_mod):
    spec, cams = axis_scene(n=8)
    sc = oracle_mod.OracleScene(spec, cams)
    h = 2.0 / 8
    idx = np.arange(8)
    cz, cy, cx = np.meshgrid(idx, idx, idx, indexing="ij")
    centre = lambda i: -1.0 + (i + 0.5) * h
    field = 0.3 * centre(cx) - 0.7 * centre(cy) + 1.1 * centre(cz) + 0.25
    grid = np.zeros((8, 8, 8, 4)); grid[..., 3] = field; grid[..., 0] = 2.0
    x = pack64(grid, np.zeros((1, 8, 16, 4)))
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = rng.uniform(-1 + h / 2, 1 - h / 2, size=3)  # interior: every corner is a real neighbour
        exp = 0.3 * p[0] - 0.7 * p[1] + 1.1 * p[2] + 0.25
        assert math.isclose(sc.sample_field(x, p, 3), exp, rel_tol=1e-12, abs_tol=1e-12)
        assert math.isclose(sc.sample_field(x, rng.uniform(-1, 1, 3), 0), 2.0, rel_tol=1e-14)


@pytest.mark.parametrize("step", [0.5, 0.3, 0.7, 1.0])
def test_uniform_grid_closed_form(oracle_mod, step):
    """sigma = s0, c = c0 everywhere, one opaque constant layer E:
    H = c0 (1 - e^{-s0 L}) + e^{-s0 L} E, with L the chord in voxel lengths."""
    n = 8
    spec, cams = axis_scene(n=n, step=step, W=5, H=5, fov=10.0)
    sc = oracle_mod.OracleScene(spec, cams)
    s0, c0, E = 0.37, np.array([0.2, 0.5, 0.9]), np.array([0.6, 0.1, 0.3])
    x = params(spec, np.r_[c0, s0], np.r_[E, 1.0])
    H = sc.render(x)[0]
    for ray in range(25):
        py, px = divmod(ray, 5)
        # ray direction in the camera frame (right=+y, down=-z, forward=-x)
        dc = np.array([(px + 0.5 - 2.5) / cams.fx[0], (py + 0.5 - 2.5) / cams.fy[0], 1.0])
        norm = np.linalg.norm(dc)
        # from (3,0,0) the ray crosses x = +1 and x = -1 inside the box for this narrow FOV
        chord_world = 2.0 * norm  # x drops by 2 while t grows by 2 * |dc| / dc_z
        L = chord_world / (2.0 / n)
        T = math.exp(-s0 * L)
        np.testing.assert_allclose(H[ray], c0 * (1 - T) + T * E, rtol=1e-12)


def test_empty_grid_returns_env_colour(oracle_mod):
    """sigma = 0 everywhere and one opaque layer whose colour is linear in the
    texel row: H equals that linear function at the exit direction's polar angle."""
    spec, cams = axis_scene(n=4, W=7, H=7, fov=40.0, env=(32, 16))
    sc = oracle_mod.OracleScene(spec, cams)
    env = np.zeros((1, 16, 32, 4))
    rows = np.arange(16)[:, None]
    env[0, :, :, 0] = 0.1 + 0.05 * rows
    env[0, :, :, 1] = 0.9 - 0.03 * rows
    env[0, :, :, 2] = 0.5
    env[0, :, :, 3] = 1.0
    grid = np.zeros((4, 4, 4, 4)); grid[..., 0:3] = 0.7
    x = pack64(grid, env)
    H = sc.render(x)[0]
    for ray in range(49):
        o, d = sc.ray(ray)
        # far intersection with the layer sphere (radius 1.8 in single precision) by polynomial roots
        R = spec.layer_radii[0]
        t = max(np.roots([d @ d, 2 * o @ d, o @ o - R ** 2]).real)
        q = (o + t * d) / R
        v = math.acos(q[2]) / math.pi * 16 - 0.5
        assert 0.0 <= v <= 15.0
        np.testing.assert_allclose(H[ray], [0.1 + 0.05 * v, 0.9 - 0.03 * v, 0.5], rtol=1e-12)


def test_env_azimuth_linear(oracle_mod):
    """A layer whose colour is linear in the texel column maps azimuth linearly."""
    spec, cams = axis_scene(n=4, W=7, H=7, fov=40.0, env=(64, 8))
    sc = oracle_mod.OracleScene(spec, cams)
    env = np.zeros((1, 8, 64, 4))
    env[0, :, :, 0] = 0.01 * np.arange(64)[None, :]
    env[0, :, :, 3] = 1.0
    x = pack64(np.zeros((4, 4, 4, 4)), env)
    H = sc.render(x)[0]
    for ray in range(49):
        o, d = sc.ray(ray)
        R = spec.layer_radii[0]
        t = max(np.roots([d @ d, 2 * o @ d, o @ o - R ** 2]).real)
        q = (o + t * d) / R
        u = (math.atan2(q[1], q[0]) / (2 * math.pi) + 0.5) * 64 - 0.5
        if 0.0 <= u <= 63.0:  # away from the wrap seam
            assert math.isclose(H[ray][0], 0.01 * u, rel_tol=1e-11)


def test_one_voxel_by_hand(oracle_mod):
    """A single voxel (index 3 along x) with sigma_j, c_j; a ray along -x through its centre
    line samples it at offsets -0.75, -0.25, 0.25, 0.75 voxel with weights 1/4, 3/4, 3/4, 1/4."""
    n = 8
    spec, cams = axis_scene(n=n, W=1, H=1, fov=10.0, bg=(0.0, 0.0, 0.0))
    # shift the camera so the principal ray runs along the centre line of voxel row (y=3, z=4)
    h = 2.0 / n
    yc, zc = -1 + 3.5 * h, -1 + 4.5 * h
    cams.origin[0] = [3.0, yc, zc]
    cams.rot[0] = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    sc = oracle_mod.OracleScene(spec, cams)
    sig, col = 1.7, np.array([0.3, 0.6, 0.8])
    grid = np.zeros((n, n, n, 4))
    grid[4, 3, 4, 0:3] = col
    grid[4, 3, 4, 3] = sig
    x = pack64(grid, np.zeros((1, 8, 16, 4)))
    H = sc.render(x)[0][0]
    # the ray travels -x: voxel x-index 4 is the 4th voxel from the entry face (x = +1)
    w = [0.25, 0.75, 0.75, 0.25]
    T, exp_H = 1.0, np.zeros(3)
    for wk in w:
        a = 1 - math.exp(-sig * wk * 0.5)
        exp_H += T * a * (col * wk)
        T *= math.exp(-sig * wk * 0.5)
    np.testing.assert_allclose(H, exp_H, rtol=1e-12)


def test_partition_of_unity(oracle_mod):
    """All colours 1 and background 1: H = sum T_k alpha_k + sum T_l alpha_l + T_end = 1."""
    w = ps.workload("ragged")
    spec = dataclasses.replace(w.spec, background=(1.0, 1.0, 1.0))
    sc = oracle_mod.OracleScene(spec, w.cams)
    x = random_x(spec, 7, sigma_max=3.0).reshape(-1, 4)
    x[:, 0:3] = 1.0
    H = sc.render(x.reshape(-1))[0]
    np.testing.assert_allclose(H, 1.0, atol=1e-12)


def pinhole_chord(spec, cams, ray):
    """Chord of a pixel ray through the grid box in shortest-voxel-side units, from the pinhole
    model and a slab test written out here (0 for a miss)."""
    per = cams.width * cams.height
    cam, pix = divmod(int(ray), per)
    py, px = divmod(pix, cams.width)
    dc = np.array([(px + 0.5 - cams.cx[cam]) / cams.fx[cam], (py + 0.5 - cams.cy[cam]) / cams.fy[cam], 1.0])
    d = np.asarray(cams.rot[cam]).reshape(3, 3) @ dc
    d /= np.linalg.norm(d)
    o = np.asarray(cams.origin[cam], dtype=np.float64)
    lo, hi = np.asarray(spec.bbox_min), np.asarray(spec.bbox_max)
    with np.errstate(divide="ignore"):
        ta, tb = (lo - o) / d, (hi - o) / d
    t0 = max(np.max(np.minimum(ta, tb)), 0.0)
    t1 = np.min(np.maximum(ta, tb))
    h = min((hi[a] - lo[a]) / n for a, n in enumerate((spec.nx, spec.ny, spec.nz)))
    return max(t1 - t0, 0.0) / h


def test_transmittance_bounds(oracle_mod, tiny):
    sc, spec, x, rays = tiny
    for ray in rays[:10]:
        s = sc.ray_samples(x, ray)
        T = np.r_[s["T"], s["T_end"]]
        assert np.all(T <= 1.0) and np.all(T >= 0.0)
        assert np.all(np.diff(T) <= 1e-15)
        if len(s["T"]):
            assert s["T"][0] == 1.0
            # the steps add up to the chord (the last one shortened)
            L = pinhole_chord(spec, sc.cams, ray)
            assert abs(s["delta"].sum() - L) <= 1e-12 * max(L, 1.0), (s["delta"].sum(), L)
            assert len(s["delta"]) == int(np.ceil(L / spec.step_vox - 1e-12))
            assert np.all(s["delta"] <= spec.step_vox + 1e-15) and np.all(s["delta"] > 0)


def test_chord_pin_on_non_unit_steps(oracle_mod):
    """Steps of 0.3 voxel on a non-cubic box: K = ceil(L / step) samples whose steps sum to L."""
    w = ps.workload("small")
    spec = dataclasses.replace(w.spec, step_vox=0.3)
    sc = oracle_mod.OracleScene(spec, w.cams)
    _, _, K = sc.footprint()
    hit = np.nonzero(K > 0)[0]
    x = random_x(spec, 2)
    for ray in hit[:: max(len(hit) // 12, 1)]:
        s = sc.ray_samples(x, ray)
        L = pinhole_chord(spec, w.cams, ray)
        assert abs(s["delta"].sum() - L) <= 1e-12 * max(L, 1.0)
        assert len(s["delta"]) == K[ray]


def test_axis_ray_footprint(oracle_mod):
    """Along a grid row through voxel centres every voxel of the row and its
    +y/+z neighbours is a trilinear corner: U = 4 N."""
    n = 8
    spec, cams = axis_scene(n=n, W=1, H=1)
    h = 2.0 / n
    cams.origin[0] = [3.0, -1 + 2.5 * h, -1 + 5.5 * h]
    cams.rot[0] = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    sc = oracle_mod.OracleScene(spec, cams)
    U, L, K = sc.footprint()
    assert U[0] == 4 * n and L[0] == 1 and K[0] == 2 * n


# ----------------------------------------------------------------------------- derivatives (Sec. III-E)

def test_rows_match_finite_differences(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    J = dense_jacobian_rows(sc, x, rays)
    err = np.abs(J - tiny_fd).max() / np.abs(tiny_fd).max()
    assert err < 1e-8, err


def test_alg1_matches_explicit_partials(tiny):
    sc, spec, x, rays = tiny
    for ray in rays:
        a = sc.ray_samples(x, ray, mode=0)
        b = sc.ray_samples(x, ray, mode=1)
        np.testing.assert_allclose(b["dHdc"], a["dHdc"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(b["dHds"], a["dHds"], rtol=1e-10, atol=1e-13)


def test_alg1_without_env_term_is_not_the_derivative(tiny, tiny_fd):
    """Alg. 1 as printed starts its colour accumulator at zero; with a visible
    environment that drops a term of dH/dsigma, which finite differences expose."""
    sc, spec, x, rays = tiny
    J2 = dense_jacobian_rows(sc, x, rays, mode=2)
    err = np.abs(J2 - tiny_fd).max() / np.abs(tiny_fd).max()
    assert err > 1e-3


def test_apply_J_matches_dense(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    v = np.random.default_rng(1).normal(size=sc.n_params)
    u = sc.apply_J(x, v, rays=rays).reshape(-1)
    ref = tiny_fd @ v
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-8


def test_apply_Jt_matches_dense(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    u = np.random.default_rng(2).normal(size=3 * len(rays))
    y = sc.apply_Jt(x, u, rays=rays)
    ref = tiny_fd.T @ u
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-8


def test_adjoint_identity(tiny):
    sc, spec, x, rays = tiny
    rng = np.random.default_rng(4)
    v = rng.normal(size=sc.n_params)
    u = rng.normal(size=3 * len(rays))
    Jv = sc.apply_J(x, v, rays=rays).reshape(-1)
    Jtu = sc.apply_Jt(x, u, rays=rays)
    assert abs(u @ Jv - Jtu @ v) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Jv) * 10


def test_JtJ_matches_dense(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    v = np.random.default_rng(5).normal(size=sc.n_params)
    y = sc.apply_JtJ(x, v, rays=rays)
    ref = tiny_fd.T @ (tiny_fd @ v)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-8
    w = np.random.default_rng(6).normal(size=sc.n_params)
    Jv = sc.apply_J(x, v, rays=rays).reshape(-1)
    Jw = sc.apply_J(x, w, rays=rays).reshape(-1)
    assert math.isclose(w @ y, Jw @ Jv, rel_tol=1e-10)
    assert v @ y >= 0


def test_blocks_match_dense_JtJ(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    targets = np.zeros((sc.n_rays, 3), np.float32)
    grad, blocks, F = sc.grad_blocks(x, targets, rays=rays)
    A = tiny_fd.T @ tiny_fd
    scale = np.abs(A).max()
    for unit in range(sc.n_units):
        Bd = A[4 * unit:4 * unit + 4, 4 * unit:4 * unit + 4]
        b = blocks[unit]
        exp = np.array([[b[0], 0, 0, b[1]], [0, b[0], 0, b[2]], [0, 0, b[0], b[3]], [b[1], b[2], b[3], b[4]]])
        assert np.abs(Bd - exp).max() <= 1e-8 * scale
    diag = np.diag(A)
    np.testing.assert_allclose(_oracle().jacobi_diag(blocks), diag, atol=1e-8 * scale)


def _oracle():
    import oracle
    return oracle


def test_gradient_matches_fd_of_objective(tiny, tiny_fd):
    sc, spec, x, rays = tiny
    rng = np.random.default_rng(8)
    targets = rng.uniform(0, 1, size=(sc.n_rays, 3)).astype(np.float32)
    grad, blocks, F = sc.grad_blocks(x, targets, rays=rays)
    H = sc.render(x, rays=rays)[0]
    r = (H - targets[rays].astype(np.float64)).reshape(-1)
    assert math.isclose(F, 0.5 * r @ r, rel_tol=1e-12)
    ref = -(tiny_fd.T @ r)
    assert np.linalg.norm(grad - ref) / np.linalg.norm(ref) < 1e-8
    # and directly: central differences of F along a random direction
    v = rng.normal(size=sc.n_params)
    eps = 1e-6
    Fp = sc.render(x + eps * v, targets, rays=rays)[2]
    Fm = sc.render(x - eps * v, targets, rays=rays)[2]
    assert math.isclose((Fp - Fm) / (2 * eps), -(grad @ v), rel_tol=1e-6)


# ----------------------------------------------------------------------------- preconditioner inverse

def test_block_inverse_is_inverse(oracle_mod):
    rng = np.random.default_rng(9)
    n = 200
    e = rng.normal(size=(n, 3))
    d = rng.uniform(0.5, 2.0, n)
    f = (e * e).sum(1) / d + rng.uniform(0.1, 1.0, n)  # SPD: f > e.e / d
    blocks = np.stack([d, e[:, 0], e[:, 1], e[:, 2], f], axis=1)
    blocks[:5] = 0.0  # empty units
    Binv = oracle_mod.block_inverse(blocks, ridge=0.0)
    B = oracle_mod.block_matrix(blocks)
    for i in range(5, n):
        np.testing.assert_allclose(B[i] @ Binv[i], np.eye(4), atol=1e-10)
    assert np.all(Binv[:5] == 0)
    jac = oracle_mod.jacobi_inverse(blocks)
    assert np.all(jac[:20] == 0)
    np.testing.assert_allclose(jac[20:24], [1 / d[5]] * 3 + [1 / f[5]])


def test_inverses_of_tiny_diagonals_are_exact(oracle_mod):
    """The inverses are the exact ones at any scale (Sec. III-G: M = diag(J^T J)): a block scaled
    by s has its inverse scaled by 1/s, down to diagonals of 1e-44 (units seen only through
    near-opaque matter), with no threshold anywhere."""
    base = np.array([[2.0, 0.3, -0.2, 0.1, 1.5],
                     [1.0, 0.0, 0.0, 0.0, 4.0],
                     [0.7, 0.5, 0.1, -0.4, 0.9]])
    B = oracle_mod.block_matrix(base)
    for scale in (1.0, 1e-30, 1e-40, 1e-44):
        blocks = base * scale
        jac = oracle_mod.jacobi_inverse(blocks).reshape(-1, 4)
        np.testing.assert_allclose(jac[:, 0], 1.0 / (scale * base[:, 0]), rtol=1e-14)
        np.testing.assert_allclose(jac[:, 3], 1.0 / (scale * base[:, 4]), rtol=1e-14)
        binv = oracle_mod.block_inverse(blocks)
        for i in range(3):
            m = max(base[i, 0], base[i, 4])
            # (s (B + rho I)) (B + rho I)^-1 / s = I: the ridge scales with the block
            prod = scale * (B[i] + 1e-6 * m * np.eye(4)) @ binv[i]
            np.testing.assert_allclose(prod, np.eye(4), atol=1e-9)
    one_sided = np.array([[1e-40, 0.0, 0.0, 0.0, 2.0]])
    jac = oracle_mod.jacobi_inverse(one_sided)
    np.testing.assert_allclose(jac, [1e40, 1e40, 1e40, 0.5], rtol=1e-14)


# ----------------------------------------------------------------------------- Alg. 2

def _spd(n, rank, seed):
    rng = np.random.default_rng(seed)
    J = rng.normal(size=(max(rank, 1), n))
    return J.T @ J, rng.normal(size=n)


def test_pcg_solves_spd_system(oracle_mod):
    A, b = _spd(12, 30, 0)
    for minv in (np.ones(12), 1.0 / np.diag(A)):
        res = oracle_mod.pcg(lambda p: A @ p, b, lambda r: minv * r, max_iters=40, abs_eps=1e-28)
        np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)


def test_pcg_singular_gives_min_norm(oracle_mod):
    A, _ = _spd(12, 5, 1)
    b = A @ np.random.default_rng(2).normal(size=12)  # consistent right-hand side in range(A)
    res = oracle_mod.pcg(lambda p: A @ p, b, lambda r: r, max_iters=30, abs_eps=1e-26)
    np.testing.assert_allclose(res.x, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-6, atol=1e-8)


def test_pcg_direction_conjugacy(oracle_mod):
    A, b = _spd(10, 40, 3)
    dirs = []
    minv = 1.0 / np.diag(A)

    def rec(p):
        dirs.append(p.copy())
        return A @ p

    oracle_mod.pcg(rec, b, lambda r: minv * r, max_iters=6)
    for i in range(len(dirs)):
        for j in range(i):
            assert abs(dirs[i] @ A @ dirs[j]) <= 1e-9 * math.sqrt((dirs[i] @ A @ dirs[i]) * (dirs[j] @ A @ dirs[j]))


def test_pcg_stopping_rules(oracle_mod):
    A, b = _spd(30, 60, 4)
    res = oracle_mod.pcg(lambda p: A @ p, b, lambda r: r, max_iters=7)
    assert res.iters == 7 and len(res.alpha) == 7 and len(res.beta) == 6
    res = oracle_mod.pcg(lambda p: A @ p, b, lambda r: r, max_iters=100, rel_tol=1e-3)
    assert math.sqrt(res.R[-1] / res.R0) <= 1e-3 and math.sqrt(res.R[-2] / res.R0) > 1e-3
    res = oracle_mod.pcg(lambda p: -(A @ p), b, lambda r: r, max_iters=5)
    assert "breakdown" in res.flags and res.iters == 0 and np.all(res.x == 0)
    res = oracle_mod.pcg(lambda p: A @ p, np.zeros(30), lambda r: r, max_iters=5)
    assert "converged" in res.flags and res.iters == 0


# ----------------------------------------------------------------------------- Alg. 3

def test_line_search_scripted(oracle_mod):
    calls = []

    def quad(g):
        calls.append(g)
        return (g - 0.3) ** 2

    g, mu, n, capped = oracle_mod.line_search(quad, F0=1.0)
    # errors at 1, .7, .49, .343, .2401: the last is the first increase, so .343 comes back
    assert math.isclose(g, 0.343, rel_tol=1e-12) and n == 5 and not capped
    assert math.isclose(mu, (0.343 - 0.3) ** 2, rel_tol=1e-12)
    # never increasing: the cap ends it and the smallest error wins
    g, mu, n, capped = oracle_mod.line_search(lambda g: g, F0=10.0, ls_max=6)
    assert capped and n == 6 and math.isclose(g, 0.7 ** 5)
    # no trial beats the current error: no step
    g, mu, n, capped = oracle_mod.line_search(lambda g: 5.0 + (g - 0.5) ** 2, F0=1.0)
    assert g == 0.0 and mu == 1.0
    # ties keep shrinking (strict comparison)
    seq = iter([3.0, 3.0, 2.0, 2.5])
    g, mu, n, capped = oracle_mod.line_search(lambda g: next(seq), F0=4.0)
    assert math.isclose(g, 0.49) and mu == 2.0


# ----------------------------------------------------------------------------- Gauss-Newton (Eq. 7)

def _observed_problem(oracle_mod, n=4, seed=21):
    spec = ps.SceneSpec(n, n, n, layer_radii=(1.8,), env_w=8, env_h=4)
    rng = np.random.default_rng(seed)
    cams = ps.make_cameras("sphere", 12, 12, 12, 50.0, 3.0, rng)
    sc = oracle_mod.OracleScene(spec, cams)
    x_gt = random_x(spec, seed + 1, sigma_max=1.0)
    x_gt.reshape(-1, 4)[spec.n_vox:, 3] = 0.8
    targets = sc.render(x_gt)[0].astype(np.float32)
    return spec, sc, x_gt, targets


def test_zero_residual_fixed_point(oracle_mod):
    spec, sc, x_gt, targets = _observed_problem(oracle_mod)
    xg = x_gt.astype(np.float32).astype(np.float64)
    out = oracle_mod.gn_step(sc, xg, sc.render(xg)[0].astype(np.float32).astype(np.float64), max_iters=5)
    # targets equal to the render up to float32 rounding: tiny gradient and a tiny step
    assert out["F_before"] < 1e-12
    assert np.abs(out["x"] - xg).max() < 1e-5


def test_gauss_newton_converges_near_ground_truth(oracle_mod):
    spec, sc, x_gt, targets = _observed_problem(oracle_mod)
    rng = np.random.default_rng(0)
    x = x_gt + 0.02 * rng.normal(size=x_gt.size)
    x = oracle_mod.project(spec, x)
    Fs = []
    for _ in range(4):
        out = oracle_mod.gn_step(sc, x, targets, precond="jacobi", max_iters=200, rel_tol=1e-10)
        Fs.append(out["F_before"])
        assert out["F_after"] <= out["F_before"]
        x = out["x"]
    Fs.append(sc.render(x, targets)[2])
    assert Fs[-1] < 1e-6 * Fs[0], Fs


def test_learned_gn_step_falls_back_to_the_block_solve(oracle_mod):
    """The learned GN step's failure rule (a reading of this library, not the paper): a learned
    solve that stalls is replaced by the exact block-Jacobi solve from Delta_0 = 0, so the step
    then equals the block step; without a failure the learned solve stands.  The learned M^-1
    here is the exact block inverse scaled by 1/2 (a valid SPD preconditioner)."""
    spec, sc, x_gt, targets = _observed_problem(oracle_mod)
    rng = np.random.default_rng(3)
    x = oracle_mod.project(spec, x_gt + 0.05 * rng.normal(size=x_gt.size))
    _, blocks, _ = sc.grad_blocks(x, targets)
    half = 0.5 * oracle_mod.block_inverse(blocks)
    opts = dict(max_iters=6, stall_ratio=1e-12)
    lrn = oracle_mod.gn_step(sc, x, targets, precond="learned", learned_minv=half, **opts)
    blk = oracle_mod.gn_step(sc, x, targets, precond="block", **opts)
    assert lrn["fallback_iters"] == 1 and "stall" in lrn["pcg"].flags
    # (the oracle's threaded sums are not bitwise repeatable: 1e-9)
    np.testing.assert_allclose(lrn["delta"], blk["delta"], rtol=1e-9, atol=1e-12 * np.abs(blk["delta"]).max())
    assert lrn["gamma"] == blk["gamma"] and abs(lrn["F_after"] - blk["F_after"]) <= 1e-9 * blk["F_after"]
    ok = oracle_mod.gn_step(sc, x, targets, precond="learned", learned_minv=half, max_iters=6)
    assert ok["fallback_iters"] is None and ok["F_after"] < ok["F_before"]
    # M^-1 / 2 and M^-1 give the same CG iterates up to the scaling of z: the same step
    ref = oracle_mod.gn_step(sc, x, targets, precond="block", max_iters=6)
    np.testing.assert_allclose(ok["delta"], ref["delta"], rtol=1e-9, atol=1e-12 * np.abs(ref["delta"]).max())


# ------------------------------------------------------------------ hierarchy (Sec. IV)

def _half_spec(spec):
    import dataclasses
    return dataclasses.replace(spec, nx=spec.nx // 2, ny=spec.ny // 2, nz=spec.nz // 2,
                               env_w=spec.env_w // 2, env_h=spec.env_h // 2)


def test_upsample_constant_field_and_sigma_scale(oracle_mod):
    """A constant grid stays constant; sigma halves with the voxel side (optical depth per
    voxel length), colours and texel opacities do not change."""
    fine = ps.SceneSpec(8, 6, 4, bbox_min=(-1, -0.75, -0.5), bbox_max=(1, 0.75, 0.5), layer_radii=(1.8, 3.0),
                        env_w=16, env_h=8)
    coarse = _half_spec(fine)
    x = ps.init_params(coarse, colour=0.3, sigma=0.8, alpha=0.25).astype(np.float64)
    y = oracle_mod.upsample(coarse, x, fine).reshape(-1, 4)
    nv = fine.n_vox
    c, sg, al = (float(np.float32(v)) for v in (0.3, 0.8, 0.25))  # the packed parameters are float32
    np.testing.assert_allclose(y[:nv, :3], c, rtol=1e-12)
    np.testing.assert_allclose(y[:nv, 3], 0.5 * sg, rtol=1e-12)
    np.testing.assert_allclose(y[nv:, :3], c, rtol=1e-12)
    np.testing.assert_allclose(y[nv:, 3], al, rtol=1e-12)
    assert y.shape[0] == fine.n_units


def test_upsample_reproduces_affine_fields_inside(oracle_mod):
    """Trilinear / bilinear interpolation is exact on affine functions of the cell-centre
    position, away from the clamped border cells (and along the periodic azimuth for a
    field periodic in it)."""
    coarse = ps.SceneSpec(6, 6, 6, layer_radii=(1.8,), env_w=12, env_h=6)
    fine = ps.SceneSpec(12, 12, 12, layer_radii=(1.8,), env_w=24, env_h=12)
    def centres(n):
        return -1.0 + (np.arange(n) + 0.5) * 2.0 / n
    zc, yc, xc = np.meshgrid(centres(6), centres(6), centres(6), indexing="ij")
    g = np.zeros((6, 6, 6, 4))
    g[..., 0] = 0.3 + 0.2 * xc - 0.1 * yc + 0.05 * zc
    g[..., 3] = 2.0 + xc + yc - zc
    vc = (np.arange(6) + 0.5) / 6.0
    e = np.zeros((1, 6, 12, 4))
    e[..., 1] = (0.2 + 0.5 * vc)[None, :, None]     # affine in the polar coordinate
    e[..., 2] = 0.7                                  # constant (and so periodic) in azimuth
    x = np.concatenate([g.reshape(-1), e.reshape(-1)])
    y = oracle_mod.upsample(coarse, x, fine)
    gy = y[:4 * fine.n_vox].reshape(12, 12, 12, 4)
    Z, Y, X = np.meshgrid(centres(12), centres(12), centres(12), indexing="ij")
    inner = (slice(1, 11),) * 3
    np.testing.assert_allclose(gy[..., 0][inner], (0.3 + 0.2 * X - 0.1 * Y + 0.05 * Z)[inner], atol=1e-12)
    np.testing.assert_allclose(gy[..., 3][inner], 0.5 * (2.0 + X + Y - Z)[inner], atol=1e-12)
    ey = y[4 * fine.n_vox:].reshape(1, 12, 24, 4)
    v = (np.arange(12) + 0.5) / 12.0
    np.testing.assert_allclose(ey[0, 1:11, :, 1], np.broadcast_to((0.2 + 0.5 * v)[1:11, None], (10, 24)), atol=1e-12)
    np.testing.assert_allclose(ey[..., 2], 0.7, atol=1e-12)


def test_upsample_wraps_in_azimuth(oracle_mod):
    """The first and last destination texel columns interpolate between the last and first
    source columns (periodic azimuth), equally weighted at the seam."""
    coarse = ps.SceneSpec(2, 2, 2, layer_radii=(1.8,), env_w=4, env_h=2)
    fine = ps.SceneSpec(4, 4, 4, layer_radii=(1.8,), env_w=8, env_h=4)
    e = np.zeros((1, 2, 4, 4))
    e[0, :, :, 0] = np.array([1.0, 2.0, 3.0, 4.0])[None, :]
    x = np.concatenate([np.zeros(4 * 8), e.reshape(-1)])
    y = oracle_mod.upsample(coarse, x, fine)[4 * fine.n_vox:].reshape(1, 4, 8, 4)
    # destination column j sits at source coordinate (j + 0.5) / 2 - 0.5
    np.testing.assert_allclose(y[0, 0, :, 0], [0.75 * 1 + 0.25 * 4, 0.75 * 1 + 0.25 * 2, 0.25 * 1 + 0.75 * 2,
                                               0.75 * 2 + 0.25 * 3, 0.25 * 2 + 0.75 * 3, 0.75 * 3 + 0.25 * 4,
                                               0.25 * 3 + 0.75 * 4, 0.75 * 4 + 0.25 * 1], atol=1e-12)


def test_upsampled_uniform_medium_renders_the_same(oracle_mod):
    """Closed form: in a uniform medium a ray's transmittance is exp(-sigma_vox * L_vox).
    Refining the grid doubles L in voxel units and the upsampling halves sigma, so every
    rendered pixel is unchanged."""
    coarse = ps.SceneSpec(8, 8, 8, layer_radii=(1.8,), env_w=16, env_h=8)
    fine = ps.SceneSpec(16, 16, 16, layer_radii=(1.8,), env_w=32, env_h=16)
    cams = ps.make_cameras("sphere", 3, 9, 7, 40.0, 3.0, np.random.default_rng(4))
    x = ps.init_params(coarse, colour=0.6, sigma=0.35, alpha=0.9).astype(np.float64)
    y = oracle_mod.upsample(coarse, x, fine)
    Hc = oracle_mod.OracleScene(coarse, cams).render(x)[0]
    Hf = oracle_mod.OracleScene(fine, cams).render(y)[0]
    np.testing.assert_allclose(Hf, Hc, rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------ auxiliary opacity residual (Sec. III-I, Eq. 10)

AUX = 0.1


@pytest.fixture(scope="module")
def tiny_aux(oracle_mod, tiny):
    sc, spec, x, rays = tiny
    sca = oracle_mod.OracleScene(spec, sc.cams, aux_lambda=AUX)
    targets = np.random.default_rng(9).uniform(0, 1, (sca.n_rays, 3)).astype(np.float32)
    return sca, spec, x, rays, targets


@pytest.fixture(scope="module")
def tiny_aux_fd(tiny_aux):
    """Central differences of all four residuals per ray (r_1..r_3 = H - C, r_4 = Eq. 10)."""
    sca, spec, x, rays, targets = tiny_aux
    eps = 1e-6
    J = np.zeros((4 * len(rays), sca.n_params))
    for j in range(sca.n_params):
        xp = x.copy(); xp[j] += eps
        xm = x.copy(); xm[j] -= eps
        rp = sca.render(xp, targets, rays=rays)[1].reshape(-1)
        rm = sca.render(xm, targets, rays=rays)[1].reshape(-1)
        J[:, j] = (rp - rm) / (2 * eps)
    return J


def test_aux_residual_closed_form(oracle_mod):
    """Uniform medium: T = e^{-s0 L} with L the chord in voxel lengths, and
    r_4 = lambda (1 - 4 (T - 1/2)^2); F adds r_4^2 / 2 to the colour residuals."""
    n = 8
    spec, cams = axis_scene(n=n, W=5, H=5, fov=10.0)
    sc = oracle_mod.OracleScene(spec, cams, aux_lambda=AUX)
    s0 = 0.13
    x = params(spec, np.r_[0.5, 0.5, 0.5, s0], np.r_[0.2, 0.2, 0.2, 1.0])
    targets = np.zeros((25, 3), np.float32)
    H, r, F, Te = sc.render(x, targets)
    assert r.shape == (25, 4)
    for ray in range(25):
        py, px = divmod(ray, 5)
        dc = np.array([(px + 0.5 - 2.5) / cams.fx[0], (py + 0.5 - 2.5) / cams.fy[0], 1.0])
        L = 2.0 * np.linalg.norm(dc) / (2.0 / n)
        T = math.exp(-s0 * L)
        assert math.isclose(r[ray, 3], AUX * (1.0 - 4.0 * (T - 0.5) ** 2), rel_tol=1e-12)
    assert math.isclose(F, 0.5 * float((r ** 2).sum()), rel_tol=1e-12)
    # off: three residuals and no extra term
    sc0 = oracle_mod.OracleScene(spec, cams)
    H0, r0, F0, _ = sc0.render(x, targets)
    assert r0.shape == (25, 3)
    assert math.isclose(F - F0, 0.5 * float((r[:, 3] ** 2).sum()), rel_tol=1e-12)


def test_aux_J_matches_finite_differences(tiny_aux, tiny_aux_fd):
    sca, spec, x, rays, targets = tiny_aux
    v = np.random.default_rng(11).normal(size=sca.n_params)
    u = sca.apply_J(x, v, rays=rays)
    assert u.shape == (len(rays), 4)
    ref = (tiny_aux_fd @ v).reshape(-1, 4)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-8
    # the fourth row depends on sigma only
    aux_rows = tiny_aux_fd[3::4]
    assert np.abs(aux_rows.reshape(len(rays), -1, 4)[:, :, :3]).max() < 1e-9


def test_aux_adjoint_JtJ_and_blocks(tiny_aux, tiny_aux_fd):
    sca, spec, x, rays, targets = tiny_aux
    rng = np.random.default_rng(12)
    u = rng.normal(size=4 * len(rays))
    y = sca.apply_Jt(x, u, rays=rays)
    ref = tiny_aux_fd.T @ u
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-8
    v = rng.normal(size=sca.n_params)
    z = sca.apply_JtJ(x, v, rays=rays)
    refz = tiny_aux_fd.T @ (tiny_aux_fd @ v)
    assert np.linalg.norm(z - refz) / np.linalg.norm(refz) < 1e-8
    grad, blocks, F = sca.grad_blocks(x, targets, rays=rays)
    r = sca.render(x, targets, rays=rays)[1].reshape(-1)
    np.testing.assert_allclose(grad, -(tiny_aux_fd.T @ r), atol=1e-8 * np.abs(grad).max())
    assert math.isclose(F, 0.5 * float(r @ r), rel_tol=1e-12)
    A = tiny_aux_fd.T @ tiny_aux_fd
    scale = np.abs(A).max()
    for unit in range(sca.n_units):
        Bd = A[4 * unit:4 * unit + 4, 4 * unit:4 * unit + 4]
        b = blocks[unit]
        exp = np.array([[b[0], 0, 0, b[1]], [0, b[0], 0, b[2]], [0, 0, b[0], b[3]], [b[1], b[2], b[3], b[4]]])
        assert np.abs(Bd - exp).max() <= 1e-8 * scale


# ------------------------------------------------------------------ rendering with the opacity threshold (Sec. IV)

def test_render_threshold_rule(oracle_mod):
    """Uniform medium with T = e^{-s0 L}: below the threshold (1 - T < 0.7) the volume is
    dropped and the pixel shows the opaque layer's colour E; above it, the normal render
    c0 (1 - T) + T E.  Threshold 0 is the normal render."""
    n = 8
    spec, cams = axis_scene(n=n, step=1.0, W=5, H=5, fov=10.0)
    sc = oracle_mod.OracleScene(spec, cams)
    c0, E = np.array([0.2, 0.5, 0.9]), np.array([0.6, 0.1, 0.3])
    for s0, dropped in ((0.01, True), (0.4, False)):
        x = params(spec, np.r_[c0, s0], np.r_[E, 1.0])
        H0 = sc.render(x)[0]
        H, Te, _ = sc.render_image(x, 0.0)
        np.testing.assert_allclose(H, H0, rtol=1e-14)
        H7, Te7, _ = sc.render_image(x, 0.7)
        np.testing.assert_allclose(Te7, Te, rtol=0)
        assert np.all((1 - Te < 0.7) == dropped)
        if dropped:
            np.testing.assert_allclose(H7, np.broadcast_to(E, H7.shape), rtol=1e-14)
        else:
            np.testing.assert_allclose(H7, H0, rtol=1e-14)


def test_psnr_of_render_against_itself_and_offset(oracle_mod):
    """MSE is zero against the targets rendered from the same parameters (PSNR infinite up to
    float32 rounding of the targets) and 10 log10(1 / d^2) for a uniform colour offset d."""
    spec, cams = axis_scene(n=4, step=1.0, W=6, H=4, fov=20.0)
    sc = oracle_mod.OracleScene(spec, cams)
    x = params(spec, np.r_[0.3, 0.4, 0.5, 0.2], np.r_[0.25, 0.25, 0.25, 1.0])
    H, _, _ = sc.render_image(x, 0.7)
    _, _, mse = sc.render_image(x, 0.7, targets=H.astype(np.float32))
    assert mse < 1e-14
    d = 0.125
    _, _, mse2 = sc.render_image(x, 0.7, targets=(H + d).astype(np.float32))
    assert abs(oracle_mod.psnr(mse2) - 10 * np.log10(1 / d ** 2)) < 1e-5


# ------------------------------------------------------------------ jittering (Sec. IV)

def test_jitter_seed_zero_is_the_plain_render(oracle_mod, tiny):
    sc, spec, x, rays = tiny
    j = oracle_mod.OracleScene(spec, sc.cams, jitter_seed=0)
    np.testing.assert_array_equal(j.render(x, rays=rays)[0], sc.render(x, rays=rays)[0])
    j.set_jitter(12345)
    assert np.abs(j.render(x, rays=rays)[0] - sc.render(x, rays=rays)[0]).max() > 1e-6


def test_jitter_generator_is_uniform(oracle_mod, tiny):
    sc = tiny[0]
    u = np.array([[sc.jitter_u(7, ray, s) for s in range(4)] for ray in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.all(np.abs(u.mean(0) - 0.5) < 0.01)
    assert np.all(np.abs(u.var(0) - 1.0 / 12.0) < 0.005)
    c = np.corrcoef(u.T)
    assert np.abs(c - np.eye(4)).max() < 0.03
    # 24-bit values: exact in single precision
    assert np.all(u * 2 ** 24 == np.round(u * 2 ** 24))
    # another seed gives other numbers
    assert abs(sc.jitter_u(8, 0, 0) - sc.jitter_u(7, 0, 0)) > 0


def test_jittered_ray_origin_stays_in_its_pixel(oracle_mod):
    w = ps.workload("small")
    sc = oracle_mod.OracleScene(w.spec, w.cams, jitter_seed=99)
    cams = w.cams
    per = cams.width * cams.height
    for ray in range(0, sc.n_rays, 97):
        cam, pix = divmod(ray, per)
        py, px = divmod(pix, cams.width)
        o, d = sc.ray(ray)
        dc = np.linalg.solve(np.asarray(cams.rot[cam]).reshape(3, 3), d)  # camera frame (right, down, forward)
        u = dc[0] / dc[2] * cams.fx[cam] + cams.cx[cam]
        v = dc[1] / dc[2] * cams.fy[cam] + cams.cy[cam]
        assert px <= u < px + 1 and py <= v < py + 1, (ray, u, v)
        assert abs(u - (px + sc.jitter_u(99, ray, 0))) < 1e-9 and abs(v - (py + sc.jitter_u(99, ray, 1))) < 1e-9


def test_jittered_samples_stay_in_their_steps(oracle_mod):
    """With sigma affine in x and a ray along -x, each sample's sigma gives back its
    position: inside its own step [k D, k D + delta_k), at the midpoint without jitter."""
    n = 16
    spec, cams = axis_scene(n=n, step=0.5, W=1, H=1, fov=1.0)
    h = 2.0 / n
    centres = -1.0 + (np.arange(n) + 0.5) * h
    grid = np.zeros((n, n, n, 4))
    grid[..., 3] = (2.0 + centres)[None, None, :]  # sigma = 2 + x at the cell centres
    x = pack64(grid, np.zeros((1, spec.env_h, spec.env_w, 4)))
    for seed in (0, 5, 6):
        sc = oracle_mod.OracleScene(spec, cams, jitter_seed=seed)
        smp = sc.ray_samples(x, 0)
        o, d = sc.ray(0)
        # the ray enters at x = +1 (d ~ -x); chord coordinate s in voxel lengths
        xs = smp["sigma"] - 2.0
        s = (1.0 - xs) / (-d[0]) / h
        K = len(s)
        k = np.arange(K)
        inner = (xs > -1 + h) & (xs < 1 - h)  # away from the clamped border cells
        lo = k * 0.5
        assert np.all(s[inner] >= lo[inner] - 1e-9) and np.all(s[inner] < lo[inner] + smp["delta"][inner] + 1e-9)
        if seed == 0:
            np.testing.assert_allclose(s[inner], (lo + 0.5 * smp["delta"])[inner], atol=1e-9)
        else:
            assert np.abs(s[inner] - (lo + 0.5 * smp["delta"])[inner]).max() > 0.05
        assert np.all(np.diff(s[inner]) > 0)  # strictly increasing: a voxel that leaves never returns


def test_jittered_rows_match_finite_differences(oracle_mod, tiny):
    sc, spec, x, rays = tiny
    j = oracle_mod.OracleScene(spec, sc.cams, jitter_seed=31)
    J = dense_jacobian_rows(j, x, rays)
    Jfd = dense_jacobian_fd(j, x, rays)
    assert np.abs(J - Jfd).max() / np.abs(Jfd).max() < 1e-8
