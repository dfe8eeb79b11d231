"""Ray sharding, emulated on one GPU.

Eq. 9 of the paper writes J^T J v as a sum of one term per residual, and the gradient, the
Jacobi diagonal, the 4x4 blocks and F are sums over rays too.  A solve spread over several
GPUs would give each GPU a share of the cameras and add the per-GPU products (one
reduce-scatter of y per product).  Here the shares run one after another on one GPU: each
camera subset gets its own scene, and the sum of the shard results must equal the unsharded
result up to the order of float atomic adds (norm-wise 1e-6), and the FP64 oracle (1e-4).
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


def shard_scenes(w, targets, bounds):
    """One scene per camera range [bounds[i], bounds[i+1]); targets [n_cams, H, W, 3]."""
    from paper_2112_05598_amd.scene import Scene
    dev = torch.device("cuda:0")
    out = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        t = torch.from_numpy(np.ascontiguousarray(targets[a:b]).reshape(-1)).to(dev)
        out.append((Scene(w.spec, w.cams.subset(range(a, b)), t, device="cuda:0"), t))
    return out


def sharded_sums(scenes, full, x, v):
    y = sum(sc.apply_JtJ(x, v).double() for sc, _ in scenes)
    parts = [sc.build_precond(x, "jacobi") for sc, _ in scenes]
    g = sum(p[0].double() for p in parts)
    B = sum(p[1].double() for p in parts)
    F = sum(p[3].item() for p in parts)
    gf, Bf, _, Ff = full.build_precond(x, "jacobi")
    yf = full.apply_JtJ(x, v)
    return (y, yf), (g, gf), (B, Bf), (F, Ff.item())


def test_shards_add_up_and_match_oracle():
    import oracle
    from paper_2112_05598_amd.scene import Scene
    w = ps.workload("cfg1")
    print(f"[shard] cfg1: {w.cams.n} cameras in shards [0,3) [3,4) [4,{w.cams.n})", flush=True)
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32)  # [n_cams * H * W, 3]
    dev = torch.device("cuda:0")
    x = w.x_init.astype(np.float32)
    tx = torch.from_numpy(x).to(dev)
    v = ps.random_vector(w.spec.n_params, 5)
    tv = torch.from_numpy(v).to(dev)
    t_all = torch.from_numpy(targets.reshape(-1)).to(dev)
    full = Scene(w.spec, w.cams, t_all, device="cuda:0")
    scenes = shard_scenes(w, targets.reshape(w.cams.n, -1, 3), [0, 3, 4, w.cams.n])
    (y, yf), (g, gf), (B, Bf), (F, Ff) = sharded_sums(scenes, full, tx, tv)
    torch.cuda.synchronize()
    assert rel(y.cpu(), yf.cpu()) <= 1e-6
    assert rel(g.cpu(), gf.cpu()) <= 1e-6
    assert rel(B.cpu(), Bf.cpu()) <= 1e-6
    assert abs(F - Ff) <= 1e-12 * Ff
    x64 = x.astype(np.float64)
    assert rel(y.cpu(), orc.apply_JtJ(x64, v.astype(np.float64))) <= 1e-4
    # the oracle's gradient of F is J^T r; the library returns -J^T r
    _, r_or, F_or, _ = orc.render(x64, targets)
    assert rel(-g.cpu().numpy(), orc.apply_Jt(x64, r_or.reshape(-1))) <= 1e-4
    assert abs(F - F_or) <= 1e-5 * F_or


def test_one_gpu_share_at_full_size():
    """The 128^3 workload with 100 cameras of 400x400 in four shares of 25 cameras: the
    shape one of four GPUs would hold."""
    w = ps.workload("cfg2")
    print(f"[shard] cfg2: {w.cams.n} cameras in 4 shards of 25", flush=True)
    from paper_2112_05598_amd.scene import Scene
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(42)
    targets = rng.uniform(0.0, 1.0, size=(w.cams.n, w.cams.height * w.cams.width, 3)).astype(np.float32)
    tx = torch.from_numpy(w.x_init).to(dev)
    tv = torch.from_numpy(ps.random_vector(w.spec.n_params, 6)).to(dev)
    full = Scene(w.spec, w.cams, torch.from_numpy(targets.reshape(-1)).to(dev), device="cuda:0")
    scenes = shard_scenes(w, targets, [0, 25, 50, 75, 100])
    (y, yf), (g, gf), (B, Bf), (F, Ff) = sharded_sums(scenes, full, tx, tv)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(y - yf.double()) / torch.linalg.norm(yf.double())) <= 1e-6
    assert float(torch.linalg.norm(g - gf.double()) / torch.linalg.norm(gf.double())) <= 1e-6
    assert float(torch.linalg.norm(B - Bf.double()) / torch.linalg.norm(Bf.double())) <= 1e-6
    assert abs(F - Ff) <= 1e-12 * Ff
