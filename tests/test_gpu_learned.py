"""GPU parity of the learned block preconditioner: features, MFMA inference and the
training kernel against the FP64 reference."""
import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", params=["tiny", "ragged"])
def setup(request):
    import oracle
    from paper_2112_05598_amd.scene import Scene
    name = request.param
    print(f"[case] learned {name}", flush=True)
    w = ps.workload(name)
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(targets.reshape(-1)).to(dev)
    sc = Scene(w.spec, w.cams, t, learned=True, device="cuda:0")
    rng = np.random.default_rng(4)
    x = w.x_init.copy().reshape(-1, 4)
    x[:, 3] += rng.uniform(0, 0.5, x.shape[0]).astype(np.float32)  # some opacity everywhere
    x = x.reshape(-1).astype(np.float32)
    return w, orc, sc, targets, t, x


def test_features_match_oracle(setup):
    """The blocks against the oracle's (1e-4), the features against the oracle's features of
    the same x and the oracle's blocks: the parameters bit for bit, the logs of the diagonals
    to their FP32 accuracy."""
    from oracle import mlp
    w, orc, sc, targets, t, x = setup
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    feat = feat.cpu().numpy()
    assert feat.shape == (sc.n_units, mlp.N_IN)
    _, b_or, _ = orc.grad_blocks(x.astype(np.float64), targets)
    f_or = mlp.features(x, b_or)
    live = np.maximum(b_or[:, 0], b_or[:, 4]) > 1e-10 * b_or[:, 0].max()
    assert rel(blocks.cpu().numpy(), b_or) <= 1e-4
    np.testing.assert_array_equal(feat[:, 0:4], x.reshape(-1, 4)[:, [3, 0, 1, 2]])
    # logs of the diagonals: absolute error = relative error of d and f.  f sums squares of
    # sigma partials whose terms cancel where a voxel's colour matches the colour behind it,
    # so a few units lose relative precision in FP32; bound the bulk and the norm
    err = np.abs(feat[live, 4:6] - f_or[live, 4:6])
    assert np.quantile(err, 0.999) <= 1e-3
    assert rel(feat[live, 4:6], f_or[live, 4:6]) <= 1e-4


def gpu_norm(feat):
    """The library's standardisation of the features (and its FP64 copy)."""
    from paper_2112_05598_amd.scene import mlp_feature_stats
    norm = mlp_feature_stats(feat)
    return norm, norm.cpu().numpy().astype(np.float64)


def test_feature_stats_match_oracle(setup):
    from oracle import mlp
    w, orc, sc, targets, t, x = setup
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    live = torch.nonzero(torch.maximum(blocks[:, 0], blocks[:, 4]) > 0).squeeze(1)
    f = feat[live].contiguous()
    _, n64 = gpu_norm(f)
    ref = mlp.feature_stats(f.cpu().numpy().astype(np.float64))
    k = mlp.N_IN
    np.testing.assert_allclose(n64[:k], ref[:k], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(n64[16:16 + k], ref[16:16 + k], rtol=1e-5)
    assert np.all(n64[k:16] == 0) and np.all(n64[16 + k:] == 0)


def test_training_rows_are_the_touched_units(setup):
    """keep = 1: every touched unit, in unit order, bit for bit; keep = 0.3: a deterministic
    subset in unit order of about 30 % of them."""
    w, orc, sc, targets, t, x = setup
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    b = blocks.cpu().numpy()
    f = feat.cpu().numpy()
    touched = np.nonzero(np.maximum(b[:, 0], b[:, 4]) > 0)[0]
    fo, bo, n = sc.training_rows(feat, blocks, 5, 1.0, len(touched) + 10)
    assert n == len(touched)
    np.testing.assert_array_equal(fo.cpu().numpy(), f[touched])
    np.testing.assert_array_equal(bo.cpu().numpy(), b[touched])
    fo1, bo1, n1 = sc.training_rows(feat, blocks, 9, 0.3, len(touched))
    fo2, bo2, n2 = sc.training_rows(feat, blocks, 9, 0.3, len(touched))
    assert n1 == n2 and torch.equal(fo1, fo2) and torch.equal(bo1, bo2)
    sd = np.sqrt(len(touched) * 0.3 * 0.7)
    assert abs(n1 - 0.3 * len(touched)) <= 5 * sd + 1
    # a subset of the touched units' rows, in unit order
    key = {tuple(r): i for i, r in enumerate(np.concatenate([f[touched], b[touched]], 1).tolist())}
    idx = [key[tuple(r)] for r in np.concatenate([fo1.cpu().numpy(), bo1.cpu().numpy()], 1).tolist()]
    assert np.all(np.diff(idx) > 0)
    # a cap below the count writes the first cap rows of the same selection
    fo3, _, n3 = sc.training_rows(feat, blocks, 9, 0.3, 17)
    assert n3 == n1 and torch.equal(fo3, fo1[:17])


def test_mlp_inference_matches_fp64_mlp(setup):
    from oracle import mlp
    w, orc, sc, targets, t, x = setup
    rng = np.random.default_rng(0)
    w64 = mlp.init_weights(3) + 0.05 * rng.normal(size=mlp.NW)
    p = mlp.unpack(w64); p["W1"][:, mlp.N_NET:] = 0; p["W3"][10:] = 0
    bits = mlp.bf16_bits(mlp.pack(p))
    wq = mlp.bits_to_f64(bits)
    wt = torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    norm, n64 = gpu_norm(feat)
    sc.mlp_set_weights(wt, norm)
    out = sc.mlp_infer(feat, blocks).cpu().numpy()
    f64, b64 = feat.cpu().numpy().astype(np.float64), blocks.cpu().numpy().astype(np.float64)
    iu = np.triu_indices(4)
    _, dis, live = mlp.normalised_block(b64)
    # the scaled form: D^-1/2 (t_d, t_f) and the factor L; compare the normalised inverses
    # L L^T = D^1/2 M^-1 D^1/2 (order-one entries)
    from gpu_checks import learned_factor
    np.testing.assert_allclose(out[live, 0], dis[live, 0], rtol=1e-6)
    np.testing.assert_allclose(out[live, 1], dis[live, 3], rtol=1e-6)
    L = learned_factor(out)
    got = (L @ np.transpose(L, (0, 2, 1)))[:, iu[0], iu[1]]
    scale = np.where(live[:, None], 1.0 / (dis[:, iu[0]] * dis[:, iu[1]] + 1e-300), 0.0)
    emu = mlp.minv(wq, n64, f64, b64, emulate_bf16=True)[:, iu[0], iu[1]] * scale
    exact = mlp.minv(wq, n64, f64, b64)[:, iu[0], iu[1]] * scale
    # same bf16 roundings of inputs and activations: FP32 accumulation and rare ties only
    assert rel(got[live], emu[live]) <= 2e-3
    # against the all-FP64 network: three bf16 roundings (unit roundoff 2^-9) per path
    assert rel(got[live], exact[live]) <= 3e-2
    assert np.all(out[~live] == 0)
    # the factor has a positive diagonal (softplus): every predicted inverse is SPD
    assert np.all(L[live][:, [0, 1, 2, 3], [0, 1, 2, 3]] > 0)


@pytest.mark.parametrize("damp", [0.0, 0.3])
def test_mlp_training_gradient(setup, damp):
    from oracle import mlp
    from paper_2112_05598_amd.scene import mlp_train_step
    w, orc, sc, targets, t, x = setup
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    live = torch.nonzero(torch.maximum(blocks[:, 0], blocks[:, 4]) > 0).squeeze(1)[:4096]
    fb, bb = feat[live].contiguous(), blocks[live].contiguous()
    rng = np.random.default_rng(1)
    w64 = mlp.init_weights(5) + 0.05 * rng.normal(size=mlp.NW)
    p = mlp.unpack(w64); p["W1"][:, mlp.N_NET:] = 0; p["W3"][10:] = 0
    bits = mlp.bf16_bits(mlp.pack(p))
    wq = mlp.bits_to_f64(bits)
    dev = fb.device
    w32 = torch.from_numpy(wq.astype(np.float32)).to(dev)
    wbf = torch.from_numpy(bits.view(np.int16)).to(dev).view(torch.bfloat16).clone()
    m = torch.zeros_like(w32); v = torch.zeros_like(w32); g = torch.zeros_like(w32)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    norm, n64 = gpu_norm(fb)
    mlp_train_step(w32, wbf, m, v, 1, 1e-4, norm, fb, bb, loss, g, damp=damp)
    torch.cuda.synchronize()
    grad_gpu = (m / 0.1).cpu().numpy()  # first Adam step from m = 0: m = (1 - beta1) g
    L_or, g_or = mlp.loss_and_grad(wq, n64, fb.cpu().numpy().astype(np.float64), bb.cpu().numpy().astype(np.float64),
                                   damp)
    assert abs(loss.item() - L_or) <= 2e-2 * L_or
    cos = grad_gpu @ g_or / (np.linalg.norm(grad_gpu) * np.linalg.norm(g_or))
    assert cos >= 0.999
    assert rel(grad_gpu, g_or) <= 5e-2
    # Adam's first step moves every weight with a gradient by lr against its sign
    moved = (w32.cpu().numpy() - wq)
    nz = np.abs(g_or) > 1e-3 * np.abs(g_or).max()
    assert np.all(np.sign(moved[nz]) == -np.sign(g_or[nz]))


def learned_weights(seed):
    """A network away from its L = I start (bf16 bits and their FP64 values)."""
    from oracle import mlp
    rng = np.random.default_rng(seed)
    w64 = mlp.init_weights(seed) + 0.05 * rng.normal(size=mlp.NW)
    p = mlp.unpack(w64); p["W1"][:, mlp.N_NET:] = 0; p["W3"][10:] = 0
    bits = mlp.bf16_bits(mlp.pack(p))
    return bits, mlp.bits_to_f64(bits)


def test_learned_gn_step_matches_oracle(setup):
    """One GN step with the learned preconditioner against the oracle's GN step (Eq. 7, Alg. 2,
    Alg. 3) with M^-1 from the FP64 network on the same features: the network's bf16 activations
    leave the per-unit inverse within the inference bound (2e-3) of the FP64 emulation, which the
    PCG scalars inherit, so they get 1e-3 here; with the library's own inverse, multiplied out
    in FP64, the solve itself matches to the J^T J v bound (1e-4)."""
    import oracle
    from oracle import mlp
    from gpu_checks import learned_minv
    from gpu_checks import check_pcg_history
    w, orc, sc, targets, t, x = setup
    bits, wq = learned_weights(7)
    tx = torch.from_numpy(x).cuda()
    feat, blocks = sc.features(tx)
    norm, n64 = gpu_norm(feat)
    sc.mlp_set_weights(torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16), norm)
    minv_gpu = learned_minv(sc.mlp_infer(feat, blocks).cpu().numpy())
    x64 = x.astype(np.float64)
    _, b_or, _ = orc.grad_blocks(x64, targets)
    minv_or = mlp.minv(wq, n64, feat.cpu().numpy().astype(np.float64), b_or, emulate_bf16=True)
    st = sc.gn_step(tx.clone(), max_iters=8, precond="learned")
    assert st["F_after"] < st["F_before"]
    assert st["pcg_iters"] >= 1 and not (st["flags"] & 1)
    for minv, tol in ((minv_gpu, 1e-4), (minv_or, 1e-3)):
        ref = oracle.gn_step(orc, x64, targets, precond="learned", max_iters=8, learned_minv=minv)
        assert abs(st["F_before"] - ref["F_before"]) <= 1e-5 * ref["F_before"]
        assert st["pcg_iters"] == ref["pcg"].iters
        check_pcg_history(st, ref["pcg"], min(5, ref["pcg"].iters), tol=tol)
        assert abs(st["F_after"] - ref["F_after"]) <= 1e-3 * ref["F_before"], (st["F_after"], ref["F_after"])


def test_failed_learned_solve_falls_back_to_block_jacobi(setup):
    """A learned solve that stalls is discarded and the step solved again with the exact block
    inverse, as the oracle's GN step does.  The stall is forced from the host: with a stall
    ratio of 1e-12 Alg. 2's early exit fires after the first update of either solve."""
    import oracle
    from gpu_checks import learned_minv
    from paper_2112_05598_amd import abi
    w, orc, sc, targets, t, x = setup
    bits, _ = learned_weights(7)
    tx = torch.from_numpy(x).cuda()
    feat, blocks = sc.features(tx)
    norm, _ = gpu_norm(feat)
    sc.mlp_set_weights(torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16), norm)
    minv_gpu = learned_minv(sc.mlp_infer(feat, blocks).cpu().numpy())
    opts = dict(max_iters=6, stall_ratio=1e-12)
    st = sc.gn_step(tx.clone(), precond="learned", **opts)
    assert st["flags"] & abi.PERF_FLAG_FALLBACK and st["flags"] & abi.PERF_FLAG_STALL
    assert st["fallback_iters"] == 1 and st["pcg_iters"] == 1
    blk = sc.gn_step(tx.clone(), precond="block", **opts)
    assert not (blk["flags"] & abi.PERF_FLAG_FALLBACK) and blk["fallback_iters"] == 0
    # the same solve up to the order of the gradient pass's float atomics
    assert abs(st["alpha"][0] - blk["alpha"][0]) <= 1e-5 * abs(blk["alpha"][0])
    assert abs(st["F_after"] - blk["F_after"]) <= 1e-5 * blk["F_before"]
    ref = oracle.gn_step(orc, x.astype(np.float64), targets, precond="learned", learned_minv=minv_gpu,
                         **opts)
    assert ref["fallback_iters"] == 1 and ref["pcg"].iters == 1
    assert abs(st["alpha"][0] - ref["pcg"].alpha[0]) <= 1e-4 * abs(ref["pcg"].alpha[0])
    assert abs(st["F_after"] - ref["F_after"]) <= 1e-3 * ref["F_before"], (st["F_after"], ref["F_after"])
    # without a failure the learned solve stands
    ok = sc.gn_step(tx.clone(), precond="learned", max_iters=6)
    assert not (ok["flags"] & abi.PERF_FLAG_FALLBACK) and ok["fallback_iters"] == 0


def test_fallback_units_take_the_exact_block_inverse(setup):
    """Threshold 0: every touched unit takes the exact block inverse (the block form with t_d
    negated), equal to the oracle's (B + rho I)^-1; a finite threshold: units the FP64 network
    places clearly above it fall back, clearly below it keep the prediction, both on the GPU."""
    import oracle
    from oracle import mlp
    from gpu_checks import block_minv
    w, orc, sc, targets, t, x = setup
    bits, wq = learned_weights(3)
    wt = torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)
    feat, blocks = sc.features(torch.from_numpy(x).cuda())
    norm, n64 = gpu_norm(feat)
    b64 = blocks.cpu().numpy().astype(np.float64)
    live = np.maximum(b64[:, 0], b64[:, 4]) > 0
    sc.mlp_set_weights(wt, norm, 0.0)
    out = sc.mlp_infer(feat, blocks).cpu().numpy()
    assert np.all(out[live, 0] < 0) and np.all(out[~live] == 0)
    blk = out[:, :8].copy()
    blk[:, 0] = -blk[:, 0]
    got = block_minv(blk)
    ref = oracle.block_inverse(b64)
    scale = np.abs(ref).max(axis=(1, 2))
    err = np.abs(got - ref).max(axis=(1, 2))[live] / scale[live]
    assert err.max() <= 1e-5, err.max()
    _, fb, q = mlp.minv(wq, n64, feat.cpu().numpy().astype(np.float64), b64, emulate_bf16=True, q_fallback=0.0,
                        return_fallback=True)
    thr = float(np.median(q[live]))
    sc.mlp_set_weights(wt, norm, thr)
    out = sc.mlp_infer(feat, blocks).cpu().numpy()
    clear_hi = live & (q > 1.05 * thr)
    clear_lo = live & (q < 0.95 * thr)
    assert clear_hi.sum() > 10 and clear_lo.sum() > 10
    assert np.all(out[clear_hi, 0] < 0) and np.all(out[clear_lo, 0] > 0)


def test_learned_gn_step_bf16_storage_matches_oracle():
    """With bf16 parameter storage the learned GN step takes its features from the parameters the
    gradient pass gathered (the bf16 copy), as perf_precond_features does for the same scene: its
    PCG scalars match the oracle's GN step at the bf16-rounded parameters, run with the library's
    own predicted inverse, to the J^T J v bound (1e-4), and the step lowers F."""
    import oracle
    from oracle import mlp
    from gpu_checks import check_pcg_history, learned_minv
    from paper_2112_05598_amd.scene import Scene
    w = ps.workload("tiny")
    print("[case] learned GN step, bf16 storage, tiny", flush=True)
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32)
    rng = np.random.default_rng(4)
    x = w.x_init.copy().reshape(-1, 4)
    x[:, 3] += rng.uniform(0, 0.5, x.shape[0]).astype(np.float32)
    x = x.reshape(-1).astype(np.float32)
    sc = Scene(w.spec, w.cams, torch.from_numpy(targets.reshape(-1)).cuda(), param_dtype="bf16", learned=True,
               device="cuda:0")
    tx = torch.from_numpy(x).cuda()
    feat, blocks = sc.features(sc.pack_bf16(tx))
    norm, _ = gpu_norm(feat)
    bits, _ = learned_weights(7)
    sc.mlp_set_weights(torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16), norm)
    minv_gpu = learned_minv(sc.mlp_infer(feat, blocks).cpu().numpy())
    st = sc.gn_step(tx.clone(), max_iters=8, precond="learned")
    assert st["F_after"] < st["F_before"] and st["fallback_iters"] == 0
    xb = mlp.bf16_round(x).astype(np.float64)
    ref = oracle.gn_step(orc, xb, targets, precond="learned", max_iters=8, learned_minv=minv_gpu)
    assert abs(st["F_before"] - ref["F_before"]) <= 1e-5 * ref["F_before"]
    assert st["pcg_iters"] == ref["pcg"].iters
    check_pcg_history(st, ref["pcg"], min(5, ref["pcg"].iters), tol=1e-4)
