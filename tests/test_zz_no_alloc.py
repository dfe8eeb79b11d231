"""The allocation-free training step (perf_mlp_train_step_noalloc) against the training step with a
caller-provided gradient buffer (perf_mlp_train_step), through the C ABI: two calls in a row, the
second on a smaller batch, each from the same state on both entry points."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    from paper_2112_05598_amd import abi
    k = abi.PERF_MLP_NFEAT
    feat = rng.normal(size=(n, k)) * rng.uniform(0.5, 3.0, k) + rng.uniform(-5, 5, k)
    d = rng.uniform(0.1, 5.0, n)
    f = rng.uniform(0.1, 5.0, n)
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    e = dirs * (rng.uniform(0.0, 0.95, n) * np.sqrt(d * f))[:, None]
    blocks = np.concatenate([d[:, None], e, f[:, None]], axis=1)
    return (torch.from_numpy(feat.astype(np.float32)).cuda(), torch.from_numpy(blocks.astype(np.float32)).cuda())


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_training_step_matches_the_buffered_one():
    from oracle import mlp
    from paper_2112_05598_amd import abi
    from paper_2112_05598_amd.scene import mlp_feature_stats
    lib = abi.load()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(3)
    w0 = mlp.init_weights(2) + 0.05 * rng.normal(size=mlp.NW)
    p = mlp.unpack(w0); p["W1"][:, mlp.N_NET:] = 0; p["W3"][10:] = 0
    w0 = mlp.pack(p).astype(np.float32)
    state = {k: torch.from_numpy(w0.copy()).cuda() if k == "w32" else torch.zeros(mlp.NW, device="cuda")
             for k in ("w32", "m", "v")}
    state["wbf"] = state["w32"].to(torch.bfloat16)
    for call, (n, seed) in enumerate(((3000, 1), (700, 2))):
        feat, blocks = _rows(n, seed)
        norm = mlp_feature_stats(feat)
        print(f"[no-alloc] call {call}: {n} rows", flush=True)
        outs = []
        for noalloc in (False, True):
            w32 = state["w32"].clone(); m = state["m"].clone(); v = state["v"].clone(); wbf = state["wbf"].clone()
            loss = torch.zeros(1, device="cuda")
            if noalloc:
                rc = lib.perf_mlp_train_step_noalloc(_p(w32), _p(wbf), _p(m), _p(v), call + 1, ctypes.c_float(1e-3),
                                                     ctypes.c_float(0.0), _p(norm), _p(feat), _p(blocks), n,
                                                     _p(loss), st)
            else:
                grad = torch.zeros(mlp.NW, device="cuda")
                rc = lib.perf_mlp_train_step(_p(w32), _p(wbf), _p(m), _p(v), call + 1, ctypes.c_float(1e-3),
                                             ctypes.c_float(0.0), _p(norm), _p(feat), _p(blocks), n, _p(loss),
                                             _p(grad), st)
            assert rc == abi.PERF_OK, lib.perf_last_error()
            torch.cuda.synchronize()
            outs.append((w32, m, v, wbf, loss))
        (w_a, m_a, v_a, b_a, l_a), (w_b, m_b, v_b, b_b, l_b) = outs
        # the gradient is summed with float atomics in either case: equal up to summation order
        assert abs(l_a.item() - l_b.item()) <= 1e-5 * abs(l_a.item())
        for a, b in ((m_a, m_b), (v_a, v_b), (w_a, w_b)):
            a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(a), (np.linalg.norm(a - b), np.linalg.norm(a))
        assert torch.count_nonzero(m_b) > mlp.NW // 2
        state = {"w32": w_a, "m": m_a, "v": v_a, "wbf": b_a}


def test_noalloc_training_step_rejects_bad_arguments():
    from paper_2112_05598_amd import abi
    lib = abi.load()
    z = torch.zeros(64, device="cuda")
    assert lib.perf_mlp_train_step_noalloc(None, _p(z), _p(z), _p(z), 1, ctypes.c_float(1e-3), ctypes.c_float(0.0),
                                           _p(z), None, None, 0, _p(z), None) == abi.PERF_EINVAL
    assert lib.perf_mlp_train_step_noalloc(_p(z), _p(z), _p(z), _p(z), 0, ctypes.c_float(1e-3), ctypes.c_float(0.0),
                                           _p(z), None, None, 0, _p(z), None) == abi.PERF_EINVAL
    assert lib.perf_mlp_train_step_noalloc(_p(z), _p(z), _p(z), _p(z), 1, ctypes.c_float(1e-3), ctypes.c_float(0.0),
                                           _p(z), None, None, 5, _p(z), None) == abi.PERF_EINVAL
