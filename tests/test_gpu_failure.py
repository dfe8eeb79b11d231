"""Failure handling of the GPU path, forced from the host (every kernel runs to its end).

* With checks on, a non-finite parameter or target makes the Gauss-Newton step return
  PERF_ENUMERIC before any solve, and leaves x untouched.
* With checks off the same input is not an error: the first p^T A p is not finite, PCG stops
  with the breakdown flag (a PCG breakdown is a flag, not an error), the line search finds no
  finite objective and the step keeps x (step length 0).
* Units that no ray touches have a zero Jacobi diagonal and get a zero inverse, so PCG never
  moves them.
"""
import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make(checks, bad_x=False, bad_target=False):
    import oracle
    from paper_2112_05598_amd.scene import Scene
    w = ps.workload("small")
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32).reshape(-1)
    x = w.x_init.astype(np.float32).copy()
    if bad_x:
        x[4 * (w.spec.n_vox // 2) + 3] = np.nan  # sigma of a central voxel
    if bad_target:
        targets[7] = np.inf
    dev = torch.device("cuda:0")
    sc = Scene(w.spec, w.cams, torch.from_numpy(targets).to(dev), device="cuda:0", checks=checks)
    return sc, torch.from_numpy(x).to(dev)


@pytest.mark.parametrize("what", ["x", "target"])
def test_checks_reject_non_finite_inputs(what):
    from paper_2112_05598_amd import abi
    print(f"[failure] checks on, non-finite {what}", flush=True)
    sc, tx = make(True, bad_x=what == "x", bad_target=what == "target")
    before = tx.clone()
    with pytest.raises(abi.PerfError) as e:
        sc.gn_step(tx, max_iters=5)
    assert e.value.code == abi.PERF_ENUMERIC
    torch.cuda.synchronize()
    assert torch.equal(torch.isnan(tx), torch.isnan(before))
    finite = torch.isfinite(before)
    assert torch.equal(tx[finite], before[finite])


def test_checks_pass_finite_inputs():
    print("[failure] checks on, finite inputs", flush=True)
    sc, tx = make(True)
    st = sc.gn_step(tx, max_iters=5)
    assert st["F_after"] < st["F_before"]


def test_unchecked_non_finite_input_stops_pcg_with_breakdown():
    from paper_2112_05598_amd import abi
    print("[failure] checks off, non-finite x", flush=True)
    sc, tx = make(False, bad_x=True)
    before = tx.clone()
    st = sc.gn_step(tx, max_iters=5, ls_max=4)
    torch.cuda.synchronize()
    assert st["flags"] & abi.PERF_FLAG_BREAKDOWN
    assert st["pcg_iters"] == 0
    assert st["flags"] & abi.PERF_FLAG_NO_DESCENT and st["gamma"] == 0.0
    finite = torch.isfinite(before)
    assert torch.equal(tx[finite], before[finite])


def test_untouched_units_get_zero_inverse():
    print("[failure] zero-diagonal units", flush=True)
    sc, tx = make(False)
    _, blocks, minv, _ = sc.build_precond(tx, "jacobi")
    _, _, binv, _ = sc.build_precond(tx, "block")
    d = blocks[:, 0].cpu().numpy()
    f = blocks[:, 4].cpu().numpy()
    dead = (d == 0) & (f == 0)
    assert dead.any() and (~dead).any()
    assert np.all(minv.view(-1, 4).cpu().numpy()[dead] == 0)
    assert np.all(binv.view(-1, 8).cpu().numpy()[dead] == 0)
