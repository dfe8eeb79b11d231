"""What the trained network gains over the method without it (Jacobi, the paper's
preconditioner), at the benchmark's horizon: Gauss-Newton with the committed learned block
preconditioner reaches the objective that 20 Jacobi-PCG GN steps (30 PCG iterations each)
reach, in fewer PCG iterations and less wall time, on a held-out seed of the 128^3
object-in-a-box kind (no training scene shares it, and it took no part in choosing the model)."""
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_learned_reaches_jacobi_objective_sooner():
    from paper_2112_05598_amd import learned
    print("[case] learned vs Jacobi GN, 20 steps, held-out seed 20005", flush=True)
    w = ps.workload("cfg4", seed=20005)
    model = learned.load_model(device="cuda:0")
    out = learned.gn_compare(w, {"learned": model}, n_steps=20, pcg_iters=30, extra_steps=3,
                             log=lambda m: print(m, flush=True))
    jac, lrn = out["jacobi"], out["learned"]
    assert jac["F"][-1] < jac["F0"]
    assert lrn["reached"], (lrn["F"], jac["F"][-1])
    assert lrn["pcg_iters"] < jac["pcg_iters"]
    assert lrn["ms"] < jac["ms"]
