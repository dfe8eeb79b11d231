"""BF16 parameter storage on the 64^3 crop of the 256^3 workload (voxels [96,160)^3, same voxel
size and environment layers, 8 cameras at 200x200 framing the crop).

Gated: the GPU's bfloat16 packing is bit-exact (round to nearest even); the FP32 path matches
the FP64 oracle at x; the BF16 path matches the oracle evaluated at the bf16-rounded x to the
FP32 tolerances (same arithmetic on rounded parameters).  Reported: every result of both paths
against the oracle at the unrounded x, printed as a table (and written to
$PERF_REPORT_DIR/precision_cfg3_crop.md when that variable is set).
"""
import os

import numpy as np
import pytest

import perf_synth as ps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def crop():
    import oracle
    from oracle import mlp
    from paper_2112_05598_amd.scene import Scene
    print("[case] precision cfg3 64^3 crop", flush=True)
    w = ps.crop_workload(ps.workload("cfg3"), 96, 64, 8, 200, 200, 14.0, "cfg3_crop")
    orc = oracle.OracleScene(w.spec, w.cams)
    targets = orc.render(w.x_gt)[0].astype(np.float32)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(targets.reshape(-1)).to(dev)
    x = (0.5 * w.x_gt + 0.5 * w.x_init).astype(np.float32)
    xb = mlp.bf16_round(x)  # the oracle's own rounding of the parameters
    s32 = Scene(w.spec, w.cams, t, device="cuda:0")
    s16 = Scene(w.spec, w.cams, t, param_dtype="bf16", device="cuda:0")
    return w, orc, targets, t, x, xb, s32, s16


def test_bf16_packing_is_exact(crop):
    from oracle import mlp
    w, orc, targets, t, x, xb, s32, s16 = crop
    packed = s32.pack_bf16(torch.from_numpy(x).cuda()).view(torch.int16).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(packed, mlp.bf16_bits(x))


def test_precision_fp32_and_bf16(crop):
    w, orc, targets, t, x, xb, s32, s16 = crop
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    tb = s32.pack_bf16(tx)
    v = ps.random_vector(s32.n_params, 11)
    tv = torch.from_numpy(v).to(dev)
    x64, v64 = x.astype(np.float64), v.astype(np.float64)
    res = {}
    for name, sc, xx in (("fp32", s32, tx), ("bf16", s16, tb)):
        r, F = sc.render_residuals(xx)
        res[name] = {"r": r.cpu().numpy(), "Jv": sc.apply_J(xx, tv).cpu().numpy(),
                     "JtJv": sc.apply_JtJ(xx, tv).cpu().numpy()}
        g, b, _, _ = sc.build_precond(xx, "jacobi")
        res[name]["grad"] = g.cpu().numpy()
        res[name]["blocks"] = b.cpu().numpy()
    ref = {}
    for name, xx in (("x", x64), ("x_bf16", xb)):
        _, r, _, _ = orc.render(xx, targets)
        g, b, _ = orc.grad_blocks(xx, targets)
        ref[name] = {"r": r, "Jv": orc.apply_J(xx, v64), "JtJv": orc.apply_JtJ(xx, v64), "grad": g, "blocks": b}
    tol = {"r": 1e-5, "Jv": 1e-4, "JtJv": 1e-4, "grad": 1e-4, "blocks": 1e-4}
    rows = []
    for k in ("r", "Jv", "JtJv", "grad", "blocks"):
        e32 = rel(res["fp32"][k], ref["x"][k])
        e16_same = rel(res["bf16"][k], ref["x_bf16"][k])
        e16 = rel(res["bf16"][k], ref["x"][k])
        rows.append((k, e32, e16_same, e16))
        assert e32 <= tol[k], (k, e32)
        assert e16_same <= tol[k], (k, e16_same)
    table = "| result | FP32 vs oracle(x) | BF16 vs oracle(bf16(x)) | BF16 vs oracle(x) |\n|---|---|---|---|\n"
    table += "".join(f"| {k} | {a:.2e} | {b:.2e} | {c:.2e} |\n" for k, a, b, c in rows)
    print(table, flush=True)
    out_dir = os.environ.get("PERF_REPORT_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "precision_cfg3_crop.md"), "w") as f:
            f.write(table)
