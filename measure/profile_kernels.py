"""Profiling script for the library's hot kernels and their rocprofv3 summaries.

  run:        python -m measure.profile_kernels run --workload cfg2 --launches 2 --copy-mib 2048 \
                  [--timing-json T.json]
  summarise:  python -m measure.profile_kernels summarise --fetch F.db --write W.db --out traffic.json \
                  [--atomic A.db --timing-json T.json]
  counters:   python -m measure.profile_kernels counters --db P1.db [--db P2.db ...] --out counters.json
  report:     python -m measure.profile_kernels report --counters counters.json --traffic traffic.json \
                  --stats kernel_stats.csv [--out table.md]

`run` launches, on the named workload at the initial parameters: the J^T J v product `--launches`
times (seeded random v), the gradient + exact-block pass, the learned preconditioner's features
(another gradient/block pass and the per-unit feature kernel), the MLP inference over every unit
and four training steps on 16384 rows; then
one plain device-to-device copy of `--copy-mib` MiB (an elementwise b = a * 1) as the
calibration kernel of the HBM counters, and the atomic probe (measure/atomic_probe.hip).  With
--timing-json it records the durations (HIP events on the launch stream) of an unprofiled run.
Run it under `rocprofv3 --pmc <counters>` once per counter set.

`summarise` reads a FETCH_SIZE and a WRITE_SIZE database, averages each counter per dispatch of the
J^T J v kernel, scales it by (known copy bytes / counted copy bytes) of the calibration copy, and
writes the HBM bytes per dispatch together with the sha256 of the kernel source they were
measured on; with --atomic (a TCC_ATOMIC pass) and --timing-json it adds the L2 atomic requests
per second of the J^T J v kernel against those of the probe, and the HBM bytes per dispatch of the
other profiled kernels.  `counters` averages every counter of the given databases per dispatch of
each kernel.  `report` writes the tables of the kernel summary: durations from the kernel trace,
VALU issue share (wave instructions over one per CU per cycle at 2.4 GHz, the wave64 FP32 rate
without packed math), the share of wave cycles spent waiting on LDS, MFMA flop/s and HBM bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))  # the repository root
KERNEL_SRC = os.path.join(ROOT, "paper_2112_05598_amd", "csrc", "raymarch.hip")
JTJ_TAG = "k_ray<3, 0>"  # the J^T J v instantiation of k_ray, FP32 parameters
COPY_TAGS = ("Mul",)  # the calibration copy: b = a * 1 (reads and writes copy-mib MiB)
KERNELS = {"k_ray<3, 0>": "jtj", "k_ray<4, 0>": "grad", "k_features": "feat", "k_mlp_infer": "mlp_infer",
           "k_mlp_train": "mlp_train"}


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def run(args):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import perf_synth as ps
    from paper_2112_05598_amd.scene import Scene, mlp_feature_stats, mlp_train_step
    from paper_2112_05598_amd import learned
    w = ps.workload(args.workload)
    dev = torch.device("cuda:0")
    sc = Scene(w.spec, w.cams, None, device="cuda:0", learned=True)
    H, _ = sc.render_residuals(torch.from_numpy(w.x_gt).to(dev))
    targets = H.clone()
    sc.set_targets(targets)
    x = torch.from_numpy(w.x_init).to(dev)
    v = torch.from_numpy(ps.random_vector(sc.n_params, 1)).to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    timing = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        ev[0].record()
        out = fn()
        ev[1].record()
        torch.cuda.synchronize()
        timing[name] = ev[0].elapsed_time(ev[1])
        print(f"[profile] {name}: {timing[name]:.3f} ms", flush=True)
        return out

    for i in range(args.launches):
        timed("jtj_ms", lambda: sc.apply_JtJ(x, v))
    timed("grad_ms", lambda: sc.build_precond(x, "none"))
    feat, blocks = timed("features_ms", lambda: sc.features(x))
    rows_f, rows_b, _ = sc.training_rows(feat, blocks, 1, 0.05, 200000)
    norm = mlp_feature_stats(rows_f)
    model = learned.load_model(device="cuda:0") if os.path.exists(learned.WEIGHTS) else None
    if model is None:
        import numpy as np
        wbf = torch.from_numpy(learned.init_weights(0).astype(np.float32)).to(dev).to(torch.bfloat16)
        model = learned.Model(wbf, norm)
    model.install(sc)
    timed("mlp_infer_ms", lambda: sc.mlp_infer(feat, blocks))
    timing["units"] = sc.n_units
    n = min(16384, rows_f.shape[0])
    w32 = model.w_bf16.float().clone()
    wbf = model.w_bf16.clone()
    m, vv, g = torch.zeros_like(w32), torch.zeros_like(w32), torch.zeros_like(w32)
    loss = torch.zeros(1, device=dev)
    fb, bb = rows_f[:n].contiguous(), rows_b[:n].contiguous()
    for t in range(1, 5):
        timed("mlp_train_ms", lambda: mlp_train_step(w32, wbf, m, vv, t, 1e-4, norm, fb, bb, loss, g))
    timing["train_rows"] = n
    n_copy = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n_copy, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(f"[profile] calibration copy of {args.copy_mib} MiB done", flush=True)
    del a, b
    from measure import probe
    st = torch.cuda.current_stream(dev).cuda_stream
    # consecutive addresses (stride 1), then one 128-byte line per lane (stride 32); the
    # scattered probe dispatches reps = 2 so the two are told apart in the counter database
    for stride, n_probe, reps in ((1, 32 << 20, 4), (32, 8 << 20, 2)):
        y = torch.zeros(n_probe * stride, dtype=torch.float32, device=dev)
        probe.atomic_add(y.data_ptr(), n_probe, 1, stride, st)  # warm
        torch.cuda.synchronize()
        ev[2].record()
        probe.atomic_add(y.data_ptr(), n_probe, reps, stride, st)
        ev[3].record()
        torch.cuda.synchronize()
        ms = ev[2].elapsed_time(ev[3])
        assert float(y[0]) == reps + 1 and float(y[(n_probe - 1) * stride]) == reps + 1
        print(f"[profile] atomic probe, stride {stride}: {n_probe * reps} atomics in {ms:.3f} ms "
              f"({n_probe * reps / ms / 1e6:.2f} G atomics/s)", flush=True)
        timing[f"probe{stride}_ms"] = ms
        timing[f"probe{stride}_atomics"] = n_probe * reps
        del y
    if args.timing_json:
        with open(args.timing_json, "w") as f:
            json.dump(timing, f)


def _per_dispatch(db: str, counter: str):
    """{kernel name: (mean counter value per dispatch, dispatches)} from a rocprofv3 database."""
    con = sqlite3.connect(db)
    tables = [r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")]
    tab = next(t for t in tables if t.startswith("counters_collection"))
    cols = [r[1] for r in con.execute(f"pragma table_info('{tab}')")]
    rows = con.execute(f"select * from '{tab}'").fetchall()
    kn, cn, cv = cols.index("kernel_name"), cols.index("counter_name"), cols.index("value")
    did = next((cols.index(c) for c in ("dispatch_id", "correlation_id", "id") if c in cols), None)
    per = {}
    for r in rows:
        if r[cn] != counter:
            continue
        key = r[did] if did is not None else len(per)
        k = (r[kn], key)
        per[k] = per.get(k, 0.0) + float(r[cv])
    agg = {}
    for (name, _), val in per.items():
        s, c = agg.get(name, (0.0, 0))
        agg[name] = (s + val, c + 1)
    return {name: (s / c, c) for name, (s, c) in agg.items()}


def summarise(args):
    out = {"kernel_sha": kernel_sha(), "workload": args.workload, "copy_bytes": args.copy_mib * (1 << 20)}
    total = 0.0
    for counter, db in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        per = _per_dispatch(db, counter)
        jtj = [(n, v) for n, v in per.items() if JTJ_TAG in n]
        cp = [(n, v) for n, v in per.items() if any(t in n for t in COPY_TAGS) and JTJ_TAG not in n]
        if len(jtj) != 1 or not cp:
            raise SystemExit(f"{db}: expected one J^T J v kernel and a copy kernel, found {list(per)}")
        (jname, (jkib, jn)), = jtj
        cname, (ckib, _) = max(cp, key=lambda t: t[1][0])
        scale = out["copy_bytes"] / (ckib * 1024.0)  # known bytes of the copy / counted bytes
        b = jkib * 1024.0 * scale
        out[counter] = {"kib_per_dispatch": jkib, "dispatches": jn, "copy_kernel": cname, "copy_kib": ckib,
                        "scale": scale, "bytes_per_dispatch": b}
        total += b
        out["kernel"] = jname
    out["bytes_per_dispatch"] = total
    # the other profiled kernels' HBM bytes, scaled by the same calibration copy
    out["kernels"] = {}
    for counter, db in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        per = _per_dispatch(db, counter)
        scale = out[counter]["scale"]
        for kname, (kib, n) in per.items():
            short = next((v for k, v in KERNELS.items() if k in kname), None)
            if short is not None:
                out["kernels"].setdefault(short, {"kernel": kname})[counter] = kib * 1024.0 * scale
    if args.atomic and args.timing_json:
        tm = json.load(open(args.timing_json))
        per = _per_dispatch(args.atomic, "TCC_ATOMIC")
        jtj = [(n, v) for n, v in per.items() if JTJ_TAG in n]
        probe = [(n, v) for n, v in per.items() if "k_atomic_probe" in n]
        if len(jtj) != 1 or not probe:
            raise SystemExit(f"{args.atomic}: expected the J^T J v kernel and the probe, found {list(per)}")
        (_, (ja, _)), = jtj
        out["atomics"] = {"jtj_requests_per_dispatch": ja, "jtj_ms": tm["jtj_ms"],
                          "jtj_requests_per_s": ja / (tm["jtj_ms"] * 1e-3)}
        # per-dispatch request counts of the probe dispatches in launch order: warm-up and timed
        # pass of stride 1, then of stride 32 (_per_dispatch averages per kernel name, so read
        # the dispatches here one by one)
        con = sqlite3.connect(args.atomic)
        tab = next(r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")
                   if r[0].startswith("counters_collection"))
        cols = [r[1] for r in con.execute(f"pragma table_info('{tab}')")]
        did = next(c for c in ("dispatch_id", "correlation_id", "id") if c in cols)
        rows = con.execute(f"select {did}, sum(value) from '{tab}' where kernel_name like '%k_atomic_probe%' "
                           f"and counter_name = 'TCC_ATOMIC' group by {did} order by {did}").fetchall()
        if len(rows) != 4:
            raise SystemExit(f"{args.atomic}: expected 4 probe dispatches, found {len(rows)}")
        for (stride, idx) in ((1, 1), (32, 3)):
            req = float(rows[idx][1])
            ms = tm[f"probe{stride}_ms"]
            out["atomics"][f"probe{stride}"] = {"requests_per_dispatch": req, "ms": ms,
                                                "requests_per_s": req / (ms * 1e-3),
                                                "lanes_per_request": tm[f"probe{stride}_atomics"] / req}
        out["atomics"]["frac_of_scattered_probe"] = (out["atomics"]["jtj_requests_per_s"]
                                                     / out["atomics"]["probe32"]["requests_per_s"])
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def counters(args):
    """Every counter of the given databases, averaged per dispatch of each profiled kernel."""
    out = {"kernel_sha": kernel_sha(), "workload": args.workload, "kernels": {}}
    for db in args.db:
        con = sqlite3.connect(db)
        tab = next(r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")
                   if r[0].startswith("counters_collection"))
        names = [r[0] for r in con.execute(f"select distinct counter_name from '{tab}'")]
        for c in names:
            for kname, (val, disp) in _per_dispatch(db, c).items():
                short = next((v for k, v in KERNELS.items() if k in kname), None)
                if short is None:
                    continue
                out["kernels"].setdefault(short, {"kernel": kname})[c] = {"per_dispatch": val, "dispatches": disp}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


# peaks used by the report (MI355X): HBM bytes/s, dense bf16 MFMA flop/s, compute units, clock
HBM_PEAK = 8.0e12
BF16_PEAK = 2.5e15
N_CU, CLOCK_HZ = 256, 2.4e9
MFMA_FLOPS = 32 * 32 * 8 * 2  # one v_mfma_f32_32x32x8_bf16 wave instruction


def _trace_ms(csv_path: str):
    """{short kernel name: (calls, average ms)} from a rocprofv3 --stats kernel_stats.csv."""
    import csv
    out = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            short = next((v for k, v in KERNELS.items() if k in row["Name"]), None)
            if short is not None:
                out[short] = (int(row["Calls"]), float(row["AverageNs"]) * 1e-6)
    return out


def report(args):
    """Markdown tables of the kernel trace, the SQ counters and the HBM counters per kernel."""
    cnt = json.load(open(args.counters))
    trf = json.load(open(args.traffic))
    tr = _trace_ms(args.stats)
    if cnt["kernel_sha"] != trf["kernel_sha"]:
        raise SystemExit("counter and traffic summaries come from different kernel sources")
    lines = [f"Kernel source sha256[:16] = `{cnt['kernel_sha']}`, workload {cnt['workload']}.", "",
             "| kernel | calls | avg ms (trace) | VALU wave-instr | VALU issue share | LDS instr | "
             "LDS-wait share | VMEM rd instr | MFMA instr | HBM GB (counted) | HBM GB/s | % HBM peak |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for short in ("jtj", "grad", "feat", "mlp_infer", "mlp_train"):
        k = cnt["kernels"].get(short)
        if k is None or short not in tr:
            continue
        calls, ms = tr[short]
        v = lambda c: k[c]["per_dispatch"]
        valu_share = v("SQ_INSTS_VALU") / (N_CU * CLOCK_HZ * ms * 1e-3)
        lds_wait = v("SQ_WAIT_INST_LDS") / v("SQ_WAVE_CYCLES")
        hb = trf.get("kernels", {}).get(short, {})
        gb = (hb.get("FETCH_SIZE", 0.0) + hb.get("WRITE_SIZE", 0.0)) / 1e9
        gbs = gb / (ms * 1e-3)
        lines.append(f"| {short} | {calls} | {ms:.3f} | {v('SQ_INSTS_VALU'):.4g} | {valu_share:.3f} | "
                     f"{v('SQ_INSTS_LDS'):.4g} | {lds_wait:.3f} | {v('SQ_INSTS_VMEM_RD'):.4g} | "
                     f"{v('SQ_INSTS_MFMA'):.4g} | {gb:.3f} | {gbs:.1f} | {100 * gbs * 1e9 / HBM_PEAK:.1f} |")
    lines += ["", "MFMA kernels (bf16 32x32x8 MFMA, 16384 flop per wave instruction):", "",
              "| kernel | MFMA flop per dispatch | TFLOP/s | % of 2.5 PFLOP/s | VALU wave-instr per MFMA instr |",
              "|---|---|---|---|---|"]
    for short in ("mlp_infer", "mlp_train"):
        k = cnt["kernels"].get(short)
        if k is None or short not in tr:
            continue
        ms = tr[short][1]
        fl = k["SQ_INSTS_MFMA"]["per_dispatch"] * MFMA_FLOPS
        ratio = k["SQ_INSTS_VALU"]["per_dispatch"] / max(k["SQ_INSTS_MFMA"]["per_dispatch"], 1.0)
        lines.append(f"| {short} | {fl:.4g} | {fl / (ms * 1e-3) / 1e12:.2f} | "
                     f"{100 * fl / (ms * 1e-3) / BF16_PEAK:.2f} | {ratio:.1f} |")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="cfg2")
    r.add_argument("--launches", type=int, default=2)
    r.add_argument("--copy-mib", type=int, default=2048)
    r.add_argument("--timing-json", default="")
    s = sub.add_parser("summarise")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--workload", default="cfg2")
    s.add_argument("--copy-mib", type=int, default=2048)
    s.add_argument("--out", required=True)
    s.add_argument("--atomic", default="")
    s.add_argument("--timing-json", default="")
    c = sub.add_parser("counters")
    c.add_argument("--db", action="append", required=True)
    c.add_argument("--workload", default="cfg2")
    c.add_argument("--out", required=True)
    q = sub.add_parser("report")
    q.add_argument("--counters", required=True)
    q.add_argument("--traffic", required=True)
    q.add_argument("--stats", required=True, help="rocprofv3 --stats kernel_stats.csv")
    q.add_argument("--out", default="")
    args = ap.parse_args()
    {"run": run, "summarise": summarise, "counters": counters, "report": report}[args.cmd](args)


if __name__ == "__main__":
    main()
