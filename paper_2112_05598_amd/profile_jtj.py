"""Profiling driver for the J^T J v kernel and its HBM-traffic summary.

  run:        python -m paper_2112_05598_amd.profile_jtj run --workload cfg2 --launches 3 --copy-mib 2048
  summarise:  python -m paper_2112_05598_amd.profile_jtj summarise --fetch F.db --write W.db --out traffic.json

`run` launches the library's J^T J v product `--launches` times on the named workload (at the
initial parameters, with a seeded random v), then one plain device-to-device copy of
`--copy-mib` MiB (an elementwise b = a * 1) as the calibration kernel.  Run it under `rocprofv3 --pmc FETCH_SIZE` and,
separately, under `rocprofv3 --pmc WRITE_SIZE`.

`summarise` reads the two rocprofv3 result databases, averages each counter per dispatch of the
J^T J v kernel, scales it by (known copy bytes / counted copy bytes) of the calibration copy,
and writes the HBM bytes per dispatch together with the sha256 of the kernel source they
were measured on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2112_05598_amd", "csrc", "raymarch.hip")
JTJ_TAG = "k_ray<3, 0>"  # the J^T J v instantiation of k_ray, FP32 parameters
COPY_TAGS = ("Mul",)  # the calibration copy: b = a * 1 (reads and writes copy-mib MiB)


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def run(args):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import perf_synth as ps
    from paper_2112_05598_amd.scene import Scene
    w = ps.workload(args.workload)
    dev = torch.device("cuda:0")
    sc = Scene(w.spec, w.cams, None, device="cuda:0")
    x = torch.from_numpy(w.x_init).to(dev)
    v = torch.from_numpy(ps.random_vector(sc.n_params, 1)).to(dev)
    for i in range(args.launches):
        sc.apply_JtJ(x, v)
        torch.cuda.synchronize()
        print(f"[profile] J^T J v launch {i + 1}/{args.launches} done", flush=True)
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(f"[profile] calibration copy of {args.copy_mib} MiB done", flush=True)


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
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="cfg2")
    r.add_argument("--launches", type=int, default=3)
    r.add_argument("--copy-mib", type=int, default=2048)
    s = sub.add_parser("summarise")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--workload", default="cfg2")
    s.add_argument("--copy-mib", type=int, default=2048)
    s.add_argument("--out", required=True)
    args = ap.parse_args()
    run(args) if args.cmd == "run" else summarise(args)


if __name__ == "__main__":
    main()
