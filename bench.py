"""Benchmark: Gauss-Newton steps (PCG with J^T J v) on one MI355X.

One step = one Gauss-Newton step of the whole path: the gradient and exact 4x4 blocks
of J^T J in one traversal, the preconditioner, PCG (30 products J^T J v), the
backtracking line search (full renders of the objective) and the projected update.

Workload: the 128^3 object-in-a-box scene (40 seeded spheres/boxes, 3 environment
layers of 256x128 at radii 1.8/3/6, 100 cameras of 400x400 on the upper hemisphere at
radius 4: 16 M rays).  Targets are rendered by the library from the ground-truth
parameters; the solve starts from grey colour 0.5, opacity 0.01.

value = rays pushed through J^T J v per second of whole-step wall time (every other
part of the step counts as overhead).  The roofline object prices the J^T J v kernel
alone: footprint bytes per launch (48 B per distinct voxel a ray touches + 192 B per
environment layer it hits, 40 B and 160 B with bf16 parameter storage, counted exactly by
the library's footprint pass) over the
kernel's average duration measured with HIP events on the launch stream.  Beside it,
counted_hbm_gbs is the HBM traffic rocprofv3 counted for the same kernel source
(profiles/jtj_cfg2_traffic.json) over the same duration: what actually crosses HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jtj_cfg2_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2112_05598_amd", "csrc", "raymarch.hip")


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per J^T J v launch from committed rocprofv3 counters, if they were taken on
    the current kernel source and this workload; None otherwise."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_sha() or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_dispatch")


def cpu_baseline(w, min_seconds: float = 10.0):
    """The FP64 oracle's J^T J v on a strided sample of the same rays, on the host cores.

    A call has a fixed cost (per-thread FP64 accumulators of P doubles, summed at the end), so
    the sample grows until one call takes at least min_seconds (or covers every ray)."""
    import numpy as np
    import oracle
    orc = oracle.OracleScene(w.spec, w.cams)
    v = np.random.default_rng(7).normal(size=orc.n_params)
    x = w.x_init.astype(np.float64)
    n = 16384
    while True:
        stride = max(orc.n_rays // n, 1)
        sample = np.arange(0, orc.n_rays, stride, dtype=np.int64)
        t0 = time.perf_counter()
        orc.apply_JtJ(x, v, rays=sample)
        dt = time.perf_counter() - t0
        print(f"[bench] oracle: {len(sample)} rays in {dt:.1f} s", file=sys.stderr, flush=True)
        if dt >= min_seconds or stride == 1:
            break
        n = int(len(sample) * min(8.0, 1.5 * min_seconds / max(dt, 1e-3)))
    return {"value": len(sample) / dt, "unit": "rays/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"J^T J v over every {stride}-th ray ({len(sample)} of {orc.n_rays} rays) at the initial "
                      f"parameters, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--pcg", type=int, default=30)
    ap.add_argument("--precond", default="jacobi")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--jitter", type=int, default=0,
                    help="jitter seed base (Sec. IV); each GN step uses base + step index; 0 = off")
    ap.add_argument("--aux", type=float, default=0.0,
                    help="weight of the auxiliary opacity residual (Eq. 10; the paper uses 0.1), 0 = off")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-preconditioner GN run to the Jacobi run's final objective")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding the rays over GPUs "
              "is a design, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import perf_synth as ps
    from paper_2112_05598_amd.scene import Scene

    dev = torch.device("cuda:0")
    w = ps.workload(args.workload)
    print(f"[bench] workload {w.name}: grid {w.spec.nx}^3, {w.spec.n_layers} layers {w.spec.env_w}x{w.spec.env_h}, "
          f"{w.cams.n} cams {w.cams.width}x{w.cams.height}, P={w.spec.n_params}", file=sys.stderr, flush=True)
    sc = Scene(w.spec, w.cams, None, param_dtype="f32", learned=not args.no_learned, device="cuda:0",
               aux_lambda=args.aux)
    x_gt = torch.from_numpy(w.x_gt).to(dev)
    H, _ = sc.render_residuals(x_gt)           # no targets yet: the render itself
    targets = H.clone()
    sc.set_targets(targets)
    if args.dtype == "bf16":
        sc = Scene(w.spec, w.cams, targets, param_dtype="bf16", learned=not args.no_learned, device="cuda:0",
                   aux_lambda=args.aux)
    _, tot = sc.footprint(per_ray=False)
    tot = tot.cpu().numpy()
    # per distinct voxel: x (16 B, or 8 B stored as bf16) + v (16 B) + y (16 B); per layer hit: 4 texels
    per_unit = 48.0 if args.dtype == "f32" else 40.0
    bytes_per_launch = per_unit * float(tot[0]) + 4.0 * per_unit * float(tot[1])

    x0 = torch.from_numpy(w.x_init).to(dev)
    opts = dict(max_iters=args.pcg, precond=args.precond)
    xw = x0.clone()
    for i in range(args.warmup):
        if args.jitter:
            sc.set_jitter(args.jitter + 1000 + i)
        sc.gn_step(xw, **opts)
        print(f"[bench] warmup step {i} done", file=sys.stderr, flush=True)
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        if args.jitter:
            sc.set_jitter(args.jitter + i)
        st = sc.gn_step(x, **opts)
        stats.append(st)
        print(f"[bench] step {i}: F {st['F_before']:.6g} -> {st['F_after']:.6g} gamma {st['gamma']:.3g} "
              f"pcg {st['pcg_iters']} ls {st['ls_trials']} {st['ms_phase'][5]:.1f} ms "
              f"(jtj {st['ms_jtj'] / max(st['n_jtj'], 1):.2f} ms avg)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    n_jtj = sum(s["n_jtj"] for s in stats)
    jtj_ms = sum(s["ms_jtj"] for s in stats) / max(n_jtj, 1)
    value = sc.n_rays * n_jtj / dt
    achieved = bytes_per_launch / (jtj_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": "J^T J.v rays/s (% HBM roofline); GN time-to-residual, learned vs Jacobi PCG",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.spec.nx}^3 RGB-sigma grid, {w.spec.n_layers} env layers "
                               f"{w.spec.env_w}x{w.spec.env_h} at radii {list(w.spec.layer_radii)}, {w.cams.n} cams "
                               f"{w.cams.width}x{w.cams.height} on the upper hemisphere r=4, 40 random spheres/boxes",
                   "rays": sc.n_rays, "params": sc.n_params, "pcg_iters_per_step": args.pcg,
                   "precond": args.precond, "step_vox": w.spec.step_vox, "aux_lambda": args.aux,
                   "jitter": args.jitter},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_ray<M_JTJ> (J^T J v)", "avg_launch_ms": jtj_ms,
                     "bytes_per_launch": bytes_per_launch, "achieved_basis": "footprint (algorithmic) bytes",
                     "counted_hbm_gbs": None if traffic is None else traffic / (jtj_ms * 1e-3) / 1e9,
                     "launches": n_jtj, "kernel_rays_per_s": sc.n_rays / (jtj_ms * 1e-3)},
        "gn": {"F": [stats[0]["F_before"]] + [s["F_after"] for s in stats],
               "ms_per_gn_step": [s["ms_phase"][5] for s in stats],
               "pcg_iters": [s["pcg_iters"] for s in stats], "gamma": [s["gamma"] for s in stats]},
        "footprint": {"sum_U": int(tot[0]), "layer_hits": int(tot[1]), "rays_in_grid": int(tot[2])},
    }
    from paper_2112_05598_amd import learned as lrn
    if not args.no_learned and args.precond == "jacobi" and not os.path.exists(lrn.WEIGHTS):
        print(f"[bench] no learned weights at {lrn.WEIGHTS}: learned comparison skipped", file=sys.stderr, flush=True)
        out["gn_learned_vs_jacobi"] = None
    elif not args.no_learned and args.precond == "jacobi":
        # GN time-to-residual: the learned preconditioner, from the same start, until it reaches
        # the objective the timed Jacobi steps ended at (same PCG iterations per step)
        model = lrn.load_model(device="cuda:0")
        model.install(sc)
        F_target = stats[-1]["F_after"]
        run = lrn.gn_run(sc, x0, "learned", args.steps + 3, args.pcg, F_stop=F_target)
        del run["x"]
        frac = [lrn.fallback_fraction(sc, x0), lrn.fallback_fraction(sc, x)]
        print(f"[bench] learned: {run['gn_steps']} GN steps, {run['pcg_iters']} PCG iterations, "
              f"{run['ms']:.0f} ms to F {run['F'][-1]:.6g} (Jacobi: {args.steps} steps, "
              f"{sum(s['pcg_iters'] for s in stats)} iterations, {dt * 1e3:.0f} ms to F {F_target:.6g})",
              file=sys.stderr, flush=True)
        out["gn_learned_vs_jacobi"] = {
            "target_F": F_target,
            "jacobi": {"gn_steps": args.steps, "pcg_iters": sum(s["pcg_iters"] for s in stats), "ms": dt * 1e3},
            "learned": {"gn_steps": run["gn_steps"], "pcg_iters": run["pcg_iters"], "ms": run["ms"],
                        "F": run["F"], "reached": run["F"][-1] <= F_target,
                        "q_fallback": model.q_fallback if math.isfinite(model.q_fallback) else None,
                        "fallback_frac_start_end": frac},
            "model": "paper_2112_05598_amd/weights/precond_mlp.npz"}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a ray sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
