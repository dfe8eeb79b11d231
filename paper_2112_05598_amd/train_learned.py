"""Train the learned block preconditioner on seeded scenes and evaluate it.

  python -m paper_2112_05598_amd.train_learned --train 10000:10200 --long 10000:10020 --out DIR

A run can be split over several processes: --save-state writes the training state (weights,
Adam moments, step count, standardisation) and --init-state continues from it on the next
chunk of seeds (--no-eval skips the evaluation of an intermediate chunk).

Training data: features and exact blocks at Gauss-Newton steps 0..gn_steps-1 of every --train
seed, plus steps gn_steps..long_steps-1 of the --long seeds (longer trajectories, so that
later GN steps are covered).  One network per damping value, all on the same data; each is
evaluated with every --fallback threshold.  Writes DIR/precond_mlp_d<damp>.npz (weights,
standardisation, fallback threshold) and DIR/report.json (loss histories; GN time to the
Jacobi run's objective at the given horizon on the held-out seeds, with exact block-Jacobi
beside it; PCG iterations to a relative residual of 1e-3 per GN step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import perf_synth as ps  # noqa: E402
from paper_2112_05598_amd import learned  # noqa: E402


def seeds(spec: str):
    if not spec:
        return []
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="10000:10200")
    ap.add_argument("--gn-steps", type=int, default=5)
    ap.add_argument("--pcg-data", type=int, default=5, help="PCG iterations per GN step of the data trajectories")
    ap.add_argument("--long", default="10000:10020", help="seeds whose trajectories run to --long-steps")
    ap.add_argument("--long-steps", type=int, default=20)
    ap.add_argument("--long-pcg", type=int, default=10)
    ap.add_argument("--per-step", type=int, default=65536)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--damp", default="0")
    ap.add_argument("--fallback", default="inf,8,4,2", help="fallback thresholds q to evaluate")
    ap.add_argument("--models", default="", help="evaluate these models instead of training: name=path.npz[,...]")
    ap.add_argument("--gn-eval", default="20000:20003", help="held-out seeds of the GN time-to-F comparison")
    ap.add_argument("--gn-steps-eval", type=int, default=20)
    ap.add_argument("--gn-pcg", type=int, default=30)
    ap.add_argument("--table", default="20000:20002", help="held-out seeds of the iterations-to-1e-3 table")
    ap.add_argument("--table-steps", default="2,6,12")
    ap.add_argument("--rel-tol", type=float, default=1e-3)
    ap.add_argument("--max-iters", type=int, default=200)
    ap.add_argument("--init-state", default="", help="continue training from this state (.npz)")
    ap.add_argument("--save-state", default="", help="write the training state here (.npz)")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--out", default="learned_out")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    report = {"train_seeds": args.train, "long_seeds": args.long, "gn_eval_seeds": args.gn_eval,
              "table_seeds": args.table, "rel_tol": args.rel_tol, "max_iters": args.max_iters}
    trained = {}
    if args.models:
        for item in args.models.split(","):
            name, path = item.split("=")
            trained[name] = learned.load_model(path)
    else:
        parts = []
        if args.train:
            parts.append(learned.generate([ps.workload("cfg4", seed=s) for s in seeds(args.train)],
                                          gn_steps=args.gn_steps, per_step=args.per_step, pcg_iters=args.pcg_data,
                                          log=log))
        if args.long and args.long_steps > args.gn_steps:
            parts.append(learned.generate([ps.workload("cfg4", seed=s) for s in seeds(args.long)],
                                          gn_steps=args.long_steps, first_step=args.gn_steps,
                                          per_step=args.per_step, pcg_iters=args.long_pcg, log=log))
        feat = torch.cat([p[0] for p in parts])
        blocks = torch.cat([p[1] for p in parts])
        del parts
        log(f"[learned] {feat.shape[0]} training samples in {time.time() - t0:.0f} s")
        hists = {}
        for damp in [float(v) for v in args.damp.split(",")]:
            t1 = time.time()
            init = learned.load_state(args.init_state) if args.init_state else None
            state, model, hist = learned.train(feat, blocks, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                               damp=damp, log=log, state=init)
            if args.save_state:
                learned.save_state(args.save_state, state)
            log(f"[learned] damp {damp}: trained in {time.time() - t1:.0f} s")
            trained[f"d{damp:g}"] = model
            hists[f"d{damp:g}"] = hist
        report.update({"gn_steps": args.gn_steps, "long_steps": args.long_steps, "samples_per_step": args.per_step,
                       "samples": int(feat.shape[0]), "epochs": args.epochs, "lr": args.lr, "batch": args.batch,
                       "loss": hists})
        del feat, blocks
        torch.cuda.empty_cache()
    if args.no_eval:
        for name, model in trained.items():
            learned.save_model(os.path.join(args.out, f"precond_mlp_{name}.npz"), model)
        report["seconds"] = time.time() - t0
        with open(os.path.join(args.out, "report.json"), "w") as f:
            json.dump(report, f, indent=1)
        log(f"[learned] chunk done in {report['seconds']:.0f} s")
        return
    nets = {}
    for name, model in trained.items():
        for q in [float(v) for v in args.fallback.split(",")]:
            nets[f"{name}_q{q:g}"] = learned.Model(model.w_bf16, model.norm, q)
    for name, model in nets.items():
        learned.save_model(os.path.join(args.out, f"precond_mlp_{name}.npz"), model)
    nets["block"] = None
    report["gn_compare"] = [learned.gn_compare(ps.workload("cfg4", seed=s), nets, n_steps=args.gn_steps_eval,
                                               pcg_iters=args.gn_pcg, log=log) for s in seeds(args.gn_eval)]
    steps = tuple(int(v) for v in args.table_steps.split(",")) if args.table_steps else ()
    if steps and args.table:
        table_nets = {k: v for k, v in nets.items() if v is not None}
        report["table"] = learned.evaluate([ps.workload("cfg4", seed=s) for s in seeds(args.table)], table_nets,
                                           rel_tol=args.rel_tol, gn_steps=steps, max_iters=args.max_iters, log=log)
    report["seconds"] = time.time() - t0
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    log(f"[learned] done in {report['seconds']:.0f} s")


if __name__ == "__main__":
    main()
