"""Train the learned block preconditioner on seeded scenes and evaluate it.

  python -m paper_2112_05598_amd.train_learned --train 10000:10032 --eval 20000:20002 --damp 0,0.3 --out DIR

One network per damping value, all on the same data.  Writes DIR/precond_mlp_bf16_d<damp>.npy
(packed bfloat16 weights, uint16 bits), DIR/precond_mlp_f32_d<damp>.npy and DIR/report.json
(loss histories; PCG iterations and milliseconds to a relative residual of 1e-3 for Jacobi,
exact block-Jacobi and each learned inverse on the held-out seeds).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import perf_synth as ps  # noqa: E402
from paper_2112_05598_amd import learned  # noqa: E402


def seeds(spec: str):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="10000:10032")
    ap.add_argument("--eval", default="20000:20002")
    ap.add_argument("--gn-steps", type=int, default=5)
    ap.add_argument("--per-step", type=int, default=65536)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--rel-tol", type=float, default=1e-3)
    ap.add_argument("--damp", default="0,0.3")
    ap.add_argument("--max-iters", type=int, default=200)
    ap.add_argument("--weights", default="",
                    help="evaluate these networks instead of training: name=path.npy[,name=path.npy]")
    ap.add_argument("--table-steps", default="2,3,4", help="GN steps of the per-step iteration table")
    ap.add_argument("--gn-eval", default="20000:20005", help="held-out seeds of the GN time-to-F comparison")
    ap.add_argument("--gn-steps-eval", type=int, default=5)
    ap.add_argument("--gn-pcg", type=int, default=30)
    ap.add_argument("--out", default="learned_out")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    report = {"train_seeds": args.train, "eval_seeds": args.eval, "gn_eval_seeds": args.gn_eval,
              "rel_tol": args.rel_tol, "max_iters": args.max_iters}
    nets = {}
    if args.weights:
        for item in args.weights.split(","):
            name, path = item.split("=")
            nets[name] = learned.load_weights(path)
    else:
        train_w = [ps.workload("cfg4", seed=s) for s in seeds(args.train)]
        feat, blocks = learned.generate(train_w, gn_steps=args.gn_steps, per_step=args.per_step, log=log)
        log(f"[learned] {feat.shape[0]} training samples in {time.time() - t0:.0f} s")
        hists = {}
        for damp in [float(s) for s in args.damp.split(",")]:
            t1 = time.time()
            w32, wbf, hist = learned.train(feat, blocks, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                           damp=damp, log=log)
            log(f"[learned] damp {damp}: trained in {time.time() - t1:.0f} s")
            bits = wbf.view(torch.int16).cpu().numpy().view(np.uint16)
            np.save(os.path.join(args.out, f"precond_mlp_bf16_d{damp:g}.npy"), bits)
            np.save(os.path.join(args.out, f"precond_mlp_f32_d{damp:g}.npy"), w32.cpu().numpy())
            nets[f"learned_d{damp:g}"] = wbf
            hists[f"learned_d{damp:g}"] = hist
        report.update({"gn_steps": args.gn_steps, "samples_per_step": args.per_step, "samples": int(feat.shape[0]),
                       "epochs": args.epochs, "lr": args.lr, "batch": args.batch, "loss": hists})
        del feat, blocks
        torch.cuda.empty_cache()
    gn_rows = [learned.gn_compare(ps.workload("cfg4", seed=s), nets, n_steps=args.gn_steps_eval,
                                  pcg_iters=args.gn_pcg, log=log) for s in seeds(args.gn_eval)]
    report["gn_compare"] = gn_rows
    steps = tuple(int(v) for v in args.table_steps.split(",")) if args.table_steps else ()
    if steps:
        eval_w = [ps.workload("cfg4", seed=s) for s in seeds(args.eval)]
        report["table"] = learned.evaluate(eval_w, nets, rel_tol=args.rel_tol, gn_steps=steps,
                                           max_iters=args.max_iters, log=log)
    report["seconds"] = time.time() - t0
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    log(f"[learned] done in {report['seconds']:.0f} s")


if __name__ == "__main__":
    main()
