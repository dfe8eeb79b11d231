"""Hierarchical (coarse-to-fine) Gauss-Newton, Sec. IV (hierarchical formulation).

The grid and the environment layers double their resolution in every dimension from one
level to the next; each level runs a fixed number of Gauss-Newton steps, and the next level
starts from the result interpolated by perf_upsample.  The images (targets and cameras) are
the same at every level.  Host control flow only: every step runs in the library's kernels.

  python -m paper_2112_05598_amd.hierarchy --workload cfg2 --levels 3 --steps 5 --pcg 30
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time
from typing import List, Sequence

import numpy as np
import torch

from .scene import Scene, upsample


def level_specs(spec, levels: int) -> List:
    """Specs from the coarsest to the finest (= spec): dimensions halved per level below it."""
    out = []
    for k in range(levels - 1, -1, -1):
        f = 2 ** k
        if spec.nx % f or spec.ny % f or spec.nz % f or spec.env_w % f or spec.env_h % f:
            raise ValueError(f"{levels} levels need grid and layer sizes divisible by {f}")
        out.append(dataclasses.replace(spec, nx=spec.nx // f, ny=spec.ny // f, nz=spec.nz // f,
                                       env_w=spec.env_w // f, env_h=spec.env_h // f))
    return out


def gn_hierarchy(spec, cams, targets: torch.Tensor, x0: torch.Tensor, levels: int, steps: Sequence[int],
                 pcg_iters: int = 30, precond: str = "jacobi", weights=None, F_stop: float = -1.0, log=print,
                 jitter_base: int = 0):
    """Run the levels; x0 is the coarsest level's start.  Returns the finest x and one record per
    GN step (level, F before/after, PCG iterations, cumulative wall time in ms).  jitter_base != 0
    jitters the samples (Sec. IV) with seed jitter_base + (GN step count) for each step."""
    specs = level_specs(spec, levels)
    if len(steps) != levels:
        raise ValueError("one step count per level")
    x = x0.clone()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, sp in enumerate(specs):
        if k > 0:
            x = upsample(specs[k - 1], x, sp)
        sc = Scene(sp, cams, targets, learned=precond == "learned", device=str(targets.device))
        if precond == "learned":
            weights.install(sc)
        for _ in range(steps[k]):
            if jitter_base:
                sc.set_jitter(jitter_base + len(recs))
            st = sc.gn_step(x, max_iters=pcg_iters, precond=precond)
            torch.cuda.synchronize()
            recs.append({"level": k, "grid": sp.nx, "F_before": st["F_before"], "F_after": st["F_after"],
                         "pcg_iters": st["pcg_iters"], "flags": st["flags"], "ms": (time.perf_counter() - t0) * 1e3})
            log(f"[hierarchy] level {k} ({sp.nx}x{sp.ny}x{sp.nz}, layers {sp.env_w}x{sp.env_h}): "
                f"F {st['F_before']:.6g} -> {st['F_after']:.6g}")
            if F_stop >= 0 and k == levels - 1 and st["F_after"] <= F_stop:
                break
        del sc
    return x, recs


def main():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import perf_synth as ps
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--steps", type=int, default=5, help="GN steps per level")
    ap.add_argument("--pcg", type=int, default=30)
    ap.add_argument("--precond", default="jacobi")
    ap.add_argument("--jitter", type=int, default=0, help="jitter seed base (0 = off)")
    ap.add_argument("--psnr-views", type=int, default=0,
                    help="held-out views (seeded, same camera rig) for PSNR of the flat and hierarchical results")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    w = ps.workload(args.workload)
    dev = torch.device("cuda:0")
    ref = Scene(w.spec, w.cams, None, device="cuda:0")
    H, _ = ref.render_residuals(torch.from_numpy(w.x_gt).to(dev))
    targets = H.clone()
    ref.set_targets(targets)
    weights = None
    if args.precond == "learned":
        from .learned import load_model
        weights = load_model(device="cuda:0")
    # flat: the finest level only, from the initial guess
    x = torch.from_numpy(w.x_init).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flat = []
    for _ in range(args.steps):
        st = ref.gn_step(x, max_iters=args.pcg, precond="jacobi" if args.precond == "learned" else args.precond)
        torch.cuda.synchronize()
        flat.append({"F_after": st["F_after"], "ms": (time.perf_counter() - t0) * 1e3})
        log(f"[flat] F {st['F_before']:.6g} -> {st['F_after']:.6g}")
    x_flat = x
    del ref
    torch.cuda.empty_cache()
    # hierarchical: coarse-to-fine from the coarsest level's initial guess
    specs = level_specs(w.spec, args.levels)
    x0 = torch.from_numpy(ps.init_params(specs[0])).to(dev)
    x_hier, recs = gn_hierarchy(w.spec, w.cams, targets, x0, args.levels, [args.steps] * args.levels, args.pcg,
                                args.precond, weights, log=log, jitter_base=args.jitter)
    quality = None
    if args.psnr_views:
        from .render import psnr, render_scene
        held = ps.make_cameras("hemisphere", args.psnr_views, w.cams.width, w.cams.height, 40.0, 4.0,
                               np.random.default_rng(12345))
        gt = render_scene(w.spec, held, None, threshold=0.0)
        images, _ = gt.render_residuals(torch.from_numpy(w.x_gt).to(dev))
        images = images.clone()
        del gt
        quality = {"views": args.psnr_views, "psnr_flat": psnr(x_flat, w.spec, held, images),
                   "psnr_hierarchy": psnr(x_hier, w.spec, held, images),
                   "psnr_init": psnr(torch.from_numpy(w.x_init).to(dev), w.spec, held, images)}
        log(f"[hierarchy] held-out PSNR: init {quality['psnr_init']:.2f} dB, flat {quality['psnr_flat']:.2f} dB, "
            f"hierarchical {quality['psnr_hierarchy']:.2f} dB")
    target = flat[-1]["F_after"]
    hit = next((r for r in recs if r["level"] == args.levels - 1 and r["F_after"] <= target), None)
    print(json.dumps({"workload": args.workload, "levels": [s.nx for s in specs], "steps_per_level": args.steps,
                      "pcg_iters": args.pcg, "precond": args.precond, "flat": flat, "hierarchy": recs,
                      "flat_final_F": target, "hierarchy_reaches_flat_F_at_ms": hit["ms"] if hit else None,
                      "jitter": args.jitter, "quality": quality}))


if __name__ == "__main__":
    main()
