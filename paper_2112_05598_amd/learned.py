"""Training and evaluation driver of the learned block preconditioner.

Training data: exact 4x4 blocks of J^T J and per-unit features computed by the library
along Gauss-Newton trajectories (Jacobi-preconditioned steps 1..5) of seeded scenes of the
128^3 object-in-a-box kind; a random subsample of the units that some ray touches per
(scene, step).  Training runs the library's MFMA forward/backward kernel and Adam.
Evaluation counts PCG iterations to a relative residual of 1e-3 on held-out seeds.
"""
from __future__ import annotations

import time
from typing import List

import numpy as np
import torch

from . import abi
from .scene import Scene, mlp_train_step


def init_weights(seed: int = 0) -> np.ndarray:
    """He-style initialisation (float64, packed order); the network starts at L = I."""
    rng = np.random.default_rng(seed)
    nh, ni, nip, no, nop = 64, 12, 16, 10, 16
    W1 = rng.normal(0, np.sqrt(2.0 / ni), (nh, nip)); W1[:, ni:] = 0.0
    W2 = rng.normal(0, np.sqrt(2.0 / nh), (nh, nh))
    W3 = 0.1 * rng.normal(0, np.sqrt(1.0 / nh), (nop, nh)); W3[no:, :] = 0.0
    b3 = np.zeros(nop); b3[[0, 2, 5, 9]] = 0.5413  # softplus^-1(1)
    return np.concatenate([W1.ravel(), np.zeros(nh), W2.ravel(), np.zeros(nh), W3.ravel(), b3])


def scene_for(workload, device="cuda:0", learned=True):
    sc = Scene(workload.spec, workload.cams, None, learned=learned, device=device)
    x_gt = torch.from_numpy(workload.x_gt).to(sc.device)
    H, _ = sc.render_residuals(x_gt)
    targets = H.clone()
    sc.set_targets(targets)
    sc._keep_targets = targets
    return sc


def generate(workloads, gn_steps=5, per_step=65536, pcg_iters=5, seed=0, log=print):
    """Features and blocks along Jacobi-GN trajectories: list of (feat, blocks) GPU tensors."""
    rng = np.random.default_rng(seed)
    feats, blocks = [], []
    for w in workloads:
        sc = scene_for(w)
        x = torch.from_numpy(w.x_init).to(sc.device)
        for step in range(gn_steps):
            f, b = sc.features(x)
            live = torch.nonzero(torch.maximum(b[:, 0], b[:, 4]) > 0).squeeze(1)
            pick = torch.from_numpy(rng.choice(live.numel(), min(per_step, live.numel()), replace=False)).to(
                sc.device)
            feats.append(f[live[pick]].clone())
            blocks.append(b[live[pick]].clone())
            sc.gn_step(x, max_iters=pcg_iters, precond="jacobi")
        log(f"[learned] data from seed {w.seed}: {sum(t.shape[0] for t in feats)} samples")
        del sc
        torch.cuda.empty_cache()
    return torch.cat(feats), torch.cat(blocks)


def train(feat, blocks, epochs=4, batch=16384, lr=2e-3, seed=0, log=print):
    dev = feat.device
    w32 = torch.from_numpy(init_weights(seed).astype(np.float32)).to(dev)
    wbf = w32.to(torch.bfloat16)
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
    grad = torch.zeros_like(w32)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    n = feat.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    t = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            t += 1
            fb = feat[idx].contiguous()
            bb = blocks[idx].contiguous()
            mlp_train_step(w32, wbf, m, v, t, lr, fb, bb, loss, grad)
            tot += loss.item()
            cnt += 1
        hist.append(tot / max(cnt, 1))
        log(f"[learned] epoch {ep}: mean loss {hist[-1]:.5f}")
    return w32, wbf, hist


def pcg_iterations(sc: Scene, x, precond: str, rel_tol=1e-3, max_iters=256):
    st = sc.gn_step(x.clone(), max_iters=max_iters, precond=precond, rel_tol=rel_tol)
    return st["pcg_iters"], st


def evaluate(workloads, wbf, rel_tol=1e-3, gn_steps=(0, 2), log=print) -> List[dict]:
    """PCG iterations and wall time to sqrt(R/R0) <= rel_tol for Jacobi, block and learned M."""
    out = []
    for w in workloads:
        sc = scene_for(w)
        sc.mlp_set_weights(wbf)
        x = torch.from_numpy(w.x_init).to(sc.device)
        for step in range(max(gn_steps) + 1):
            if step in gn_steps:
                row = {"seed": w.seed, "gn_step": step}
                for pc in ("jacobi", "block", "learned"):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    it, st = pcg_iterations(sc, x, pc, rel_tol)
                    torch.cuda.synchronize()
                    row[pc] = {"iters": it, "ms": (time.perf_counter() - t0) * 1e3, "F_after": st["F_after"],
                               "converged": bool(st["flags"] & abi.PERF_FLAG_CONVERGED)}
                out.append(row)
                log(f"[learned] seed {w.seed} step {step}: " +
                    ", ".join(f"{pc} {row[pc]['iters']} it {row[pc]['ms']:.0f} ms" for pc in ("jacobi", "block",
                                                                                            "learned")))
            sc.gn_step(x, max_iters=5, precond="jacobi")
        del sc
        torch.cuda.empty_cache()
    return out
