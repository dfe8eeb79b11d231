"""Training and evaluation code of the learned block preconditioner.

Training data: exact 4x4 blocks of J^T J and per-unit features computed by the library
along Gauss-Newton trajectories (Jacobi-preconditioned steps 1..5) of seeded scenes of the
128^3 object-in-a-box kind; a random subsample of the units that some ray touches per
(scene, step).  Training runs the library's MFMA forward/backward kernel and Adam.
Evaluation counts PCG iterations to a relative residual of 1e-3 on held-out seeds.
"""
from __future__ import annotations

import os
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
    W3 = np.zeros((nop, nh))  # start exactly at L = I: the Jacobi preconditioner
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


def fold_normalisation(w: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Weights trained on (feature - mu) / sd, rewritten for raw features: W1 / sd and
    b1 - W1 (mu / sd) on the 12 real inputs."""
    w = np.array(w, dtype=np.float64)
    nh, nip = 64, 16
    W1 = w[:nh * nip].reshape(nh, nip)
    b1 = w[nh * nip:nh * nip + nh]
    W1f = W1.copy()
    W1f[:, :12] = W1[:, :12] / sd[None, :]
    b1f = b1 - W1[:, :12] @ (mu / sd)
    w[:nh * nip] = W1f.ravel()
    w[nh * nip:nh * nip + nh] = b1f
    return w


def train(feat, blocks, epochs=4, batch=16384, lr=5e-4, seed=0, damp=0.0, log=print):
    """Adam on the library's training kernel towards the damped normalised inverse
    (B~ + damp I)^-1; features are standardised for training and the standardisation is
    folded into the first layer of the returned weights."""
    dev = feat.device
    mu = feat.mean(0)
    sd = feat.std(0).clamp_min(1e-3)
    feat = ((feat - mu) / sd).contiguous()
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
            mlp_train_step(w32, wbf, m, v, t, lr, fb, bb, loss, grad, damp=damp)
            tot += loss.item()
            cnt += 1
        hist.append(tot / max(cnt, 1))
        log(f"[learned] damp {damp} epoch {ep}: mean loss {hist[-1]:.5f}")
    wf = fold_normalisation(w32.cpu().numpy(), mu.cpu().numpy().astype(np.float64),
                            sd.cpu().numpy().astype(np.float64))
    w32 = torch.from_numpy(wf.astype(np.float32)).to(dev)
    wbf = w32.to(torch.bfloat16)
    return w32, wbf, hist


def pcg_iterations(sc: Scene, x, precond: str, rel_tol=1e-3, max_iters=256):
    st = sc.gn_step(x.clone(), max_iters=max_iters, precond=precond, rel_tol=rel_tol)
    return st["pcg_iters"], st


def evaluate(workloads, nets, rel_tol=1e-3, gn_steps=(1, 3), max_iters=200, log=print) -> List[dict]:
    """PCG iterations and wall time to sqrt(R/R0) <= rel_tol for Jacobi, exact block-Jacobi and
    each learned network of `nets` ({name: bf16 weights}), at the given steps of a Jacobi-GN
    trajectory from the initial parameters."""
    out = []
    for w in workloads:
        sc = scene_for(w)
        x = torch.from_numpy(w.x_init).to(sc.device)
        for step in range(max(gn_steps) + 1):
            if step in gn_steps:
                row = {"seed": w.seed, "gn_step": step}
                runs = [("jacobi", "jacobi", None), ("block", "block", None)]
                runs += [(name, "learned", wbf) for name, wbf in nets.items()]
                for name, pc, wbf in runs:
                    if wbf is not None:
                        sc.mlp_set_weights(wbf)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    it, st = pcg_iterations(sc, x, pc, rel_tol, max_iters)
                    torch.cuda.synchronize()
                    row[name] = {"iters": it, "ms": (time.perf_counter() - t0) * 1e3, "F_after": st["F_after"],
                                 "ms_precond": st["ms_phase"][1], "ms_pcg": st["ms_phase"][2],
                                 "converged": bool(st["flags"] & abi.PERF_FLAG_CONVERGED)}
                out.append(row)
                log(f"[learned] seed {w.seed} step {step}: " +
                    ", ".join(f"{name} {row[name]['iters']} it {row[name]['ms']:.0f} ms" for name, _, _ in runs))
            sc.gn_step(x, max_iters=5, precond="jacobi")
        del sc
        torch.cuda.empty_cache()
    return out


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "precond_mlp_bf16.npy")


def load_weights(path: str = WEIGHTS, device="cuda:0") -> torch.Tensor:
    """Packed bfloat16 weights (uint16 bits on disk) as a device bfloat16 tensor."""
    bits = np.load(path, allow_pickle=False)
    if bits.dtype != np.uint16 or bits.size != abi.PERF_MLP_NW:
        raise ValueError(f"{path}: expected {abi.PERF_MLP_NW} uint16 values")
    return torch.from_numpy(bits.view(np.int16).copy()).to(device).view(torch.bfloat16)


def gn_run(sc: Scene, x0, precond: str, n_steps: int, pcg_iters: int, rel_tol: float = 0.0,
           F_stop: float = -1.0) -> dict:
    """Gauss-Newton from x0 with the given preconditioner; stops after n_steps or once F <= F_stop.
    Wall time covers every step (preconditioner set-up, features and inference included)."""
    x = x0.clone()
    F, iters, F0 = [], 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        st = sc.gn_step(x, max_iters=pcg_iters, precond=precond, rel_tol=rel_tol)
        F0 = st["F_before"] if F0 is None else F0
        iters += st["pcg_iters"]
        F.append(st["F_after"])
        if F_stop >= 0 and st["F_after"] <= F_stop:
            break
    torch.cuda.synchronize()
    return {"F0": F0, "F": F, "pcg_iters": iters, "gn_steps": len(F), "ms": (time.perf_counter() - t0) * 1e3}


def gn_compare(w, nets, n_steps=5, pcg_iters=30, rel_tol=0.0, extra_steps=3, log=print) -> dict:
    """Jacobi-PCG GN for n_steps, then GN with each learned network of `nets` ({name: bf16
    weights}) until it reaches the Jacobi run's final F (at most n_steps + extra_steps), with the
    same PCG settings."""
    sc = scene_for(w)
    x0 = torch.from_numpy(w.x_init).to(sc.device)
    jac = gn_run(sc, x0, "jacobi", n_steps, pcg_iters, rel_tol)
    out = {"seed": w.seed, "pcg_iters_per_step": pcg_iters, "rel_tol": rel_tol, "jacobi": jac}
    msg = f"[learned] GN seed {w.seed}: jacobi {jac['pcg_iters']} it {jac['ms']:.0f} ms F {jac['F'][-1]:.6g}"
    for name, wbf in nets.items():
        sc.mlp_set_weights(wbf)
        r = gn_run(sc, x0, "learned", n_steps + extra_steps, pcg_iters, rel_tol, F_stop=jac["F"][-1])
        r["reached"] = r["F"][-1] <= jac["F"][-1]
        out[name] = r
        msg += (f"; {name} {r['gn_steps']} steps {r['pcg_iters']} it {r['ms']:.0f} ms F {r['F'][-1]:.6g}"
                + ("" if r["reached"] else " (not reached)"))
    log(msg)
    del sc
    torch.cuda.empty_cache()
    return out
