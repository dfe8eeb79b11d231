"""Training and evaluation code of the learned block preconditioner.

Training data: exact 4x4 blocks of J^T J and per-unit features computed by the library
along Gauss-Newton trajectories (Jacobi-preconditioned) of seeded scenes of the 128^3
object-in-a-box kind; a random subset of the units that some ray touches per (scene, step),
drawn by the library.  The standardisation of the features is computed by the library, and
training runs the library's MFMA forward/backward kernel and Adam.  Evaluation counts PCG
iterations to a relative residual of 1e-3 and GN time to a target objective on held-out seeds.

A model is (bfloat16 weights, FP32 standardisation, fallback threshold q): a unit whose
prediction misses its own normalised block by more than q takes the exact block inverse.
"""
from __future__ import annotations

import dataclasses
import os
import time
from typing import Dict, List

import numpy as np
import torch

from . import abi
from .scene import Scene, mlp_feature_stats, mlp_train_step


@dataclasses.dataclass
class Model:
    w_bf16: torch.Tensor      # [PERF_MLP_NW] bfloat16
    norm: torch.Tensor        # [PERF_MLP_NNORM] float32
    q_fallback: float = float("inf")

    def install(self, sc: Scene):
        sc.mlp_set_weights(self.w_bf16, self.norm, self.q_fallback)


def init_weights(seed: int = 0) -> np.ndarray:
    """He-style initialisation (float64, packed order); the network starts at L = I."""
    rng = np.random.default_rng(seed)
    nh, ni, nip, no, nop = 64, 10, 16, 10, 16  # 6 features + the block's coupling (3) and Schur log
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


def generate(workloads, gn_steps=5, per_step=65536, pcg_iters=5, seed=0, log=print, first_step=0):
    """Features and blocks along Jacobi-GN trajectories (steps first_step .. gn_steps - 1 are
    sampled, about per_step touched units each): (feat [n, PERF_MLP_NFEAT], blocks [n, 5]) GPU tensors."""
    feats, blocks = [], []
    for w in workloads:
        sc = scene_for(w)
        x = torch.from_numpy(w.x_init).to(sc.device)
        for step in range(gn_steps):
            if step >= first_step:
                f, b = sc.features(x)
                key = (seed * 1000003 + w.seed * 131 + step) & 0xFFFFFFFF
                fo, bo = _sample(sc, f, b, key, per_step)
                feats.append(fo.clone())
                blocks.append(bo.clone())
            sc.gn_step(x, max_iters=pcg_iters, precond="jacobi")
        log(f"[learned] data from seed {w.seed}: {sum(t.shape[0] for t in feats)} samples")
        del sc
        torch.cuda.empty_cache()
    return torch.cat(feats), torch.cat(blocks)


def _sample(sc: Scene, f, b, key: int, per_step: int):
    """About per_step rows of the touched units, drawn by the library (count first, then keep
    each with probability per_step / touched)."""
    _, _, touched = sc.training_rows(f, b, key, 1.0, 0)  # eligible rows: touched, finite
    keep = min(1.0, per_step / max(touched, 1))
    fo, bo, _ = sc.training_rows(f, b, key, keep, int(per_step * 1.2) + 1024)
    return fo, bo


def train(feat, blocks, epochs=4, batch=16384, lr=5e-4, seed=0, damp=0.0, log=print, state=None):
    """Adam on the library's training kernel towards the damped normalised inverse
    (B~ + damp I)^-1, with the features standardised by the library's statistics of the
    training set.  state (from an earlier call: FP32 master weights, Adam moments, step count,
    standardisation) continues a training run on new data.  Returns (state, model, loss
    history)."""
    dev = feat.device
    if state is None:
        norm = mlp_feature_stats(feat)
        w32 = torch.from_numpy(init_weights(seed).astype(np.float32)).to(dev)
        m = torch.zeros_like(w32)
        v = torch.zeros_like(w32)
        t = 0
    else:
        norm, w32, m, v, t = (state["norm"].to(dev), state["w32"].to(dev), state["m"].to(dev), state["v"].to(dev),
                              int(state["t"]))
    wbf = w32.to(torch.bfloat16)
    grad = torch.zeros_like(w32)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    n = feat.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed + t)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            t += 1
            fb = feat[idx].contiguous()
            bb = blocks[idx].contiguous()
            mlp_train_step(w32, wbf, m, v, t, lr, norm, fb, bb, loss, grad, damp=damp)
            lv = loss.item()
            if not np.isfinite(lv):
                raise FloatingPointError(f"non-finite training loss at step {t}")
            tot += lv
            cnt += 1
        hist.append(tot / max(cnt, 1))
        log(f"[learned] damp {damp} epoch {ep}: mean loss {hist[-1]:.5f}")
    state = {"norm": norm, "w32": w32, "m": m, "v": v, "t": t}
    return state, Model(wbf.clone(), norm), hist


def save_state(path: str, state: dict):
    np.savez(path, **{k: (v.cpu().numpy() if torch.is_tensor(v) else np.array([v])) for k, v in state.items()})


def load_state(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {"norm": torch.from_numpy(z["norm"]), "w32": torch.from_numpy(z["w32"]), "m": torch.from_numpy(z["m"]),
                "v": torch.from_numpy(z["v"]), "t": int(z["t"][0])}


def pcg_iterations(sc: Scene, x, precond: str, rel_tol=1e-3, max_iters=256):
    st = sc.gn_step(x.clone(), max_iters=max_iters, precond=precond, rel_tol=rel_tol)
    return st["pcg_iters"], st


def evaluate(workloads, nets: Dict[str, Model], rel_tol=1e-3, gn_steps=(1, 3), max_iters=200,
             log=print) -> List[dict]:
    """PCG iterations and wall time to sqrt(R/R0) <= rel_tol for Jacobi, exact block-Jacobi and
    each learned model of `nets`, at the given steps of a Jacobi-GN trajectory from the initial
    parameters."""
    out = []
    for w in workloads:
        sc = scene_for(w)
        x = torch.from_numpy(w.x_init).to(sc.device)
        for step in range(max(gn_steps) + 1):
            if step in gn_steps:
                row = {"seed": w.seed, "gn_step": step}
                runs = [("jacobi", "jacobi", None), ("block", "block", None)]
                runs += [(name, "learned", mdl) for name, mdl in nets.items()]
                for name, pc, mdl in runs:
                    if mdl is not None:
                        mdl.install(sc)
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


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "precond_mlp.npz")


def save_model(path: str, model: Model):
    np.savez(path, w_bf16_bits=model.w_bf16.view(torch.int16).cpu().numpy().view(np.uint16),
             norm=model.norm.cpu().numpy().astype(np.float32),
             q_fallback=np.array([model.q_fallback], dtype=np.float64))


def load_model(path: str = WEIGHTS, device="cuda:0", q_fallback=None) -> Model:
    """The packed bfloat16 weights (uint16 bits), the standardisation and the fallback threshold
    from an .npz written by save_model (loaded without pickle)."""
    with np.load(path, allow_pickle=False) as z:
        bits, norm, q = z["w_bf16_bits"], z["norm"], float(z["q_fallback"][0])
    if bits.dtype != np.uint16 or bits.size != abi.PERF_MLP_NW or norm.size != abi.PERF_MLP_NNORM:
        raise ValueError(f"{path}: expected {abi.PERF_MLP_NW} uint16 weights and {abi.PERF_MLP_NNORM} norm values")
    w = torch.from_numpy(bits.view(np.int16).copy()).to(device).view(torch.bfloat16)
    nm = torch.from_numpy(norm.astype(np.float32)).to(device)
    return Model(w, nm, q if q_fallback is None else float(q_fallback))


def fallback_fraction(sc: Scene, x) -> float:
    """Share of the touched units whose prediction the installed model's threshold sends to the
    exact block inverse at x (the library marks them with a negative t_d)."""
    feat, blocks = sc.features(x)
    out = sc.mlp_infer(feat, blocks)[:, 0].cpu().numpy()
    live = np.count_nonzero(out)
    return float(np.count_nonzero(out < 0) / max(live, 1))


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
        iters += st["pcg_iters"] + st["fallback_iters"]
        F.append(st["F_after"])
        if F_stop >= 0 and st["F_after"] <= F_stop:
            break
    torch.cuda.synchronize()
    return {"F0": F0, "F": F, "pcg_iters": iters, "gn_steps": len(F), "ms": (time.perf_counter() - t0) * 1e3,
            "x": x}


def gn_compare(w, nets: Dict[str, Model], n_steps=5, pcg_iters=30, rel_tol=0.0, extra_steps=3, log=print) -> dict:
    """Jacobi-PCG GN for n_steps, then GN with each learned model of `nets` until it reaches the
    Jacobi run's final F (at most n_steps + extra_steps), with the same PCG settings."""
    sc = scene_for(w)
    x0 = torch.from_numpy(w.x_init).to(sc.device)
    jac = gn_run(sc, x0, "jacobi", n_steps, pcg_iters, rel_tol)
    out = {"seed": w.seed, "pcg_iters_per_step": pcg_iters, "rel_tol": rel_tol, "jacobi": jac}
    msg = f"[learned] GN seed {w.seed}: jacobi {jac['pcg_iters']} it {jac['ms']:.0f} ms F {jac['F'][-1]:.6g}"
    log(msg + " (running the others)")
    for name, mdl in nets.items():
        pc = "learned"
        if name == "block":
            pc = "block"
        else:
            mdl.install(sc)
        r = gn_run(sc, x0, pc, n_steps + extra_steps, pcg_iters, rel_tol, F_stop=jac["F"][-1])
        r["reached"] = r["F"][-1] <= jac["F"][-1]
        del r["x"]
        if pc == "learned":
            r["fallback_frac"] = [fallback_fraction(sc, x0), fallback_fraction(sc, jac["x"])]
        out[name] = r
        log(f"[learned]   seed {w.seed} {name}: {r['gn_steps']} steps {r['pcg_iters']} it {r['ms']:.0f} ms "
            f"F {r['F'][-1]:.6g}" + (f" fallback {r['fallback_frac'][0]:.3f} at x0, {r['fallback_frac'][1]:.3f} "
                                     f"at Jacobi's end" if pc == "learned" else ""))
        msg += (f"; {name} {r['gn_steps']} steps {r['pcg_iters']} it {r['ms']:.0f} ms F {r['F'][-1]:.6g}"
                + ("" if r["reached"] else " (not reached)"))
    del jac["x"]
    log(msg)
    del sc
    torch.cuda.empty_cache()
    return out
