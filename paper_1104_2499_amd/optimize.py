"""Gradient-based ratchet design: Adam on (U0, a, d2) of many parameter sets at once.

Each set k is an ensemble of n particles; its objective is |L_k|, the magnitude of its window mean
velocity (the quantity the paper plots against the load force), maximised by Adam with the
pathwise gradients of the checkpointed adjoint (abp_adjoint through MeanVelocity). After every
step the parameters are projected to U0 in [0.05, 4], a in [0, 0.5], d2 in [0, 2]. At the end the
plain batched integrator recomputes every set's current at the final parameters; it must equal the
adjoint's forward loss bit for bit (same trajectories, same reduction).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api
from .adjoint import GRAD_KEYS, AdjointConfig, mean_velocity, param_rows
from .workloads import PARAM_KEYS, WORKLOADS, sweep_table

_WL = WORKLOADS["adjoint-batched-1k"]

FREE = ("U0", "a", "d2")
BOUNDS = {"U0": (0.05, 4.0), "a": (0.0, 0.5), "d2": (0.0, 2.0)}


@dataclass
class AdamResult:
    theta: np.ndarray          # [n_sets, 8] final (U0, a, D, d2, q, c, gamma0, F0)
    history: np.ndarray        # [iters + 1] mean |L| over sets before each step and at the end
    final_loss: np.ndarray     # [n_sets] adjoint forward loss at the final parameters
    verify_mean_v: np.ndarray  # [n_sets] plain batched integrator at the final parameters
    seconds: float
    particle_steps: float      # forward + backward work of the optimisation (in forward units)


def initial_theta(n_sets: int, seed: int) -> np.ndarray:
    """Initial parameters drawn like the ratchet sweep (D log-uniform, U0, a, d2 uniform)."""
    table, _, _ = sweep_table(n_sets, seed=seed)
    col = {k: i for i, k in enumerate(PARAM_KEYS)}
    return np.ascontiguousarray(table[:, [col[k] for k in GRAD_KEYS]])


def adam_ratchet(n_sets: int = 1024, n: int = 1024, steps: int = 50_000, window: int = 10_000,
                 ckpt: int = _WL["ckpt"], iters: int = 50, seed: int = 3, lr: float = 1e-2,
                 lookback: int = 0, stage: int = _WL["stage"], verbose: bool = False) -> AdamResult:
    """Adam on (U0, a, d2) of n_sets sets maximising |L_k|. lookback > 0 uses the decayed adjoint
    estimator; the default is the exact pathwise gradient. The parameters live on the device for
    the whole loop (the library reads its parameter rows there)."""
    cfg = AdjointConfig(n=n, steps=steps, window=window, ckpt=ckpt, seed=seed, lookback=lookback,
                        stage=stage)
    dev = torch.device("cuda")
    theta0 = torch.tensor(initial_theta(n_sets, seed), dtype=torch.float64, device=dev)
    idx = [GRAD_KEYS.index(k) for k in FREE]
    free = theta0[:, idx].clone().requires_grad_(True)
    fixed = theta0.clone()
    opt = torch.optim.Adam([free], lr=lr)
    lo = torch.tensor([BOUNDS[k][0] for k in FREE], dtype=torch.float64, device=dev)
    hi = torch.tensor([BOUNDS[k][1] for k in FREE], dtype=torch.float64, device=dev)
    history = []
    t0 = time.perf_counter()

    def assemble(f):
        cols = list(torch.unbind(fixed, dim=1))
        for j, i in enumerate(idx):
            cols[i] = f[:, j]
        return torch.stack(cols, dim=1)

    for it in range(iters):
        L = mean_velocity(assemble(free), cfg)
        objective = -L.abs().sum()
        opt.zero_grad()
        objective.backward()
        opt.step()
        with torch.no_grad():
            free.copy_(torch.maximum(torch.minimum(free, hi), lo))
        history.append(float(L.detach().abs().mean()))
        if verbose:
            print(f"iter {it:3d}: mean |<v>| = {history[-1]:.6e}", flush=True)
    theta = assemble(free.detach())
    final = mean_velocity(theta, cfg).detach().cpu().numpy()
    history.append(float(np.abs(final).mean()))
    seconds = time.perf_counter() - t0
    rows = param_rows(theta, cfg)
    sw = api.sweep(rows, np.full(n_sets, n, dtype=np.int32), np.full(n_sets, steps, np.int64),
                   np.full(n_sets, window, np.int64), dt=cfg.dt, scheme="em", seed=seed, bins=0)
    work = float(n_sets) * n * steps * (2 * iters + 1)
    return AdamResult(theta.cpu().numpy(), np.array(history), final, sw.mean_v, seconds, work)


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sets", type=int, default=1024)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=50_000)
    ap.add_argument("--window", type=int, default=10_000)
    ap.add_argument("--ckpt", type=int, default=_WL["ckpt"])
    ap.add_argument("--stage", type=int, default=_WL["stage"], choices=[0, 8, 16])
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--lookback", type=int, default=0)
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    r = adam_ratchet(args.sets, args.n, args.steps, args.window, args.ckpt, args.iters, args.seed,
                     lookback=args.lookback, stage=args.stage,
                     verbose=not args.quiet)
    print(json.dumps({"workload": "adjoint-batched-1k", "lookback": args.lookback,
                      "seconds": r.seconds,
                      "mean_abs_v_start": r.history[0], "mean_abs_v_end": r.history[-1],
                      "verify_equal": bool(np.array_equal(r.final_loss, r.verify_mean_v)),
                      "forward_units_per_s": r.particle_steps / r.seconds}), flush=True)
