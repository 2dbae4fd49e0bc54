"""Seeded synthetic workloads: parameter values, sizes and parameter-set tables.

This module holds no arithmetic of the method. It only fixes the inputs that both the HIP library
and the FP64 oracle consume, so the two sides can be run on identical problems.

Model parameters follow Eqs. (1)-(3) of the paper (energy depot q, c, coupling d2; friction
gamma0; load force F0; noise intensity D; ratchet amplitude U0, second-harmonic weight a, phase
phi). The paper prints no parameter values, step size, horizon or initial condition, so the
workloads below are synthetic; their values are the ones this project benchmarks on.
"""
from __future__ import annotations

import numpy as np

PARAM_KEYS = ("U0", "a", "phi", "gamma0", "F0", "d2", "q", "c", "D")

# Physics shared by the single-set workloads.
BASE_PARAMS = dict(U0=1.0, a=0.25, phi=0.0, gamma0=1.0, F0=0.0, d2=1.0, q=1.0, c=0.1, D=0.1)

WORKLOADS = {
    # parity case: small enough for the oracle to finish in well under a second
    "ensemble-1k-em": dict(n=1024, steps=10_000, dt=1e-3, scheme="em", window=5_000, bins=256,
                           seed=42),
    # throughput case: 2^20 particles, 1e5 stochastic-Heun steps
    "ensemble-1m-heun": dict(n=1 << 20, steps=100_000, dt=1e-3, scheme="heun", window=50_000,
                             bins=256, seed=7),
    # ratchet parameter sweep, one persistent launch
    "sweep-4096": dict(n_sets=4096, dt=1e-3, scheme="em", bins=256, seed=11),
    # pathwise gradient of the window mean velocity
    "adjoint-64k": dict(n=65536, steps=10_000, dt=1e-3, window=2_000, ckpt=100, seed=42),
    # batched adjoint driving Adam on (U0, a, d2)
    "adjoint-batched-1k": dict(n_sets=1024, n=1024, steps=50_000, dt=1e-3, window=10_000,
                               ckpt=48, stage=16, iters=50, seed=3),
}


def sweep_table(n_sets: int = 4096, seed: int = 11, traj=(64, 4096), steps=(20_000, 200_000)):
    """Ratchet sweep: D log-uniform in [1e-3, 1], U0 ~ U[0.5, 2], a ~ U[0, 0.5], d2 ~ U[0, 2],
    other parameters as BASE_PARAMS; per-set trajectory and step counts uniform integers in the
    inclusive ranges. Returns (params [n_sets, 9] float64 in PARAM_KEYS order, n_traj int32,
    n_steps int64)."""
    rng = np.random.default_rng(seed)
    table = np.tile(np.array([BASE_PARAMS[k] for k in PARAM_KEYS], dtype=np.float64), (n_sets, 1))
    col = {k: i for i, k in enumerate(PARAM_KEYS)}
    table[:, col["D"]] = 10.0 ** rng.uniform(-3.0, 0.0, n_sets)
    table[:, col["U0"]] = rng.uniform(0.5, 2.0, n_sets)
    table[:, col["a"]] = rng.uniform(0.0, 0.5, n_sets)
    table[:, col["d2"]] = rng.uniform(0.0, 2.0, n_sets)
    n_traj = rng.integers(traj[0], traj[1] + 1, n_sets).astype(np.int32)
    n_steps = rng.integers(steps[0], steps[1] + 1, n_sets).astype(np.int64)
    return table, n_traj, n_steps


def params_row(table: np.ndarray, k: int) -> dict:
    return {key: float(table[k, i]) for i, key in enumerate(PARAM_KEYS)}
