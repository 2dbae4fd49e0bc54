"""The paper's own workloads, run on the batched integrator and measured the way Sec. 3 measures.

load_force_curve(): mean drift velocity <v> against the load force F0, one parameter set per F0
value, all sets in one persistent launch (the use case behind Fig. 2: in Sec. 2 each work item is
one value of the load force, and all of them run at once). The load power -F0 <v> is returned
beside it (positive when the particles move against the load), and the depot efficiency
-F0 <v> / q: the useful power per unit of the energy flux q that feeds the depot, Eq. (1) (the
paper names the efficiency question but leaves its definition to the works it cites).

scaling(): time of one integration call against the number of work items, repeated R times with
the first repeats discarded (Sec. 3 runs 20 and averages the last 15), for several step counts
including zero steps; the per-step cost is the slope of a least-squares line of time against the
step count and the offset its intercept (Sec. 3.2, Fig. 6 methodology). On MI355X the "bands" the
paper saw on a 9800 GT are expected at multiples of the resident capacity.

density_cost(): cost of the time-accumulated histogram of x mod 1 (the particle density the paper
displays while the ensemble runs, Sec. 2) against the sampling stride: one integration call with
and without sampling, its time per sample and per sampled particle.
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from . import api
from .workloads import BASE_PARAMS, PARAM_KEYS


def load_force_curve(F0, params: dict | None = None, n: int = 4096, steps: int = 100_000,
                     window: int | None = None, scheme: str = "heun", seed: int = 1,
                     bins: int = 0, tune=None):
    """<v>(F0) for each load force in F0 (one set each). Returns dict of numpy arrays."""
    F0 = np.asarray(F0, dtype=np.float64)
    base = dict(BASE_PARAMS, **(params or {}))
    table = np.tile(np.array([base[k] for k in PARAM_KEYS], dtype=np.float64), (F0.size, 1))
    table[:, PARAM_KEYS.index("F0")] = F0
    window = steps // 2 if window is None else window
    r = api.sweep(table, np.full(F0.size, n, np.int32), np.full(F0.size, steps, np.int64),
                  np.full(F0.size, window, np.int64), scheme=scheme, seed=seed, bins=bins,
                  tune=tune)
    power = -F0 * r.mean_v
    return {"F0": F0, "mean_v": r.mean_v, "stderr": r.stderr, "load_power": power,
            "efficiency": power / base["q"]}


def _time_call(n: int, steps: int, scheme: str, state, snap, ws, stream) -> float:
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    api.reset_state(state, 1, 0, stream)
    api.integrate(state, steps, BASE_PARAMS, scheme=scheme, seed=1, win_begin=0, snap=snap, ws=ws,
                  n_bins=0, stream=stream)
    api.reduce(ws, n, 0, 1.0, stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3  # microseconds


def scaling(sizes, steps=(0, 1000, 10_000), scheme: str = "em", repeats: int = 20,
            keep: int = 15) -> list[dict]:
    """Per size: mean and sd of the call time (us) over the last `keep` of `repeats` runs at each
    step count, and the least-squares per-step cost and offset."""
    stream = torch.cuda.current_stream()
    rows = []
    for n in sizes:
        state, snap = api.State.empty(n), api.State.empty(n)
        ws = api.reduce_workspace(n, 0)
        row = {"n": int(n)}
        means = []
        for S in steps:
            t = [_time_call(n, S, scheme, state, snap, ws, stream) for _ in range(repeats)]
            t = np.array(t[repeats - keep:])
            row[f"t{S}_us"] = float(t.mean())
            row[f"sd{S}_us"] = float(t.std(ddof=1))
            means.append(t.mean())
        slope, icpt = np.polyfit(np.array(steps, dtype=np.float64), np.array(means), 1)
        row["us_per_step"] = float(slope)
        row["offset_us"] = float(icpt)
        row["particle_steps_per_s"] = float(n / (slope * 1e-6)) if slope > 0 else None
        rows.append(row)
    return rows


def density_cost(strides=(0, 10_000, 1000, 100, 10, 1), n: int = 1 << 20, steps: int = 20_000,
                 scheme: str = "heun", bins: int = 256, repeats: int = 5) -> list[dict]:
    """Median time (ms, HIP events around the integration call) of n particles x `steps` steps
    with the x mod 1 histogram accumulated every `stride` absolute steps (0 = off), and the
    extra time per sample over the unsampled call."""
    stream = torch.cuda.current_stream()
    state = api.State.empty(n)
    acc = torch.zeros(bins, dtype=torch.int64, device=state.cell.device)
    rows, base_ms = [], None
    for stride in strides:
        times = []
        for _ in range(repeats + 1):
            api.reset_state(state, 1, 0, stream)
            acc.zero_()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            api.integrate(state, steps, BASE_PARAMS, scheme=scheme, seed=1, stream=stream,
                          hist_stride=stride, hist_acc=acc if stride else None)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times[1:]))
        samples = steps // stride if stride else 0
        total = int(acc.sum().item())
        row = {"stride": stride, "samples": samples, "ms": ms, "counts_ok": total == n * samples}
        if stride == 0:
            base_ms = ms
        elif base_ms is not None:
            row["extra_ms"] = ms - base_ms
            row["extra_us_per_sample"] = (ms - base_ms) * 1e3 / samples
            row["extra_ps_per_particle_sample"] = (ms - base_ms) * 1e9 / (samples * n)
        rows.append(row)
    return rows


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="load-force curve, scaling and density-sampling "
                                             "experiments")
    ap.add_argument("what", choices=["force", "scaling", "density"])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--scheme", choices=["em", "heun"], default="em",
                    help="integration scheme of the scaling measurement")
    args = ap.parse_args()
    if args.what == "force":
        F0 = np.linspace(-1.0, 0.5, 31)
        t0 = time.perf_counter()
        out = load_force_curve(F0, steps=20_000 if args.quick else 100_000)
        secs = time.perf_counter() - t0
        for f, v, s, p, eta in zip(out["F0"], out["mean_v"], out["stderr"], out["load_power"],
                                   out["efficiency"]):
            print(json.dumps({"F0": round(float(f), 4), "mean_v": float(v), "stderr": float(s),
                              "load_power": float(p), "efficiency": float(eta)}))
        print(json.dumps({"seconds": secs}))
    elif args.what == "density":
        for row in density_cost():
            print(json.dumps(row), flush=True)
    else:
        sizes = [2 ** k for k in range(0, 21)]
        if not args.quick:
            sizes += list(range(16384, 16384 * 40 + 1, 16384))
        for row in scaling(sorted(set(sizes)), scheme=args.scheme, repeats=8 if args.quick else 20,
                           keep=5 if args.quick else 15):
            print(json.dumps(row), flush=True)
