"""Autotuner for the launch shape of the integrators.

A candidate is (block, ppl, unroll, lookahead, waves_per_simd): threads per workgroup, particles
per lane, the loop form (one or two Philox blocks per trip, or the next block's noise computed
ahead of the steps) and (for the persistent sweep) the residency the grid is sized for.
The single-set integrator is tuned for two occupancy bands, because the best loop form differs:
"forward" on 2^20 particles (16 wavefronts per SIMD: issue-bound) and "forward-small" on 65536
(one wavefront per SIMD, where a wavefront's own instruction stream is all a SIMD issues);
lookups for ensembles of at most two wavefronts per SIMD use the small band's entry.
Every candidate computes bit-identical results (the reductions are tiled independently of the
launch shape), so the tuner only times them: each candidate runs a short probe workload after a
warm-up launch, timed with HIP events on the launch stream, and the fastest is kept.

Results are cached as JSON in the file named by ABP_TUNE_CACHE (default
~/.cache/abp_tune.json), keyed by device architecture, CU count, kernel and scheme.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import torch

from . import api
from .workloads import BASE_PARAMS, sweep_table

BLOCKS = (64, 128, 256)
PPLS = (1, 2)
UNROLLS = (1, 2)
WAVES = (4, 8)


def cache_path() -> str:
    return os.environ.get("ABP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "abp_tune.json"))


def device_key(kind: str, scheme: str) -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name).split(":")[0]
    return f"{arch}:{p.multi_processor_count}:{kind}:{scheme}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> bool:
    """Write the cache; False (and nothing cached) if its location is not writable."""
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        return False
    return True


LOOPS = ((1, 1), (2, 1), (1, 2))  # (unroll, lookahead)


def candidates(kind: str):
    waves = WAVES if kind == "batched" else (8,)
    for block, ppl, (unroll, la), wps in itertools.product(BLOCKS, PPLS, LOOPS, waves):
        yield dict(block=block, ppl=ppl, unroll=unroll, lookahead=la, waves_per_simd=wps)


def small_band_limit() -> int:
    """Largest ensemble that fills at most two wavefronts per SIMD of the current device."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return p.multi_processor_count * 4 * 2 * 64


def _time(fn, reps: int = 2) -> float:
    stream = torch.cuda.current_stream()
    fn()  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _forward_probe(scheme: str, n: int = 1 << 20, steps: int = 2000):
    state = api.State.empty(n)
    snap = api.State.empty(n)
    ws = api.reduce_workspace(n, 256)

    def make(tune):
        def fn():
            api.reset_state(state, 7)
            api.integrate(state, steps, BASE_PARAMS, scheme=scheme, seed=7, win_begin=steps // 2,
                          snap=snap, ws=ws, n_bins=256, tune=tune)
        return fn
    return make, n * steps


def _batched_probe(scheme: str, n_sets: int = 512, step_scale: float = 0.05):
    table, n_traj, n_steps = sweep_table(4096, seed=11)
    pick = np.linspace(0, 4095, n_sets).astype(np.int64)
    table, n_traj = table[pick], n_traj[pick]
    n_steps = np.maximum(100, (n_steps[pick] * step_scale).astype(np.int64))
    buf = api.SweepBuffers.make(table, n_traj, n_steps, bins=256)

    def make(tune):
        def fn():
            api.sweep_enqueue(buf, scheme=scheme, seed=11, bins=256, tune=tune)
        return fn
    return make, float((n_traj.astype(np.int64) * n_steps).sum())


def tune(kind: str = "forward", scheme: str = "heun", force: bool = False,
         verbose: bool = False, probe: dict | None = None) -> dict:
    """Best launch shape for `kind` ("forward" or "batched") and `scheme`; cached. `probe`
    overrides the probe workload's sizes (forward: n, steps; batched: n_sets, step_scale)."""
    key = device_key(kind, scheme)
    cache = _load_cache()
    if not force and key in cache:
        return cache[key]["tune"]
    if kind == "forward-small":
        make, work = _forward_probe(scheme, **(probe or dict(n=65536, steps=4000)))
    elif kind == "forward":
        make, work = _forward_probe(scheme, **(probe or {}))
    else:
        make, work = _batched_probe(scheme, **(probe or {}))
    results = []
    for cand in candidates(kind):
        ms = _time(make(cand))
        results.append((ms, cand))
        if verbose:
            print(f"{kind}/{scheme} {cand}: {ms:.3f} ms  {work / ms * 1e3:.3e} particle-steps/s",
                  flush=True)
    ms, best = min(results, key=lambda r: r[0])
    cache[key] = {"tune": best, "ms": ms, "particle_steps": work,
                  "all": [{"ms": m, **c} for m, c in results]}
    _store_cache(cache)
    return best


def lookup(kind: str, scheme: str, n: int | None = None) -> dict | None:
    """The cached shape, or None if this device has not been tuned. For the single-set
    integrator, an ensemble of n particles within the small band uses that band's entry."""
    cache = _load_cache()
    if kind == "forward" and n is not None and n <= small_band_limit():
        entry = cache.get(device_key("forward-small", scheme))
        if entry is not None:
            return entry["tune"]
    entry = cache.get(device_key(kind, scheme))
    return None if entry is None else entry["tune"]


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="tune the launch shapes and cache the result")
    ap.add_argument("--kind", choices=["forward", "forward-small", "batched", "all"],
                    default="all")
    ap.add_argument("--scheme", choices=["em", "heun", "all"], default="all")
    ap.add_argument("--force", action="store_true")
    args = ap.parse_args()
    kinds = ["forward", "forward-small", "batched"] if args.kind == "all" else [args.kind]
    schemes = ["em", "heun"] if args.scheme == "all" else [args.scheme]
    for k in kinds:
        for s in schemes:
            print(k, s, tune(k, s, force=args.force, verbose=True), flush=True)
