#!/usr/bin/env python3
"""Benchmark of the ABP ensemble integrator on one MI355X.

One step = the whole hot path once over the throughput workload "ensemble-1m-heun": 2^20
particles, initial condition from Philox, 1e5 stochastic-Heun steps of Eqs. (1)-(3) with dt = 1e-3,
window snapshot at step 5e4, fused per-tile reduction, and the FP64 finalize (mean drift velocity,
its standard error, 256-bin histogram of x mod 1). Inputs are synthetic and resident on the device.

Prints one JSON line: particle-steps/s for the whole job, the VALU roofline of the dominant kernel
(timed with HIP events on the stream it runs on), and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD16 at 2.4 GHz = 256 * 64 lanes * 2.4e9 full-rate VALU lane-slots/s.
VALU_LANE_SLOTS_PER_S = 256 * 64 * 2.4e9
FP32_VECTOR_PEAK_TFLOPS = 157.3

# VALU cost of one particle-step of the hot loop, counted from the gfx950 ISA of
# k_integrate<HEUN, 1, 1> (one Philox block = 4 steps per loop trip) and weighted by the issue cost
# of each instruction class measured on the device (profiles/valu_issue_rates.txt):
#   full-rate FP32/INT ops per 4 steps, transcendentals per 4 steps, v_mad_u64_u32 per 4 steps.
ISA_HEUN = dict(full=156, trans=16, mad64=16)
ISA_EM = dict(full=96, trans=12, mad64=16)
# FP32 arithmetic of the method per particle-step (FMA = 2), transcendentals counted as 1 each:
# Heun 2 drift evaluations (14 each) + predictor 7 + corrector 10 + Box-Muller share 3 + 4 trans.
FLOP_PER_STEP = dict(heun=49 + 4, em=25 + 3)


def issue_cost(counts: dict, rates: dict) -> float:
    """Lane-slots per particle-step (full-rate op = 1 slot)."""
    return (counts["full"] + counts["trans"] * rates["trans"] + counts["mad64"] * rates["mad64"]) / 4.0


def load_rates() -> dict:
    """Issue cost (in full-rate slots) of a transcendental and of v_mad_u64_u32 on gfx950, as
    measured by the committed microbenchmark summary; defaults to the CDNA quarter rate."""
    rates = dict(trans=4.0, mad64=4.0, source="assumed quarter rate")
    path = os.path.join(ROOT, "profiles", "valu_issue_rates.txt")
    if os.path.exists(path):
        for line in open(path):
            if line.startswith("trans_slots:"):
                rates["trans"] = float(line.split(":")[1])
            elif line.startswith("mad64_slots:"):
                rates["mad64"] = float(line.split(":")[1])
        rates["source"] = "profiles/valu_issue_rates.txt"
    return rates


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1104_2499_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(wl: dict, params: dict, seconds_budget: float = 15.0) -> dict:
    """The FP64 oracle on a bounded sample of the workload (same scheme, dt, steps per particle),
    timed on the host cores. Particles are independent, so the rate scales with the sample."""
    import numpy as np

    import oracle

    scheme = oracle.HEUN if wl["scheme"] == "heun" else oracle.EM
    # calibrate on a short run, then size the sample to the budget
    n_cal, s_cal = 256, 2000
    x, v, e = oracle.init_state(n_cal, wl["seed"])
    t0 = time.perf_counter()
    oracle.integrate(params, x, v, e, s_cal, dt=wl["dt"], scheme=scheme, seed=wl["seed"])
    rate = n_cal * s_cal / (time.perf_counter() - t0)
    steps = wl["steps"]
    n = int(max(64, min(wl["n"], rate * seconds_budget / steps)))
    n = (n // 64) * 64
    ids = (np.arange(n, dtype=np.uint64) * (wl["n"] // n)).astype(np.uint64)
    x, v, e = oracle.init_state(n, wl["seed"], ids=ids)
    t0 = time.perf_counter()
    xe, ve, ee, xs, _ = oracle.integrate(params, x, v, e, steps, dt=wl["dt"], scheme=scheme,
                                         seed=wl["seed"], ids=ids,
                                         win_begin=steps - wl["window"])
    oracle.reduce(xs, xe, wl["window"] * wl["dt"], wl["bins"])
    dt_s = time.perf_counter() - t0
    return {"value": n * steps / dt_s, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} of {wl['n']} particles (evenly spaced ids), full {steps} steps, "
                      f"{dt_s:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ensemble-1m-heun",
                    choices=["ensemble-1m-heun", "ensemble-1k-em"])
    ap.add_argument("--sim-steps", type=int, default=None,
                    help="override the SDE step count (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", default=None, help="block,ppl,unroll (default: library default)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import BASE_PARAMS, WORKLOADS

    wl = dict(WORKLOADS[args.workload])
    if args.sim_steps:
        wl["steps"] = args.sim_steps
        wl["window"] = args.sim_steps // 2
    n, S, W, bins, dt, seed = wl["n"], wl["steps"], wl["window"], wl["bins"], wl["dt"], wl["seed"]
    tune = None
    if args.tune:
        b, p, u = (int(t) for t in args.tune.split(","))
        tune = dict(block=b, ppl=p, unroll=u)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    state = api.State.empty(n, dev)
    snap = api.State.empty(n, dev)
    ws = api.reduce_workspace(n, bins, dev)
    out = hist = None
    ev = []

    def one_step(timed: bool):
        nonlocal out, hist
        api.reset_state(state, seed, 0, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.integrate(state, S, BASE_PARAMS, dt, wl["scheme"], seed, 0, 0, S - W, snap, ws, bins,
                      tune, stream)
        e1.record(stream)
        if timed:
            ev.append((e0, e1))
        out, hist = api.reduce(ws, n, bins, W * dt, stream)

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    ps = n * S
    value = ps * args.steps / wall
    rates = load_rates()
    isa = ISA_HEUN if wl["scheme"] == "heun" else ISA_EM
    slots = issue_cost(isa, rates)
    kern_rate = ps / (kern_ms * 1e-3)
    achieved = slots * kern_rate / 1e12
    peak = VALU_LANE_SLOTS_PER_S / 1e12
    kernel = "k_integrate_" + wl["scheme"]
    traffic = load_traffic(kernel, args.workload)
    o = out.cpu()
    line = {
        "metric": "particle-steps/s (FP32) and % VALU peak",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "particles": n, "sde_steps": S, "scheme": wl["scheme"],
                   "dt": dt, "window": W, "bins": bins, "seed": seed, "params": BASE_PARAMS,
                   "tuning": tune or "default"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": kernel, "kernel_ms": kern_ms,
                     "slots_per_particle_step": slots, "issue_rates": rates,
                     "fp32_tflops": FLOP_PER_STEP[wl["scheme"]] * kern_rate / 1e12,
                     "fp32_flop_frac": FLOP_PER_STEP[wl["scheme"]] * kern_rate / 1e12
                     / FP32_VECTOR_PEAK_TFLOPS},
        "result": {"mean_v": float(o[0]), "stderr": float(o[1]),
                   "hist_total": int(hist.sum().item())},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, BASE_PARAMS)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
