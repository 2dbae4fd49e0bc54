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

# MI355X figures: 256 CUs x 4 SIMDs, 2.4 GHz peak engine clock, FP32 vector peak 157.3 TFLOP/s.
N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic FP32 FLOPs of the method per particle-step (FMA = 2): drift 14 (phase add, 2 FMAs for
# F0 - U', 2 for f_v, mul + 2 FMAs for f_e), EM update 7, Heun predictor 7 + corrector 10 + a second
# drift, and half a Box-Muller pair (5 per pair). Transcendentals are counted separately.
FLOP_PER_STEP = dict(em=24, heun=48)
TRANS_PER_STEP = dict(em=3, heun=4)
# VALU instructions per particle-step in the hot loop of k_integrate<scheme, 1, 1> (gfx950 ISA, one
# aligned 8-step span = two Philox blocks per loop trip: EM 241, Heun 361).
VALU_INSTR_PER_STEP = dict(em=241 / 8, heun=361 / 8)
# FP32 FLOPs per particle-step as the hardware counts them (SQ_INSTS_VALU_FLOPS_FP32: FMA = 2,
# add, mul and transcendental = 1), including the high/low bookkeeping and Box-Muller, from the
# same loops: Heun 144 FMA, 79 add/sub, 28 mul, 32 transcendental per span; EM 72, 47, 20, 24.
COUNTED_FLOP_PER_STEP = dict(em=235 / 8, heun=427 / 8)
# Issue time of v_cos/v_sin/v_log/v_sqrt_f32 per wave64 instruction per SIMD, measured by
# ubench/valu_rates.hip (profiles/valu_issue_rates.txt).
TRANS_NS_PER_WAVE_INSTR = 3.45
UBENCH = os.path.join(ROOT, "paper_1104_2499_amd", "ubench", "valu_rates")
STEPS_PER_TRIP = 8  # one loop trip of k_integrate: an aligned 8-step span


def mix_ceiling() -> dict:
    """The measured issue ceiling of the integrators' own instruction mix: ubench/valu_rates
    --mix replays one 4-step loop trip of k_integrate (its gfx950 instruction sequence) on
    registers that never wait for each other, at 1, 2, 4 and 8 wavefronts per SIMD; returns
    {scheme: {waves_per_simd: ns per trip per wavefront per SIMD}}. Run as a child process."""
    import subprocess

    res = subprocess.run([UBENCH, "--mix"], capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        raise RuntimeError("valu_rates --mix failed: " + res.stderr[-500:])
    out: dict = {}
    for line in res.stdout.splitlines():
        if line.startswith("mix_"):
            key, val = line.split(":")
            _, scheme, _, _, w = key.split("_")  # mix_<scheme>_trip_ns_w<W>
            out.setdefault(scheme, {})[int(w[1:])] = float(val)
    return out


KERNEL_SOURCES = ("common.hpp", "device.hpp", "reduce.hpp", "integrate.hpp", "integrate_heun.hip")


def source_hash() -> str:
    """Hash of the sources the Heun integrator kernel is built from, and of its build flags."""
    from paper_1104_2499_amd import build

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1104_2499_amd", "csrc")
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(" ".join(build.flags_for(os.path.join(csrc, KERNEL_SOURCES[-1]))).encode())
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
            "kind": "oracle", "host_cpu": _host_cpu(),
            "sample": f"{n} of {wl['n']} particles (evenly spaced ids), full {steps} steps, "
                      f"{dt_s:.1f} s"}


def _host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _gpu_ms(fn, reps: int) -> float:
    """Median wall time of `fn` in ms (each call synchronised), after one warm-up call."""
    import numpy as np
    import torch

    fn()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(t))


def _gpu_ensemble_ms(wl: dict, reps: int) -> float:
    """One whole run of a plain-ensemble workload on the GPU (initial state, integration with the
    window snapshot and fused reduction, finalize), median ms."""
    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import BASE_PARAMS

    n, S = wl["n"], wl["steps"]
    state, snap = api.State.empty(n), api.State.empty(n)
    ws = api.reduce_workspace(n, wl["bins"])

    def run():
        api.reset_state(state, wl["seed"])
        api.integrate(state, S, BASE_PARAMS, wl["dt"], wl["scheme"], wl["seed"], 0, 0,
                      S - wl["window"], snap, ws, wl["bins"])
        api.reduce(ws, n, wl["bins"], wl["window"] * wl["dt"])
    return _gpu_ms(run, reps)


def cpu_baselines_all() -> list:
    """The FP64 oracle on every workload, with all host cores and with one, beside the GPU time
    of the same workload. The oracle runs the whole workload where that takes seconds and an
    evenly spaced sample of particles (and of parameter sets) otherwise; particles are
    independent, so its time for the whole workload is the sample's time scaled by work."""
    import numpy as np

    import oracle
    from paper_1104_2499_amd import adjoint
    from paper_1104_2499_amd.optimize import initial_theta
    from paper_1104_2499_amd.workloads import BASE_PARAMS, WORKLOADS, params_row, sweep_table

    all_cores = oracle.num_threads()
    out = []

    def timed_cpu(fn, work: float, threads: int, sample: str) -> dict:
        oracle.set_num_threads(threads)
        t0 = time.perf_counter()
        fn()
        sec = time.perf_counter() - t0
        oracle.set_num_threads(all_cores)
        return {"threads": threads, "sample": sample, "particle_steps": work, "seconds": sec,
                "rate": work / sec}

    def ensemble(wl, n_sample):
        scheme = oracle.HEUN if wl["scheme"] == "heun" else oracle.EM
        ids = (np.arange(n_sample, dtype=np.uint64) * (wl["n"] // n_sample)).astype(np.uint32)

        def run():
            x, v, e = oracle.init_state(n_sample, wl["seed"], ids=ids)
            xe, _, _, xs, _ = oracle.integrate(BASE_PARAMS, x, v, e, wl["steps"], dt=wl["dt"],
                                               scheme=scheme, seed=wl["seed"], ids=ids,
                                               win_begin=wl["steps"] - wl["window"])
            oracle.reduce(xs, xe, wl["window"] * wl["dt"], wl["bins"])
        return run, float(n_sample) * wl["steps"]

    # plain ensembles: the parity case in full, the throughput case on a sample
    for name, n_all, n_one, reps in (("ensemble-1k-em", 1024, 1024, 20),
                                     ("ensemble-1m-heun", 16384, 512, 2)):
        wl = WORKLOADS[name]
        work = float(wl["n"]) * wl["steps"]
        run, w = ensemble(wl, n_all)
        cpu = timed_cpu(run, w, all_cores, f"{n_all} of {wl['n']} particles, full steps")
        run1, w1 = ensemble(wl, n_one)
        one = timed_cpu(run1, w1, 1, f"{n_one} of {wl['n']} particles, full steps")
        g_ms = _gpu_ensemble_ms(wl, reps)
        out.append({"workload": name, "unit": "particle-steps/s", "particle_steps": work,
                    "gpu_ms": g_ms, "gpu_rate": work / (g_ms * 1e-3), "oracle_all_cores": cpu,
                    "oracle_one_core": one})

    # parameter sweep: every 64th set with its first 64 trajectories at its full step count
    wl = WORKLOADS["sweep-4096"]
    table, n_traj, n_steps = sweep_table(wl["n_sets"], seed=wl["seed"])
    work = float((n_traj.astype(np.int64) * n_steps).sum())

    def sweep_sample(every, m):
        sets = range(0, wl["n_sets"], every)
        w = float(sum(min(int(n_traj[k]), m) * int(n_steps[k]) for k in sets))

        def run():
            for k in sets:
                n, S = min(int(n_traj[k]), m), int(n_steps[k])
                x, v, e = oracle.init_state(n, wl["seed"], k)
                xe, _, _, xs, _ = oracle.integrate(params_row(table, k), x, v, e, S, dt=wl["dt"],
                                                   seed=wl["seed"], set_id=k,
                                                   win_begin=S - S // 2)
                oracle.reduce(xs, xe, (S // 2) * wl["dt"], wl["bins"])
        return run, w

    run, w = sweep_sample(64, 64)
    cpu = timed_cpu(run, w, all_cores, "64 sets (every 64th), first 64 trajectories each")
    run1, w1 = sweep_sample(256, 16)
    one = timed_cpu(run1, w1, 1, "16 sets (every 256th), first 16 trajectories each")
    g_ms = sweep_bench(reps=1)["ms"]
    out.append({"workload": "sweep-4096", "unit": "particle-steps/s", "particle_steps": work,
                "gpu_ms": g_ms, "gpu_rate": work / (g_ms * 1e-3), "oracle_all_cores": cpu,
                "oracle_one_core": one})

    # adjoint: forward + pathwise gradient of the window mean velocity
    wl = WORKLOADS["adjoint-64k"]

    def adj_sample(wl, n, params):
        """oracle.adjoint (forward with the trajectory stored, then the reverse sweep) on n
        evenly spaced particles of set 0."""
        ids = (np.arange(n, dtype=np.uint64) * (wl["n"] // n)).astype(np.uint32)

        def run():
            x, v, e = oracle.init_state(n, wl["seed"], 0, ids=ids)
            oracle.adjoint(params, x, v, e, wl["steps"], wl["window"], dt=wl["dt"],
                           seed=wl["seed"], ids=ids)
        return run, float(n) * wl["steps"]

    work = float(wl["n"]) * wl["steps"]
    run, w = adj_sample(wl, wl["n"], BASE_PARAMS)
    cpu = timed_cpu(run, w, all_cores, "all 65536 particles")
    run1, w1 = adj_sample(wl, 1024, BASE_PARAMS)
    one = timed_cpu(run1, w1, 1, "1024 of 65536 particles")

    def plain():  # the oracle's forward alone on the same ensemble, for its own cost ratio
        x, v, e = oracle.init_state(wl["n"], wl["seed"])
        oracle.integrate(BASE_PARAMS, x, v, e, wl["steps"], dt=wl["dt"], seed=wl["seed"],
                         win_begin=wl["steps"] - wl["window"])
    fwd = timed_cpu(plain, work, all_cores, "all 65536 particles, forward only")
    a = adjoint_bench(reps=5)
    g_ms = a["adjoint_forward_ms"] + a["adjoint_backward_ms"]
    out.append({"workload": "adjoint-64k", "unit": "particle-steps/s (forward + gradient)",
                "particle_steps": work, "gpu_ms": g_ms, "gpu_rate": work / (g_ms * 1e-3),
                "gpu_cost_ratio": a["cost_ratio"], "oracle_all_cores": cpu,
                "oracle_one_core": one, "oracle_forward_seconds": fwd["seconds"],
                "oracle_cost_ratio": cpu["seconds"] / fwd["seconds"]})

    # batched adjoint: one Adam iteration's forward + gradients, sampled on set 0
    wl = WORKLOADS["adjoint-batched-1k"]
    theta = initial_theta(wl["n_sets"], wl["seed"])
    p0 = dict(BASE_PARAMS)
    p0.update({k: float(theta[0, i]) for i, k in enumerate(adjoint.GRAD_KEYS)})
    work = float(wl["n_sets"]) * wl["n"] * wl["steps"]
    run, w = adj_sample(wl, wl["n"], p0)
    cpu = timed_cpu(run, w, all_cores, "set 0 of 1024 (all its 1024 particles)")
    run1, w1 = adj_sample(wl, 64, p0)
    one = timed_cpu(run1, w1, 1, "64 evenly spaced particles of set 0")
    b = adjoint_batched_bench(wl["stage"], wl["ckpt"], reps=2)
    g_ms = b["forward_ms"] + b["backward_ms"]
    out.append({"workload": "adjoint-batched-1k", "unit": "particle-steps/s (forward + gradient)",
                "particle_steps": work, "gpu_ms": g_ms, "gpu_rate": work / (g_ms * 1e-3),
                "oracle_all_cores": cpu, "oracle_one_core": one})

    for r in out:
        r["host_cpu"] = _host_cpu()
        r["gpu_over_oracle_all_cores"] = r["gpu_rate"] / r["oracle_all_cores"]["rate"]
    return out


def sweep_bench(reps: int = 2, tune_batched=None, tune_single=None) -> dict:
    """The 4096-set ratchet sweep in one persistent launch, and the single-set throughput of the
    same scheme (2^20 particles of the base parameters) for comparison; each with its launch
    shape (None = library default)."""
    import numpy as np
    import torch

    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import BASE_PARAMS, WORKLOADS, sweep_table

    wl = WORKLOADS["sweep-4096"]
    table, n_traj, n_steps = sweep_table(wl["n_sets"], seed=wl["seed"])
    work = float((n_traj.astype(np.int64) * n_steps).sum())
    # lanes past a set's last trajectory in its last 64-particle tile still step (masked)
    lanes = float(((n_traj.astype(np.int64) + 63) // 64 * 64 * n_steps).sum())
    # tables resident on the device before the timed region; each timed sweep plans its work
    # list on the device, integrates and finalises
    buf = api.SweepBuffers.make(table, n_traj, n_steps, bins=wl["bins"])

    def one_sweep():
        api.sweep_enqueue(buf, wl["dt"], wl["scheme"], wl["seed"], wl["bins"], tune_batched)
    one_sweep()
    api.check_device_status(buf.status, "sweep")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one_sweep()
    torch.cuda.synchronize()
    t_sweep = (time.perf_counter() - t0) / reps
    api.check_device_status(buf.status, "sweep")
    mean_v = buf.out[:, 0].cpu().numpy()

    n, S = 1 << 20, 20_000
    state, snap = api.State.empty(n), api.State.empty(n)
    rws = api.reduce_workspace(n, wl["bins"])

    def single():
        api.reset_state(state, wl["seed"])
        api.integrate(state, S, BASE_PARAMS, wl["dt"], wl["scheme"], wl["seed"], 0, 0, S // 2, snap,
                      rws, wl["bins"], tune_single)
        api.reduce(rws, n, wl["bins"], S // 2 * wl["dt"])
    single()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        single()
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    v_sweep, v_single = work / t_sweep, n * S / t_single
    return {"workload": "sweep-4096", "value": v_sweep, "unit": "particle-steps/s",
            "ms": t_sweep * 1e3, "particle_steps": work, "scheme": wl["scheme"],
            "single_set_value": v_single, "single_set_config": f"{n} particles x {S} steps",
            "ratio_to_single_set": v_sweep / v_single,
            "masked_lane_fraction": 1.0 - work / lanes,
            "finite_sets": int(np.isfinite(mean_v).sum())}


def adjoint_bench(reps: int = 10, scheme: str = "em", ckpt: int | None = None) -> dict:
    """Cost of the checkpointed adjoint (forward with checkpoints + backward) relative to the
    plain forward of the same ensemble and scheme: 65536 particles, 1e4 steps, W = 2000,
    checkpoints every K = 100 steps unless `ckpt` is given."""
    import numpy as np
    import torch

    from paper_1104_2499_amd import adjoint, api
    from paper_1104_2499_amd.workloads import BASE_PARAMS, WORKLOADS

    wl = WORKLOADS["adjoint-64k"]
    n, S, W = wl["n"], wl["steps"], wl["window"]
    K = wl["ckpt"] if ckpt is None else ckpt
    stream = torch.cuda.current_stream()
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=K, seed=wl["seed"], scheme=scheme)
    theta = torch.tensor([[BASE_PARAMS[k] for k in adjoint.GRAD_KEYS]], dtype=torch.float64)
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(1, cfg)
    gloss = torch.ones(1, dtype=torch.float64, device="cuda")
    state, snap = api.State.empty(n), api.State.empty(n)
    rws = api.reduce_workspace(n, 0)

    def plain():
        api.reset_state(state, wl["seed"])
        api.integrate(state, S, BASE_PARAMS, wl["dt"], scheme, wl["seed"], 0, 0, S - W, snap, rws,
                      0)
        return api.reduce(rws, n, 0, W * wl["dt"])[0]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    # five interleaved trials of each; medians (the one-wavefront-per-SIMD plain forward varies by
    # a few percent from run to run)
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    trials = [(timed(plain),
               timed(lambda: adjoint.forward(rows, cfg, ws, status=status, check_status=False)),
               timed(lambda: adjoint.backward(rows, cfg, ws, gloss, status=status,
                                              check_status=False)))
              for _ in range(5)]
    t_plain, t_fwd, t_bwd = (float(np.median([t[i] for t in trials])) for i in range(3))
    api.check_device_status(status, "adjoint")
    loss = float(adjoint.forward(rows, cfg, ws)[0].cpu())
    mean_v = float(plain()[0].cpu())
    return {"workload": "adjoint-64k", "scheme": scheme, "ckpt": K,
            "workspace_bytes": int(ws.numel()), "plain_forward_ms": t_plain,
            "adjoint_forward_ms": t_fwd,
            "adjoint_backward_ms": t_bwd, "cost_ratio": (t_fwd + t_bwd) / t_plain,
            "plain_forward_particle_steps_per_s": n * S / (t_plain * 1e-3),
            "loss_equals_forward_mean": loss == mean_v,
            "particle_steps": n * S}


def adjoint_batched_bench(stage: int, ckpt: int, reps: int = 3) -> dict:
    """One iteration of the batched-adjoint workload (1024 sets x 1024 particles x 5e4 EM steps,
    W = 1e4): forward with checkpoints and backward, for a register staging length and a
    checkpoint interval; medians of `reps` timed iterations after one warm-up."""
    import numpy as np
    import torch

    from paper_1104_2499_amd import adjoint
    from paper_1104_2499_amd.optimize import initial_theta
    from paper_1104_2499_amd.workloads import WORKLOADS

    wl = WORKLOADS["adjoint-batched-1k"]
    theta = torch.tensor(initial_theta(wl["n_sets"], wl["seed"]))
    cfg = adjoint.AdjointConfig(n=wl["n"], steps=wl["steps"], window=wl["window"], ckpt=ckpt,
                                seed=wl["seed"], stage=stage)
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(wl["n_sets"], cfg)
    gloss = torch.ones(wl["n_sets"], dtype=torch.float64, device="cuda")
    adjoint.forward(rows, cfg, ws)
    adjoint.backward(rows, cfg, ws, gloss)
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    times = []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        adjoint.forward(rows, cfg, ws, status=status, check_status=False)
        ev[1].record()
        adjoint.backward(rows, cfg, ws, gloss, status=status, check_status=False)
        ev[2].record()
        ev[2].synchronize()
        times.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])))
    from paper_1104_2499_amd import api
    api.check_device_status(status, "adjoint")
    nbytes = int(ws.numel())
    del ws
    torch.cuda.empty_cache()
    return {"workload": "adjoint-batched-1k", "stage": stage, "ckpt": ckpt,
            "workspace_bytes": nbytes,
            "forward_ms": float(np.median([t[0] for t in times])),
            "backward_ms": float(np.median([t[1] for t in times]))}


def adjoint_batched_item(iters: int = 50) -> dict:
    """The batched-adjoint workload (1024 sets x 1024 particles x 5e4 EM steps, W = 1e4; K = 48,
    16-step staging, two wavefronts per SIMD): one forward + backward iteration against the plain
    batched forward of the same sets, then the 50-iteration Adam loop on (U0, a, d2) with the exact
    pathwise gradient (the headline item), and beside it the same loop on the decayed estimator
    (look-back 1000 steps)."""
    import numpy as np
    import torch

    from paper_1104_2499_amd import api, optimize
    from paper_1104_2499_amd.adjoint import AdjointConfig, param_rows
    from paper_1104_2499_amd.workloads import WORKLOADS

    wl = WORKLOADS["adjoint-batched-1k"]
    it = adjoint_batched_bench(wl["stage"], wl["ckpt"], reps=2)
    # the plain batched integrator on the same sets and initial parameters
    theta = torch.tensor(optimize.initial_theta(wl["n_sets"], wl["seed"]))
    cfg = AdjointConfig(n=wl["n"], steps=wl["steps"], window=wl["window"], seed=wl["seed"])
    buf = api.SweepBuffers.make(param_rows(theta, cfg), np.full(wl["n_sets"], wl["n"], np.int32),
                                np.full(wl["n_sets"], wl["steps"], np.int64),
                                np.full(wl["n_sets"], wl["window"], np.int64), bins=0)

    def plain():
        api.sweep_enqueue(buf, wl["dt"], "em", wl["seed"], 0)
    plain_ms = _gpu_ms(plain, 2)
    api.check_device_status(buf.status, "sweep")
    del buf
    def adam(lookback: int, estimator: str) -> dict:
        r = optimize.adam_ratchet(wl["n_sets"], wl["n"], wl["steps"], wl["window"], wl["ckpt"],
                                  iters, wl["seed"], lookback=lookback, stage=wl["stage"])
        torch.cuda.empty_cache()
        return {"iterations": iters, "estimator": estimator, "seconds": r.seconds,
                "mean_abs_v_start": float(r.history[0]), "mean_abs_v_end": float(r.history[-1]),
                "mean_abs_v_rose": bool(r.history[-1] > r.history[0]),
                "final_loss_equals_plain_forward": bool(np.array_equal(r.final_loss,
                                                                       r.verify_mean_v))}
    exact = adam(0, "exact pathwise gradient")
    decayed = adam(1000, "decayed adjoint, look-back 1000 steps")
    return {"workload": "adjoint-batched-1k", "scheme": "em", "ckpt": wl["ckpt"],
            "stage": wl["stage"], "forward_ms": it["forward_ms"], "backward_ms": it["backward_ms"],
            "plain_forward_ms": plain_ms,
            "cost_ratio": (it["forward_ms"] + it["backward_ms"]) / plain_ms,
            "adam": exact, "adam_decayed": decayed}


def adjoint_gradient_snr() -> list[dict]:
    """How informative the per-set gradients of the batched-adjoint sets are (1024 sets x 1024
    particles, EM, dt = 1e-3, the Adam loop's initial parameters, K = 48): for the exact pathwise
    gradient at a short (1e4 steps, W = 2e3) and at the workload's horizon (5e4, W = 1e4), and the
    decayed estimator (look-back 1000) at the latter, per set and per Adam parameter (U0, a, d2)
    the |mean| of the per-particle gradients over its standard error, and their RMS; beside them
    the objective's own |<v>| over its standard error from the plain batched forward. Medians
    over the sets."""
    import numpy as np
    import torch

    from paper_1104_2499_amd import adjoint, api
    from paper_1104_2499_amd.optimize import initial_theta
    from paper_1104_2499_amd.workloads import WORKLOADS

    wl = WORKLOADS["adjoint-batched-1k"]
    n_sets, n = wl["n_sets"], wl["n"]
    theta = torch.tensor(initial_theta(n_sets, wl["seed"]))
    cols = [adjoint.GRAD_KEYS.index(k) for k in ("U0", "a", "d2")]
    out = []
    for steps, window, lookback in ((10_000, 2_000, 0), (wl["steps"], wl["window"], 0),
                                    (wl["steps"], wl["window"], 1000)):
        cfg = adjoint.AdjointConfig(n=n, steps=steps, window=window, ckpt=wl["ckpt"],
                                    seed=wl["seed"], lookback=lookback, stage=wl["stage"])
        rows = adjoint.param_rows(theta, cfg)
        buf = api.SweepBuffers.make(rows, np.full(n_sets, n, np.int32),
                                    np.full(n_sets, steps, np.int64),
                                    np.full(n_sets, window, np.int64), bins=0)
        api.sweep_enqueue(buf, wl["dt"], "em", wl["seed"], 0)
        torch.cuda.synchronize()
        api.check_device_status(buf.status, "sweep")
        mv = buf.out.cpu().numpy()
        del buf
        ws = adjoint.workspace(n_sets, cfg)
        loss = adjoint.forward(rows, cfg, ws)
        _, gp = adjoint.backward(rows, cfg, ws, torch.ones(n_sets, dtype=torch.float64),
                                 per_particle=True)
        g = gp[:, :, cols].cpu().numpy()  # statistics on the host
        snr = np.abs(g.mean(1)) / (g.std(1, ddof=1) / n ** 0.5)
        rms = np.sqrt((g * g).mean(1))
        del ws, gp
        torch.cuda.empty_cache()
        out.append({"workload": "adjoint-batched-1k", "steps": steps, "window": window,
                    "estimator": "exact" if lookback == 0 else f"lookback {lookback}",
                    "loss_equals_plain_forward": bool(np.array_equal(loss.cpu().numpy(),
                                                                     mv[:, 0])),
                    "objective_abs_over_stderr": float(np.median(np.abs(mv[:, 0]) / mv[:, 1])),
                    "grad_abs_over_stderr": dict(zip(("U0", "a", "d2"),
                                                     np.median(snr, 0).tolist())),
                    "sets_with_grad_over_2_stderr": dict(zip(("U0", "a", "d2"),
                                                             (snr > 2).mean(0).tolist())),
                    "grad_rms": dict(zip(("U0", "a", "d2"), np.median(rms, 0).tolist()))})
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ensemble-1m-heun",
                    choices=["ensemble-1m-heun", "ensemble-1k-em"])
    ap.add_argument("--sim-steps", type=int, default=None,
                    help="override the SDE step count (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 4096-set sweep line item")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device copy (reference for HBM counters)")
    ap.add_argument("--tune", default="auto",
                    help='launch shapes: "auto" (the autotuner\'s, tuned once per device and '
                         'cached), "default" (the library\'s) or block,ppl,unroll[,lookahead]')
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint cost measurements (EM and Heun), one JSON line each")
    ap.add_argument("--adjoint-ckpt", type=int, nargs="*", default=None,
                    help="checkpoint intervals for --adjoint-only (default: the workload's)")
    ap.add_argument("--adjoint-batched", action="store_true",
                    help="only one batched-adjoint iteration per (staging, K) variant")
    ap.add_argument("--adjoint-snr", action="store_true",
                    help="only the signal-to-noise of the batched-adjoint gradients, one JSON line "
                         "per horizon and estimator")
    ap.add_argument("--cpu-baselines", action="store_true",
                    help="only the FP64 oracle on every workload (all host cores and one) beside "
                         "the GPU time of the same workload, one JSON line each")
    args = ap.parse_args()

    if args.cpu_baselines:
        for r in cpu_baselines_all():
            print(json.dumps(r), flush=True)
        return 0

    if args.adjoint_batched:
        for stage, ckpt in ((16, 48), (16, 64), (16, 80), (16, 160), (8, 48), (8, 80), (8, 160)):
            print(json.dumps(adjoint_batched_bench(stage, ckpt)), flush=True)
        return 0

    if args.adjoint_snr:
        for r in adjoint_gradient_snr():
            print(json.dumps(r), flush=True)
        return 0

    if args.adjoint_only:
        for ckpt in args.adjoint_ckpt or [None]:
            for scheme in ("em", "heun"):
                print(json.dumps(adjoint_bench(scheme=scheme, ckpt=ckpt)), flush=True)
        return 0

    if args.copy_probe:
        # a plain device-to-device copy of known size: the reference that scales the HBM
        # counters (FETCH_SIZE, WRITE_SIZE) of the integrator's profile
        import torch

        nbytes = 1 << 29
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}), flush=True)
        return 0

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the ensemble would "
              "shard by particles or parameter sets); run with --gpus 1", file=sys.stderr)
        return 2

    # the instruction-mix ceiling, measured in a child process before this one touches the GPU
    ceiling = mix_ceiling()

    import torch

    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import BASE_PARAMS, WORKLOADS

    wl = dict(WORKLOADS[args.workload])
    if args.sim_steps:
        wl["steps"] = args.sim_steps
        wl["window"] = args.sim_steps // 2
    n, S, W, bins, dt, seed = wl["n"], wl["steps"], wl["window"], wl["bins"], wl["dt"], wl["seed"]
    tune = tune_batched = tune_em = None
    if args.tune == "auto":
        from paper_1104_2499_amd import tune as autotune

        tune = autotune.tune("forward", wl["scheme"])
        if not args.no_sweep:
            tune_batched = autotune.tune("batched", WORKLOADS["sweep-4096"]["scheme"])
            tune_em = autotune.tune("forward", WORKLOADS["sweep-4096"]["scheme"])
    elif args.tune != "default":
        fields = [int(t) for t in args.tune.split(",")]
        tune = dict(zip(("block", "ppl", "unroll", "lookahead"), fields))
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

    kern_all = [a.elapsed_time(b) for a, b in ev]
    kern_ms = sum(kern_all) / len(kern_all)
    kern_sd = (sum((t - kern_ms) ** 2 for t in kern_all) / max(1, len(kern_all) - 1)) ** 0.5
    ps = n * S
    value = ps * args.steps / wall
    scheme = wl["scheme"]
    kern_rate = ps / (kern_ms * 1e-3)          # particle-steps/s of the integrator kernel
    achieved = FLOP_PER_STEP[scheme] * kern_rate / 1e12
    kernel = "k_integrate_" + scheme
    traffic = load_traffic(kernel, args.workload)
    lane_instr = VALU_INSTR_PER_STEP[scheme] * kern_rate
    # the same instruction mix replayed without dependencies at full residency (8 wavefronts per
    # SIMD) sets the ceiling: 8 particle-steps per lane per trip on every lane of every SIMD
    n_simd = torch.cuda.get_device_properties(dev).multi_processor_count * 4
    trip_ns = ceiling[scheme][8]
    ceiling_rate = n_simd * 64 * STEPS_PER_TRIP / (trip_ns * 1e-9)
    trans_rate = TRANS_PER_STEP[scheme] * kern_rate
    trans_peak = N_SIMD * 64 / (TRANS_NS_PER_WAVE_INSTR * 1e-9)
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": kernel, "kernel_ms": kern_ms,
                     "kernel_ms_sd": kern_sd,
                     "flop_per_particle_step": FLOP_PER_STEP[scheme],
                     "counted_flop_per_particle_step": COUNTED_FLOP_PER_STEP[scheme],
                     "counted_tflops": COUNTED_FLOP_PER_STEP[scheme] * kern_rate / 1e12,
                     "valu_issue": {"instr_per_particle_step": VALU_INSTR_PER_STEP[scheme],
                                    "lane_instr_per_s": lane_instr,
                                    "mix_ceiling_trip_ns": trip_ns,
                                    "mix_ceiling_particle_steps_per_s": ceiling_rate,
                                    "kernel_over_mix_ceiling": kern_rate / ceiling_rate,
                                    "mix_trip_ns_by_waves_per_simd": ceiling[scheme]},
                     "transcendental": {"per_particle_step": TRANS_PER_STEP[scheme],
                                        "per_s": trans_rate, "peak_per_s": trans_peak,
                                        "frac": trans_rate / trans_peak}},
        "result": {"mean_v": float(o[0]), "stderr": float(o[1]),
                   "hist_total": int(hist.sum().item())},
    }
    if not args.no_sweep:
        line["sweep"] = sweep_bench(tune_batched=tune_batched, tune_single=tune_em)
        line["sweep"]["tuning"] = {"batched": tune_batched or "default",
                                   "single_set": tune_em or "default"}
        line["adjoint"] = adjoint_bench()
        line["adjoint_heun"] = adjoint_bench(scheme="heun")
        line["adjoint_batched"] = adjoint_batched_item()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, BASE_PARAMS)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
