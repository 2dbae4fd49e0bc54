"""Python front end of libabp: torch tensors for device memory and streams, ctypes for the calls.

Every numerical step runs in the HIP library; this module only allocates buffers, fills the ABI
structs and checks status codes.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .workloads import BASE_PARAMS, PARAM_KEYS

SCHEMES = {"em": _lib.ABP_EM, "heun": _lib.ABP_HEUN}


class AbpError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        msg = lib.abp_status_str(status).decode()
        super().__init__(f"{where}: {_lib.STATUS_NAMES.get(status, status)} ({msg})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != _lib.ABP_OK:
        raise AbpError(status, where)


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p | None:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def scheme_id(scheme) -> int:
    if isinstance(scheme, str):
        return SCHEMES[scheme.lower()]
    return int(scheme)


def make_params(params: dict | None = None) -> _lib.AbpParams:
    d = dict(BASE_PARAMS)
    if params:
        unknown = set(params) - set(PARAM_KEYS)
        if unknown:
            raise KeyError(f"unknown parameter(s) {sorted(unknown)}")
        d.update(params)
    return _lib.AbpParams(*[float(d[k]) for k in PARAM_KEYS])


def make_tuning(tune, kind: str = "forward", scheme="em", n: int | None = None
                ) -> _lib.AbpTuning | None:
    """ABI tuning from None (library default), a dict of launch-shape fields, or "auto" (the
    shape the autotuner cached for this device, kernel kind, scheme and -- for an ensemble of n
    particles -- occupancy band; default if none)."""
    if isinstance(tune, str):
        if tune != "auto":
            raise ValueError('tune must be None, a dict of launch-shape fields, or "auto"')
        from . import tune as _tune

        name = scheme.lower() if isinstance(scheme, str) else (
            "em" if scheme == _lib.ABP_EM else "heun")
        tune = _tune.lookup(kind, name, n)
    if tune is None:
        return None
    if isinstance(tune, _lib.AbpTuning):
        return tune
    t = dict(tune)
    return _lib.AbpTuning(int(t.get("block", 0)), int(t.get("ppl", 0)), int(t.get("unroll", 0)),
                          int(t.get("waves_per_simd", 0)), int(t.get("lookahead", 0)))


@dataclass
class State:
    """Structure-of-arrays particle state on the device, FP32 high/low pairs:
    x = cell + xf + lo[0], v = v + lo[1], e = e + lo[2] (lo has shape [3, n])."""
    cell: torch.Tensor
    xf: torch.Tensor
    v: torch.Tensor
    e: torch.Tensor
    lo: torch.Tensor
    id0: int = 0

    @property
    def n(self) -> int:
        return self.cell.numel()

    @staticmethod
    def empty(n: int, device="cuda", id0: int = 0) -> "State":
        f = dict(dtype=torch.float32, device=device)
        return State(torch.empty(n, dtype=torch.int32, device=device), torch.empty(n, **f),
                     torch.empty(n, **f), torch.empty(n, **f), torch.empty((3, n), **f), id0)

    def clone(self) -> "State":
        return State(self.cell.clone(), self.xf.clone(), self.v.clone(), self.e.clone(),
                     self.lo.clone(), self.id0)

    def tensors(self):
        return (self.cell, self.xf, self.v, self.e, self.lo)

    def abi(self) -> _lib.AbpState:
        n = self.n
        for t, dt, k in ((self.cell, torch.int32, n), (self.xf, torch.float32, n),
                         (self.v, torch.float32, n), (self.e, torch.float32, n),
                         (self.lo, torch.float32, 3 * n)):
            if t.dtype != dt or not t.is_contiguous() or t.numel() != k:
                raise ValueError("state tensors must be contiguous int32/float32 of sizes n,n,n,n,3n")
        return _lib.AbpState(self.cell.data_ptr(), self.xf.data_ptr(), self.v.data_ptr(),
                             self.e.data_ptr(), self.lo.data_ptr(), n, self.id0, 0)

    def x64(self) -> torch.Tensor:
        """Positions (cell + xf) + lx in float64, as the library evaluates them."""
        return (self.cell.double() + self.xf.double()) + self.lo[0].double()

    def v64(self) -> torch.Tensor:
        return self.v.double() + self.lo[1].double()

    def e64(self) -> torch.Tensor:
        return self.e.double() + self.lo[2].double()


def reset_state(s: State, seed: int, set_id: int = 0, stream=None) -> State:
    """Write the workload initial condition (x0 ~ U[0,1) from Philox, v0 = e0 = 0) into `s`."""
    abi = s.abi()
    check(_lib.load().abp_init_state(ctypes.byref(abi), seed, set_id, _stream(stream)),
          "abp_init_state")
    return s


def init_state(n: int, seed: int, set_id: int = 0, id0: int = 0, device="cuda",
               stream=None) -> State:
    return reset_state(State.empty(n, device, id0), seed, set_id, stream)


def philox(ctr: torch.Tensor, key: torch.Tensor, stream=None) -> torch.Tensor:
    """Philox4x32-10 on the device; ctr [m,4] and key [m,2] int32 tensors holding u32 bits."""
    if ctr.dtype != torch.int32 or key.dtype != torch.int32:
        raise TypeError("ctr and key must be int32 tensors (u32 bit patterns)")
    ctr = ctr.contiguous()
    key = key.contiguous()
    m = ctr.shape[0]
    out = torch.empty((m, 4), dtype=torch.int32, device=ctr.device)
    check(_lib.load().abp_philox(m, _ptr(ctr), _ptr(key), _ptr(out), _stream(stream)),
          "abp_philox")
    return out


def reduce_workspace(n: int, n_bins: int, device="cuda") -> torch.Tensor:
    nbytes = int(_lib.load().abp_reduce_workspace_bytes(n, n_bins))
    if nbytes == 0:
        raise ValueError("invalid reduction size")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def integrate(state: State, n_steps: int, params: dict | None = None, dt: float = 1e-3,
              scheme="em", seed: int = 42, set_id: int = 0, step0: int = 0, win_begin: int = -1,
              snap: State | None = None, ws: torch.Tensor | None = None, n_bins: int = 0,
              tune=None, stream=None, hist_stride: int = 0,
              hist_acc: torch.Tensor | None = None) -> None:
    """Advance `state` in place (abp_integrate). With `ws`, also leave the reduction partials.
    hist_stride > 0 adds x mod 1 at every absolute step that is a multiple of it to hist_acc
    (int64 [bins] on the device, holding u64 counts; the caller zeroes it)."""
    p = make_params(params)
    r = _lib.AbpRun(dt, n_steps, step0, win_begin, seed, set_id, scheme_id(scheme))
    if hist_stride:
        if hist_acc is None or hist_acc.dtype != torch.int64 or not hist_acc.is_contiguous():
            raise ValueError("hist_stride needs hist_acc: a contiguous int64 device tensor")
        r.hist_stride, r.d_hist_acc, r.hist_bins = hist_stride, hist_acc.data_ptr(), hist_acc.numel()
    s = state.abi()
    sn = snap.abi() if snap is not None else None
    t = make_tuning(tune, "forward", scheme, state.n)
    check(_lib.load().abp_integrate(ctypes.byref(p), ctypes.byref(r), ctypes.byref(s),
                                    ctypes.byref(sn) if sn is not None else None, _ptr(ws),
                                    0 if ws is None else ws.numel(), n_bins,
                                    ctypes.byref(t) if t is not None else None, _stream(stream)),
          "abp_integrate")


def reduce(ws: torch.Tensor, n: int, n_bins: int, window_time: float, stream=None):
    """(mean velocity, standard error) as a float64 [2] tensor and the uint64 histogram."""
    out = torch.empty(2, dtype=torch.float64, device=ws.device)
    hist = torch.empty(max(n_bins, 1), dtype=torch.int64, device=ws.device)
    check(_lib.load().abp_reduce(_ptr(ws), ws.numel(), n, n_bins, window_time, _ptr(out),
                                 _ptr(hist) if n_bins > 0 else None, _stream(stream)),
          "abp_reduce")
    return out, hist[:n_bins]


def reduce_state(snap: State, end: State, n_bins: int, ws: torch.Tensor, stream=None) -> None:
    a, b = snap.abi(), end.abi()
    check(_lib.load().abp_reduce_state(ctypes.byref(a), ctypes.byref(b), n_bins, _ptr(ws),
                                       ws.numel(), _stream(stream)), "abp_reduce_state")


@dataclass
class Result:
    mean_v: float
    stderr: float
    hist: torch.Tensor
    state: State
    snap: State
    occupancy: torch.Tensor | None = None  # time-accumulated histogram (hist_stride > 0)


def run(params: dict | None = None, n: int = 1024, steps: int = 10_000, window: int | None = None,
        dt: float = 1e-3, scheme="em", seed: int = 42, bins: int = 256, set_id: int = 0,
        tune=None, device="cuda", stream=None, hist_stride: int = 0) -> Result:
    """Initial condition, `steps` steps, window mean velocity over the last `window` steps
    (default: the last half) and the histogram of the final x mod 1; with hist_stride > 0 also
    the histogram of x mod 1 accumulated every hist_stride steps (bins bins)."""
    window = steps // 2 if window is None else window
    if not 1 <= window <= steps:
        raise ValueError("need 1 <= window <= steps")
    st = init_state(n, seed, set_id, device=device, stream=stream)
    snap = State.empty(n, device)
    ws = reduce_workspace(n, bins, device)
    occ = torch.zeros(bins, dtype=torch.int64, device=device) if hist_stride else None
    integrate(st, steps, params, dt, scheme, seed, set_id, 0, steps - window, snap, ws, bins,
              tune, stream, hist_stride, occ)
    out, hist = reduce(ws, n, bins, window * dt, stream)
    o = out.cpu()
    return Result(float(o[0]), float(o[1]), hist, st, snap, occ)


@dataclass
class SweepResult:
    mean_v: np.ndarray   # [n_sets] float64
    stderr: np.ndarray   # [n_sets] float64
    hist: torch.Tensor   # [n_sets, n_bins] int64 (u64 counts) on the device


def params_table(table) -> np.ndarray:
    """[n_sets, 9] float64 in PARAM_KEYS order from an array or a list of dicts."""
    if isinstance(table, np.ndarray):
        t = np.ascontiguousarray(table, dtype=np.float64)
    else:
        t = np.array([[float(dict(BASE_PARAMS, **row)[k]) for k in PARAM_KEYS] for row in table],
                     dtype=np.float64)
    if t.ndim != 2 or t.shape[1] != len(PARAM_KEYS):
        raise ValueError("parameter table must be [n_sets, 9]")
    return t


def n_tiles(n_traj) -> int:
    """Tiles of 64 particles over all sets: the size the batched workspace is queried with."""
    nt = np.asarray(n_traj, dtype=np.int64)
    return int(((nt + 63) // 64).sum())


def batched_workspace(n_sets: int, tiles: int, n_bins: int, device="cuda") -> torch.Tensor:
    nbytes = int(_lib.load().abp_batched_workspace_bytes(n_sets, tiles, n_bins))
    if nbytes == 0:
        raise ValueError("invalid batched sweep sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@dataclass
class SweepBuffers:
    """Device tables and outputs of one sweep shape (reused across calls and graph replays)."""
    params: torch.Tensor   # [n_sets, 9] float64
    ntraj: torch.Tensor    # [n_sets] int32
    nsteps: torch.Tensor   # [n_sets] int64
    window: torch.Tensor | None  # [n_sets] int64, or None for n_steps // 2
    ws: torch.Tensor
    out: torch.Tensor      # [n_sets, 2] float64
    hist: torch.Tensor     # [n_sets, max(bins, 1)] int64 (u64 counts)
    status: torch.Tensor   # [1] int32, the device-side status

    @staticmethod
    def make(table, n_traj, n_steps, window=None, bins: int = 256, ws=None,
             device="cuda") -> "SweepBuffers":
        t = table if torch.is_tensor(table) else torch.from_numpy(params_table(table))
        nt = torch.as_tensor(n_traj, dtype=torch.int32)
        ns = torch.as_tensor(n_steps, dtype=torch.int64)
        win = None if window is None else torch.as_tensor(window, dtype=torch.int64)
        if t.ndim != 2 or t.shape[1] != len(PARAM_KEYS):
            raise ValueError("parameter table must be [n_sets, 9]")
        n_sets = t.shape[0]
        if nt.shape != (n_sets,) or ns.shape != (n_sets,):
            raise ValueError("n_traj and n_steps need one entry per set")
        if win is not None and win.shape != (n_sets,):
            raise ValueError("window needs one entry per set")
        if ws is None:
            ws = batched_workspace(n_sets, n_tiles(nt.cpu().numpy()), bins, device)

        def dev(x, dtype):
            return None if x is None else x.to(device=device, dtype=dtype).contiguous()

        out = torch.empty((n_sets, 2), dtype=torch.float64, device=device)
        hist = torch.empty((n_sets, max(bins, 1)), dtype=torch.int64, device=device)
        status = torch.empty(1, dtype=torch.int32, device=device)
        return SweepBuffers(dev(t, torch.float64), dev(nt, torch.int32), dev(ns, torch.int64),
                            dev(win, torch.int64), ws, out, hist, status)


def sweep_enqueue(buf: SweepBuffers, dt: float = 1e-3, scheme="em", seed: int = 11,
                  bins: int = 256, tune=None, stream=None) -> None:
    """Enqueue abp_integrate_batched on the buffers' device tables (no host wait; capturable).
    The device-side status lands in buf.status."""
    cfg = _lib.AbpBatch(dt, seed, scheme_id(scheme), bins)
    tn = make_tuning(tune, "batched", scheme)
    check(_lib.load().abp_integrate_batched(
        buf.params.shape[0], _ptr(buf.params), _ptr(buf.ntraj), _ptr(buf.nsteps),
        _ptr(buf.window), ctypes.byref(cfg), ctypes.byref(tn) if tn is not None else None,
        _ptr(buf.ws), buf.ws.numel(), _ptr(buf.out), _ptr(buf.hist) if bins > 0 else None,
        _ptr(buf.status), _stream(stream)), "abp_integrate_batched")


def check_device_status(status: torch.Tensor, where: str) -> None:
    """Raise AbpError if a device-side status word holds an error (waits for it)."""
    check(int(status.item()), where + " (device tables)")


def sweep(table, n_traj, n_steps, window=None, dt: float = 1e-3, scheme="em", seed: int = 11,
          bins: int = 256, tune=None, ws: torch.Tensor | None = None, device="cuda",
          stream=None) -> SweepResult:
    """One persistent launch over many parameter sets (abp_integrate_batched). Set k runs
    n_traj[k] particles for n_steps[k] steps with Philox set id k and averages over the last
    window[k] steps (default n_steps[k] // 2). Host tables are uploaded to the device first."""
    buf = SweepBuffers.make(table, n_traj, n_steps, window, bins, ws, device)
    sweep_enqueue(buf, dt, scheme, seed, bins, tune, stream)
    if stream is not None:
        stream.synchronize()
    check_device_status(buf.status, "abp_integrate_batched")
    o = buf.out.cpu().numpy()
    return SweepResult(o[:, 0].copy(), o[:, 1].copy(), buf.hist[:, :bins])
