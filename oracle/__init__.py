"""FP64 CPU oracle for the active-Brownian-particle ensemble integrator -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. It is a thin ctypes binding over ``abp_oracle.c`` (plain C, IEEE double, OpenMP over
particles), which shares no code with the HIP library.

Model: Zabicki, "OpenCL/OpenGL approach for studying active Brownian motion", Sec. 2, Eqs. (1)-(3);
loop shape: Fig. 1 (random draw -> Box-Muller -> update, per step). Noise: Philox4x32-10
(Salmon et al., SC'11) with counter (step/4, particle, set, domain) and key = 64-bit seed.

Parameters are passed as a dict with the keys of ``PARAM_KEYS``; missing keys default to the
workload values (gamma0 = d2 = q = 1, c = 0.1, D = 0.1, U0 = 1, a = 0.25, F0 = phi = 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "abp_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

PARAM_KEYS = ("U0", "a", "phi", "gamma0", "F0", "d2", "q", "c", "D")
DEFAULTS = dict(U0=1.0, a=0.25, phi=0.0, gamma0=1.0, F0=0.0, d2=1.0, q=1.0, c=0.1, D=0.1)
GRAD_KEYS = ("U0", "a", "D", "d2", "q", "c", "gamma0", "F0")
EM, HEUN = 0, 1


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, IEEE: no fast-math, OpenMP)."""
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", SRC, "-o", LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in PARAM_KEYS]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64, u64, u32, i32, f64 = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                               ctypes.c_double)
    lib.orc_philox_many.argtypes = [i64, vp, vp, vp]
    lib.orc_normals.argtypes = [u64, u32, u32, i64, i64, vp]
    lib.orc_init_state.argtypes = [i64, u64, u32, vp, vp, vp, vp]
    lib.orc_potential.argtypes = [P(_Params), f64]
    lib.orc_potential.restype = f64
    lib.orc_integrate.argtypes = [P(_Params), ctypes.c_int, f64, i64, i64, i64, u64, u32, i64, vp,
                                  vp, vp, vp, vp, vp, f64]
    lib.orc_integrate.restype = ctypes.c_int
    lib.orc_reduce.argtypes = [i64, vp, vp, f64, i32, vp, vp]
    lib.orc_rk4.argtypes = [P(_Params), f64, i64, i64, vp, vp, vp]
    lib.orc_adjoint.argtypes = [P(_Params), ctypes.c_int, f64, i64, i64, u64, u32, i64, vp, vp,
                                vp, vp, vp, vp, f64, i64]
    lib.orc_adjoint.restype = ctypes.c_int
    lib.orc_complex_step.argtypes = [P(_Params), ctypes.c_int, ctypes.c_int, f64, f64, i64, i64,
                                     u64, u32, i64, vp, vp, vp, vp, vp, vp]
    lib.orc_complex_step.restype = ctypes.c_int
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _params(p: dict | None) -> _Params:
    d = dict(DEFAULTS)
    if p:
        unknown = set(p) - set(PARAM_KEYS)
        if unknown:
            raise KeyError(f"unknown parameter(s) {sorted(unknown)}")
        d.update(p)
    return _Params(*[float(d[k]) for k in PARAM_KEYS])


def _ptr(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _ids(ids, n):
    if ids is None:
        return None
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    if ids.shape != (n,):
        raise ValueError("ids must have one entry per particle")
    return ids


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Use n threads in later calls (timing only; results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of each row: ctr [m,4] u32, key [m,2] u32 -> [m,4] u32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    if ctr.shape[0] != key.shape[0]:
        raise ValueError("ctr and key must have the same number of rows")
    out = np.empty_like(ctr)
    _load().orc_philox_many(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def normals(seed: int, particle: int, set_id: int, step0: int, count: int) -> np.ndarray:
    """The normals xi_n, n in [step0, step0+count), of one particle's noise stream."""
    z = np.empty(count, dtype=np.float64)
    _load().orc_normals(seed, particle, set_id, step0, count, _ptr(z))
    return z


def init_state(n: int, seed: int, set_id: int = 0, ids=None):
    """x0 ~ U[0,1) (24-bit, exact), v0 = e0 = 0. Returns (x, v, e) float64 arrays."""
    x = np.empty(n, np.float64); v = np.empty(n, np.float64); e = np.empty(n, np.float64)
    ids = _ids(ids, n)
    _load().orc_init_state(n, seed, set_id, _ptr(ids), _ptr(x), _ptr(v), _ptr(e))
    return x, v, e


def potential(params: dict | None, x: float) -> float:
    p = _params(params)
    return float(_load().orc_potential(ctypes.byref(p), float(x)))


def integrate(params: dict | None, x, v, e, n_steps: int, dt: float = 1e-3, scheme: int = EM,
              seed: int = 42, set_id: int = 0, step0: int = 0, win_begin: int = -1, ids=None,
              x_snap=None, v_sum=None, eps: float = 0.0):
    """Advance copies of (x, v, e) by n_steps from absolute step step0.

    Returns (x, v, e, x_snap, v_sum). ``x_snap`` holds x at absolute index ``win_begin`` when the
    window opens inside [step0, step0 + n_steps] and is carried in from ``x_snap`` otherwise;
    ``v_sum`` accumulates v_n over window steps (time-average estimator). ``eps`` != 0 applies
    the rounding-sensitivity model after each step (x += eps u, v and e scaled by 1 + eps u)."""
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    e = np.array(e, dtype=np.float64, copy=True)
    n = x.shape[0]
    xs = np.full(n, np.nan) if x_snap is None else np.array(x_snap, dtype=np.float64, copy=True)
    vs = np.zeros(n) if v_sum is None else np.array(v_sum, dtype=np.float64, copy=True)
    ids = _ids(ids, n)
    p = _params(params)
    rc = _load().orc_integrate(ctypes.byref(p), scheme, dt, step0, n_steps, win_begin, seed,
                               set_id, n, _ptr(ids), _ptr(x), _ptr(v), _ptr(e), _ptr(xs), _ptr(vs),
                               float(eps))
    if rc != 0:
        raise ValueError("oracle integrate rejected its arguments")
    return x, v, e, xs, vs


def reduce(x_snap, x_end, window_time: float, n_bins: int = 256):
    """(mean velocity, standard error, uint64 histogram of x_end mod 1)."""
    xs = np.ascontiguousarray(x_snap, dtype=np.float64)
    xe = np.ascontiguousarray(x_end, dtype=np.float64)
    out = np.zeros(2)
    hist = np.zeros(max(n_bins, 1), dtype=np.uint64)
    _load().orc_reduce(xs.shape[0], _ptr(xs), _ptr(xe), window_time, n_bins, _ptr(out),
                       _ptr(hist))
    return float(out[0]), float(out[1]), hist[:n_bins]


def occupancy(params: dict | None, x, v, e, n_steps: int, stride: int, n_bins: int = 256,
              dt: float = 1e-3, scheme: int = EM, seed: int = 42, set_id: int = 0,
              step0: int = 0, ids=None):
    """Time-accumulated histogram of x mod 1: the particle density displayed while the ensemble
    runs (Sec. 2). By definition the sum, over the absolute steps n in (step0, step0 + n_steps]
    that are multiples of `stride`, of the histogram of the positions x_n; computed here as
    integrate to each such n, then reduce's histogram. Returns (hist, x, v, e) at the end."""
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    e = np.array(e, dtype=np.float64, copy=True)
    acc = np.zeros(n_bins, dtype=np.uint64)
    end = step0 + n_steps
    at = step0
    for target in range((step0 // stride + 1) * stride, end + 1, stride):
        x, v, e, _, _ = integrate(params, x, v, e, target - at, dt, scheme, seed, set_id, at,
                                  ids=ids)
        at = target
        acc += reduce(x, x, 1.0, n_bins)[2]
    x, v, e, _, _ = integrate(params, x, v, e, end - at, dt, scheme, seed, set_id, at, ids=ids)
    return acc, x, v, e


def rk4(params: dict | None, x, v, e, n_steps: int, dt: float):
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    e = np.array(e, dtype=np.float64, copy=True)
    p = _params(params)
    _load().orc_rk4(ctypes.byref(p), dt, n_steps, x.shape[0], _ptr(x), _ptr(v), _ptr(e))
    return x, v, e


def adjoint(params: dict | None, x0, v0, e0, n_steps: int, window: int, dt: float = 1e-3,
            seed: int = 42, set_id: int = 0, ids=None, eps: float = 0.0, lookback: int = 0,
            scheme: int = EM):
    """Per-particle J_i = (x_S - x_{S-W})/(W dt) and dJ_i/d(U0, a, D, d2, q, c, gamma0, F0)
    [n, 8] by the discrete adjoint of the scheme (EM or Heun) with the full trajectory stored.
    eps != 0 linearises around the path perturbed by the rounding-sensitivity model (a
    conditioning probe). lookback = T > 0 (EM only) gives the decayed estimator (each window
    velocity's sensitivity damped by 1 - 1/T per step)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    e0 = np.ascontiguousarray(e0, dtype=np.float64)
    n = x0.shape[0]
    J = np.empty(n); g = np.empty((n, len(GRAD_KEYS)))
    ids = _ids(ids, n)
    p = _params(params)
    rc = _load().orc_adjoint(ctypes.byref(p), scheme, dt, n_steps, window, seed, set_id, n,
                             _ptr(ids), _ptr(x0), _ptr(v0), _ptr(e0), _ptr(J), _ptr(g),
                             float(eps), int(lookback))
    if rc != 0:
        raise ValueError(f"oracle adjoint failed (rc={rc})")
    return J, g


def complex_step(params: dict | None, which: int, x0, v0, e0, n_steps: int, window: int,
                 dt: float = 1e-3, seed: int = 42, set_id: int = 0, ids=None, h: float = 1e-30,
                 scheme: int = EM):
    """Per-particle dJ_i/dtheta_which (GRAD_KEYS order) by the complex-step method; also
    returns Re J_i."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    e0 = np.ascontiguousarray(e0, dtype=np.float64)
    n = x0.shape[0]
    dJ = np.empty(n); Jre = np.empty(n)
    ids = _ids(ids, n)
    p = _params(params)
    rc = _load().orc_complex_step(ctypes.byref(p), scheme, which, h, dt, n_steps, window, seed,
                                  set_id, n, _ptr(ids), _ptr(x0), _ptr(v0), _ptr(e0), _ptr(dJ),
                                  _ptr(Jre))
    if rc != 0:
        raise ValueError("oracle complex step rejected its arguments")
    return dJ, Jre
