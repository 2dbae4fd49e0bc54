"""ctypes binding of libabp.so (include/abp.h). Argument marshalling only.

The library is built in-tree by ``paper_1104_2499_amd.build``; if it is missing, ``load()`` raises:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

from .workloads import PARAM_KEYS

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libabp.so")

ABP_OK, ABP_E_ARG, ABP_E_HIP, ABP_E_WORKSPACE, ABP_E_DEVICE = range(5)
ABP_EM, ABP_HEUN = 0, 1
ABI_VERSION = 4
NOALLOC_MAX_PARTICLES = 1 << 24
STATUS_NAMES = {0: "ABP_OK", 1: "ABP_E_ARG", 2: "ABP_E_HIP", 3: "ABP_E_WORKSPACE",
                4: "ABP_E_DEVICE"}


class AbpParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in PARAM_KEYS]


class AbpRun(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("n_steps", ctypes.c_int64), ("step0", ctypes.c_int64),
                ("win_begin", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("set_id", ctypes.c_uint32), ("scheme", ctypes.c_int32),
                ("hist_stride", ctypes.c_int64), ("d_hist_acc", ctypes.c_void_p),
                ("hist_bins", ctypes.c_int32), ("pad", ctypes.c_int32)]


class AbpState(ctypes.Structure):
    _fields_ = [("d_cell", ctypes.c_void_p), ("d_xf", ctypes.c_void_p), ("d_v", ctypes.c_void_p),
                ("d_e", ctypes.c_void_p), ("d_lo", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("id0", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class AbpTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("ppl", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("lookahead", ctypes.c_int32)]


class AbpBatch(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("seed", ctypes.c_uint64), ("scheme", ctypes.c_int32),
                ("n_bins", ctypes.c_int32)]


class AbpAdjointCfg(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("n_steps", ctypes.c_int64), ("window", ctypes.c_int64),
                ("ckpt_every", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("lookback", ctypes.c_int64), ("scheme", ctypes.c_int32),
                ("stage_steps", ctypes.c_int32)]


_P = ctypes.POINTER
_vp, _i32, _i64, _u32, _u64, _f64, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_size_t)

# name -> (restype, argtypes); mirrors include/abp.h
SIGNATURES = {
    "abp_abi_version": (ctypes.c_int, []),
    "abp_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "abp_init_state": (ctypes.c_int, [_P(AbpState), _u64, _u32, _vp]),
    "abp_philox": (ctypes.c_int, [_i64, _vp, _vp, _vp, _vp]),
    "abp_reduce_workspace_bytes": (_sz, [_i64, _i32]),
    "abp_integrate": (ctypes.c_int, [_P(AbpParams), _P(AbpRun), _P(AbpState), _P(AbpState), _vp,
                                     _sz, _i32, _P(AbpTuning), _vp]),
    "abp_reduce": (ctypes.c_int, [_vp, _sz, _i64, _i32, _f64, _vp, _vp, _vp]),
    "abp_reduce_state": (ctypes.c_int, [_P(AbpState), _P(AbpState), _i32, _vp, _sz, _vp]),
    "abp_integrate_reduce_noalloc": (ctypes.c_int, [_P(AbpParams), _P(AbpRun), _P(AbpState),
                                                    _P(AbpState), _i32, _f64, _vp, _vp,
                                                    _P(AbpTuning), _vp]),
    "abp_batched_workspace_bytes": (_sz, [_i32, _i64, _i32]),
    "abp_integrate_batched": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _P(AbpBatch),
                                             _P(AbpTuning), _vp, _sz, _vp, _vp, _vp, _vp]),
    "abp_adjoint_workspace_bytes": (_sz, [_i32, _i64, _i64, _i64]),
    "abp_adjoint": (ctypes.c_int, [_i32, _i32, _vp, _i64, _P(AbpAdjointCfg), _vp, _sz, _vp, _vp,
                                   _vp, _vp, _vp, _vp]),
}


class LibraryMissing(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load libabp.so once and attach the signatures.

    torch is imported first so that libabp.so binds to the HIP runtime torch has loaded (both
    carry the soname libamdhip64.so.7): the library runs on torch's streams and memory, and one
    process must not hold two HIP runtimes."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} is not built; run `python -m paper_1104_2499_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
