"""CPU checks of the C ABI: the library builds, loads, exports every declared entry point, and
rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abp_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_1104_2499_amd import _lib

    names = declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no Python binding"


def test_version_and_status_strings(lib):
    from paper_1104_2499_amd import _lib

    assert lib.abp_abi_version() == _lib.ABI_VERSION
    for s in range(5):
        assert lib.abp_status_str(s)
    assert lib.abp_status_str(99) == b"unknown status"


def test_workspace_queries(lib):
    assert lib.abp_reduce_workspace_bytes(0, 256) == 0
    assert lib.abp_reduce_workspace_bytes(100, 3) == 0
    assert lib.abp_reduce_workspace_bytes(100, 8192) == 0
    a = lib.abp_reduce_workspace_bytes(1 << 20, 256)
    assert a >= (1 << 14) * 16 + 256 * 4
    assert lib.abp_reduce_workspace_bytes(64, 0) >= 16


def test_adjoint_workspace_sizes(lib):
    """28 bytes per lane per checkpoint segment plus the sub-window slots of one segment; a K
    beyond the run behaves as one segment; sizes past 2^62 bytes are refused (0)."""
    one = lib.abp_adjoint_workspace_bytes(1, 65536, 10_000, 100)   # K -> 112, 90 segments
    assert 28 * 65536 * (90 + 14) <= one <= 28 * 65536 * (90 + 14) + 65536 * 100
    assert lib.abp_adjoint_workspace_bytes(1, 64, 100, 10**15) == \
        lib.abp_adjoint_workspace_bytes(1, 64, 100, 100)
    assert lib.abp_adjoint_workspace_bytes(1, 1 << 31, 1 << 34, 16) == 0
    assert lib.abp_adjoint_workspace_bytes(0, 64, 100, 10) == 0
    assert lib.abp_adjoint_workspace_bytes(1, 64, 100, 0) == 0
    assert lib.abp_adjoint_workspace_bytes(1, 64, (1 << 34) + 1, 10) == 0


def _state(n=64, ptr=0x1000, id0=0):
    from paper_1104_2499_amd import _lib

    return _lib.AbpState(ptr, ptr, ptr, ptr, ptr, n, id0, 0)


def test_integrate_rejects_bad_arguments_without_a_device(lib):
    from paper_1104_2499_amd import _lib
    from paper_1104_2499_amd.api import make_params

    p = make_params()
    good = _lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0)
    s = _state()
    E_ARG = _lib.ABP_E_ARG

    def call(p_=p, r=good, s_=s, snap=None, ws=None, wsb=0, bins=0, tune=None):
        return lib.abp_integrate(ctypes.byref(p_) if p_ is not None else None,
                                 ctypes.byref(r) if r is not None else None,
                                 ctypes.byref(s_) if s_ is not None else None,
                                 ctypes.byref(snap) if snap is not None else None,
                                 ws, wsb, bins, ctypes.byref(tune) if tune else None, None)

    assert call(p_=None) == E_ARG
    assert call(r=None) == E_ARG
    assert call(s_=None) == E_ARG
    for bad in (_lib.AbpRun(0.0, 100, 0, -1, 42, 0, 0), _lib.AbpRun(-1e-3, 100, 0, -1, 42, 0, 0),
                _lib.AbpRun(float("nan"), 100, 0, -1, 42, 0, 0),
                _lib.AbpRun(1e-3, -1, 0, -1, 42, 0, 0), _lib.AbpRun(1e-3, 100, -4, -1, 42, 0, 0),
                _lib.AbpRun(1e-3, 1 << 34, 1, -1, 42, 0, 0),
                _lib.AbpRun(1e-3, 100, 0, -2, 42, 0, 0), _lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 7)):
        assert call(r=bad) == E_ARG
    assert call(s_=_state(n=0)) == E_ARG
    assert call(s_=_state(ptr=0x1002)) == E_ARG            # misaligned
    assert call(s_=_state(n=10, id0=0xFFFFFFFF)) == E_ARG   # ids overflow 32 bits
    assert call(s_=_state(n=(1 << 31) + 1)) == E_ARG        # past the largest ensemble
    bad_p = make_params(dict(D=-0.1))
    assert call(p_=bad_p) == E_ARG
    assert call(p_=make_params(dict(U0=float("inf")))) == E_ARG
    # window inside the call but no snapshot buffer
    assert call(r=_lib.AbpRun(1e-3, 100, 0, 50, 42, 0, 0)) == E_ARG
    # reduction without a window, or with bad bins / small workspace
    ws = 0x10000
    assert call(ws=ws, wsb=1 << 20, bins=256, snap=_state()) == E_ARG
    win = _lib.AbpRun(1e-3, 100, 0, 50, 42, 0, 0)
    assert call(r=win, ws=ws, wsb=1 << 20, bins=100, snap=_state()) == E_ARG
    assert call(r=win, ws=ws, wsb=16, bins=256, snap=_state()) == _lib.ABP_E_WORKSPACE
    # time-accumulated histogram: negative stride, bad bins, missing or misaligned array
    for stride, ptr, bins_ in ((-1, 0x10000, 64), (10, 0x10000, 0), (10, 0x10000, 48),
                               (10, 0x10000, 8192), (10, 0, 64), (10, 0x10004, 64)):
        assert call(r=_lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0, stride, ptr, bins_)) == E_ARG
    assert call(r=_lib.AbpRun(1e-3, 1 << 24, 0, -1, 42, 0, 0, 1, 0x10000, 64)) == E_ARG
    assert call(tune=_lib.AbpTuning(96, 1, 1, 0)) == E_ARG
    assert call(tune=_lib.AbpTuning(256, 3, 1, 0)) == E_ARG
    assert call(tune=_lib.AbpTuning(256, 1, 4, 0)) == E_ARG
    assert call(tune=_lib.AbpTuning(256, 1, 2, 0, 2)) == E_ARG  # look-ahead needs unroll 1
    assert call(tune=_lib.AbpTuning(256, 1, 1, 0, 3)) == E_ARG


def test_valid_call_without_gpu_reports_device(lib):
    """On this host there is no gfx950 device: a valid call must say so, not crash or compute."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1104_2499_amd import _lib
    from paper_1104_2499_amd.api import make_params

    p = make_params()
    r = _lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0)
    s = _state()
    st = lib.abp_integrate(ctypes.byref(p), ctypes.byref(r), ctypes.byref(s), None, None, 0, 0,
                           None, None)
    assert st == _lib.ABP_E_DEVICE


def test_other_entry_points_validate(lib):
    from paper_1104_2499_amd import _lib

    E_ARG = _lib.ABP_E_ARG
    assert lib.abp_philox(0, 0x1000, 0x1000, 0x1000, None) == E_ARG
    assert lib.abp_philox(4, None, 0x1000, 0x1000, None) == E_ARG
    assert lib.abp_init_state(None, 1, 0, None) == E_ARG
    assert lib.abp_reduce(None, 1 << 20, 10, 256, 1.0, 0x1000, 0x1000, None) == E_ARG
    assert lib.abp_reduce(0x10000, 1 << 20, 10, 256, 0.0, 0x1000, 0x1000, None) == E_ARG
    assert lib.abp_reduce(0x10000, 1 << 20, 10, 256, 1.0, 0x1000, None, None) == E_ARG
    # a workspace shorter than the query for (n, n_bins) is refused before any device access
    need = lib.abp_reduce_workspace_bytes(1 << 20, 256)
    assert lib.abp_reduce(0x10000, need - 1, 1 << 20, 256, 1.0, 0x1000, 0x1000,
                          None) == _lib.ABP_E_WORKSPACE
    a, b = _state(), _state(n=32)
    assert lib.abp_reduce_state(ctypes.byref(a), ctypes.byref(b), 256, 0x10000, 1 << 20,
                                None) == E_ARG
    b = _state()
    assert lib.abp_reduce_state(ctypes.byref(a), ctypes.byref(b), 256, 0x10000, 8,
                                None) == _lib.ABP_E_WORKSPACE


def test_parameters_that_overflow_fp32_are_rejected(lib):
    """The kernels run on FP32 coefficients: finite FP64 values that overflow FP32 (or a time
    step that rounds to zero, or 1 / (2D) past the FP32 range in the adjoint) are invalid
    arguments, reported before anything is enqueued (no device is needed to see that)."""
    from paper_1104_2499_amd import _lib
    from paper_1104_2499_amd.api import make_params

    E_ARG = _lib.ABP_E_ARG
    s = _state()
    run = _lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0)
    bad_params = [dict(U0=1e39), dict(d2=1e39), dict(F0=3.5e38), dict(gamma0=-1e39),
                  dict(D=1e300)]
    for bad in bad_params:
        p = make_params(bad)
        assert lib.abp_integrate(ctypes.byref(p), ctypes.byref(run), ctypes.byref(s), None, None,
                                 0, 0, None, None) == E_ARG, bad
    tiny_dt = _lib.AbpRun(1e-50, 100, 0, -1, 42, 0, 0)
    p = make_params()
    assert lib.abp_integrate(ctypes.byref(p), ctypes.byref(tiny_dt), ctypes.byref(s), None, None,
                             0, 0, None, None) == E_ARG

    # the batched and adjoint parameter tables live on the device and are checked there
    # (tests/test_gpu_batched.py, tests/test_gpu_adjoint.py)


def test_batched_and_adjoint_validate_host_arguments(lib):
    """The scalars, pointers and workspace size of the device-table calls are checked on the host
    before anything is enqueued; the tables themselves are not read here."""
    from paper_1104_2499_amd import _lib

    E_ARG, E_WS = _lib.ABP_E_ARG, _lib.ABP_E_WORKSPACE
    assert lib.abp_batched_workspace_bytes(0, 10, 0) == 0
    assert lib.abp_batched_workspace_bytes(4, 3, 0) == 0          # fewer tiles than sets
    assert lib.abp_batched_workspace_bytes(4, 8, 100) == 0        # bins not a power of two
    assert lib.abp_batched_workspace_bytes(4, 1 << 31, 0) == 0
    assert lib.abp_batched_workspace_bytes((1 << 20) + 1, 1 << 21, 0) == 0
    small = lib.abp_batched_workspace_bytes(4, 8, 64)
    big = lib.abp_batched_workspace_bytes(4, 1000, 64)
    assert small > 0 and big - small >= 24 * 992  # 8 + 16 bytes per tile

    cfg = _lib.AbpBatch(1e-3, 11, 0, 64)
    T = 0x10000  # a stand-in device address: nothing is read on these paths

    def batched(n_sets=4, params=T, ntraj=T, nsteps=T, window=None, cfg_=cfg, ws=T,
                wsb=small, out=T, hist=T, status=None, tune=None):
        return lib.abp_integrate_batched(n_sets, params, ntraj, nsteps, window,
                                         ctypes.byref(cfg_) if cfg_ is not None else None,
                                         ctypes.byref(tune) if tune else None, ws, wsb, out,
                                         hist, status, None)

    assert batched(n_sets=0) == E_ARG
    assert batched(params=None) == E_ARG
    assert batched(params=T + 4) == E_ARG
    assert batched(ntraj=T + 2) == E_ARG
    assert batched(nsteps=None) == E_ARG
    assert batched(window=T + 4) == E_ARG
    assert batched(status=T + 2) == E_ARG
    assert batched(cfg_=None) == E_ARG
    assert batched(cfg_=_lib.AbpBatch(0.0, 11, 0, 64)) == E_ARG
    assert batched(cfg_=_lib.AbpBatch(1e-3, 11, 2, 64)) == E_ARG
    assert batched(cfg_=_lib.AbpBatch(1e-3, 11, 0, 48)) == E_ARG
    assert batched(hist=None) == E_ARG
    assert batched(ws=T + 128) == E_ARG
    assert batched(tune=_lib.AbpTuning(256, 1, 1, 9)) == E_ARG
    # a workspace without room for one tile per set
    assert batched(wsb=lib.abp_batched_workspace_bytes(4, 4, 64) - 256) == E_WS

    acfg = _lib.AbpAdjointCfg(1e-3, 100, 20, 16, 42, 0, 0, 0)
    need = lib.abp_adjoint_workspace_bytes(1, 64, 100, 16)

    def adj(phase=0, params=T, n=64, cfg_=acfg, ws=T, wsb=need, loss=T, gloss=T, grad=T,
            gp=None, status=None):
        return lib.abp_adjoint(phase, 1, params, n, ctypes.byref(cfg_), ws, wsb, loss, gloss,
                               grad, gp, status, None)

    assert adj(params=None) == E_ARG
    assert adj(params=T + 4) == E_ARG
    assert adj(loss=None) == E_ARG
    assert adj(phase=1, gloss=None) == E_ARG
    assert adj(phase=1, gp=T + 4) == E_ARG
    assert adj(status=T + 1) == E_ARG
    assert adj(cfg_=_lib.AbpAdjointCfg(1e-3, 100, 101, 16, 42, 0, 0, 0)) == E_ARG
    assert adj(cfg_=_lib.AbpAdjointCfg(1e-3, 100, 20, 16, 42, 5, 1, 0)) == E_ARG  # Heun look-back
    assert adj(cfg_=_lib.AbpAdjointCfg(1e-3, 100, 20, 16, 42, 0, 0, 12)) == E_ARG
    assert adj(wsb=need - 1) == E_WS


def test_ctypes_structs_match_the_c_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets of include/abp.h, as a C
    compiler lays them out (a mismatch would hand the library shifted arguments)."""
    import shutil
    import subprocess

    from paper_1104_2499_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"abp_params": _lib.AbpParams, "abp_run": _lib.AbpRun, "abp_state": _lib.AbpState,
               "abp_tuning": _lib.AbpTuning, "abp_batch": _lib.AbpBatch,
               "abp_adjoint_cfg": _lib.AbpAdjointCfg}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "abp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_ctypes_signatures_match_the_c_prototypes():
    """Every binding in _lib.SIGNATURES has the prototype's argument count, and each scalar
    argument and result the C type's width and signedness (pointers bound as pointers)."""
    from paper_1104_2499_amd import _lib

    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    scalar = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "uint32_t": ctypes.c_uint32,
              "uint64_t": ctypes.c_uint64, "double": ctypes.c_double, "size_t": ctypes.c_size_t,
              "int": ctypes.c_int, "abp_status": ctypes.c_int}

    def is_pointer_type(t):
        return t in (ctypes.c_void_p, ctypes.c_char_p) or (
            isinstance(t, type) and issubclass(t, ctypes._Pointer))

    protos = re.findall(r"\n([A-Za-z_][\w ]*?\*?)\s*\b(abp_\w+)\s*\(([^;]*?)\)\s*;", text)
    assert len(protos) == len(_lib.SIGNATURES)
    for ret, name, args in protos:
        restype, argtypes = _lib.SIGNATURES[name]
        ret = ret.replace("const", "").strip()
        if "*" in ret:
            assert is_pointer_type(restype), name
        else:
            assert restype is scalar[ret], (name, ret)
        args = [a.strip() for a in " ".join(args.split()).split(",")]
        if args == ["void"]:
            args = []
        assert len(args) == len(argtypes), name
        for a, t in zip(args, argtypes):
            if "*" in a:
                assert is_pointer_type(t), (name, a)
            else:
                ctype = a.replace("const ", "").rsplit(" ", 1)[0].strip()
                assert t is scalar[ctype], (name, a)


def test_noalloc_entry_point_validates(lib):
    """The allocation-free integrate + reduce checks its arguments like abp_integrate, refuses
    ensembles larger than its fixed scratch with ABP_E_WORKSPACE, and reports a missing gfx950
    device, all before anything is enqueued."""
    import torch

    from paper_1104_2499_amd import _lib
    from paper_1104_2499_amd.api import make_params

    p = make_params()
    win = _lib.AbpRun(1e-3, 100, 0, 50, 42, 0, 0)

    def call(r=win, n=64, bins=256, wt=0.05, out=0x1000, hist=0x2000):
        s, snap = _state(n=n), _state(n=n)
        return lib.abp_integrate_reduce_noalloc(ctypes.byref(p), ctypes.byref(r),
                                                ctypes.byref(s), ctypes.byref(snap), bins, wt,
                                                out, hist, None, None)

    assert call(r=_lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0)) == _lib.ABP_E_ARG  # no window
    assert call(bins=100) == _lib.ABP_E_ARG
    assert call(wt=0.0) == _lib.ABP_E_ARG
    assert call(out=None) == _lib.ABP_E_ARG
    assert call(out=0x1004) == _lib.ABP_E_ARG
    assert call(hist=None) == _lib.ABP_E_ARG
    assert call(hist=None, bins=0) != _lib.ABP_E_ARG
    assert call(n=_lib.NOALLOC_MAX_PARTICLES + 1) == _lib.ABP_E_WORKSPACE
    if not torch.cuda.is_available():
        assert call(n=_lib.NOALLOC_MAX_PARTICLES) == _lib.ABP_E_DEVICE
