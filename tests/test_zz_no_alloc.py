"""The allocation-free entry point against abp_integrate + abp_reduce, through the C ABI: the same
state, snapshot, mean velocity, standard error and histogram, bit for bit, on two calls in a row
(the second on a smaller ensemble, so that stale scratch contents from the first would show)."""
import ctypes

import pytest
import torch

from paper_1104_2499_amd import _lib, api

pytestmark = pytest.mark.gpu


def _reference(n, steps, window, scheme, bins, seed):
    st = api.init_state(n, seed)
    snap = api.State.empty(n)
    ws = api.reduce_workspace(n, bins)
    api.integrate(st, steps, None, 1e-3, scheme, seed, 0, 0, steps - window, snap, ws, bins)
    out, hist = api.reduce(ws, n, bins, window * 1e-3)
    return st, snap, out, hist


def _noalloc(lib, n, steps, window, scheme, bins, seed):
    st = api.init_state(n, seed)
    snap = api.State.empty(n)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    hist = torch.full((max(bins, 1),), -1, dtype=torch.int64, device="cuda")
    p = api.make_params(None)
    r = _lib.AbpRun(1e-3, steps, 0, steps - window, seed, 0, api.scheme_id(scheme))
    s, sn = st.abi(), snap.abi()
    status = lib.abp_integrate_reduce_noalloc(
        ctypes.byref(p), ctypes.byref(r), ctypes.byref(s), ctypes.byref(sn), bins,
        window * 1e-3, ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(hist.data_ptr()) if bins > 0 else None, None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    api.check(status, "abp_integrate_reduce_noalloc")
    return st, snap, out, hist[:bins]


def _same(a, b):
    ta, tb = a.tensors(), b.tensors()
    return all(torch.equal(x, y) for x, y in zip(ta, tb))


@pytest.mark.parametrize("cases", [
    [(5000, 1200, 600, "em", 256, 42), (700, 1000, 300, "heun", 64, 7)],
    [(1 << 20, 400, 200, "heun", 256, 3), (130, 403, 17, "em", 4096, 5)],
])
def test_noalloc_matches_integrate_and_reduce(gpu, cases):
    for n, steps, window, scheme, bins, seed in cases:
        print(f"noalloc case n={n} steps={steps} window={window} {scheme} bins={bins}", flush=True)
        ref = _reference(n, steps, window, scheme, bins, seed)
        got = _noalloc(gpu, n, steps, window, scheme, bins, seed)
        torch.cuda.synchronize()
        assert _same(ref[0], got[0]) and _same(ref[1], got[1])
        assert torch.equal(ref[2], got[2]), (ref[2].tolist(), got[2].tolist())
        assert torch.equal(ref[3], got[3])
        assert int(got[3].sum()) == n


def test_noalloc_rejects_ensembles_past_its_scratch(gpu):
    n = _lib.NOALLOC_MAX_PARTICLES + 1
    st = api.State.empty(n)
    snap = api.State.empty(n)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    hist = torch.zeros(256, dtype=torch.int64, device="cuda")
    p = api.make_params(None)
    r = _lib.AbpRun(1e-3, 8, 0, 4, 1, 0, 0)
    s, sn = st.abi(), snap.abi()
    assert gpu.abp_integrate_reduce_noalloc(
        ctypes.byref(p), ctypes.byref(r), ctypes.byref(s), ctypes.byref(sn), 256, 4e-3,
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(hist.data_ptr()), None,
        None) == _lib.ABP_E_WORKSPACE
