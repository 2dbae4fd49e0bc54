"""Property checks of the workspace-size queries of include/abp.h over their whole argument ranges
(hypothesis; no device needed): no query crashes or wraps around, a size is 0 exactly when the
arguments break the documented limits, and a nonzero size holds every array the layout places in
it, with at most the alignment padding on top."""
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

MAX_PARTICLES = 1 << 31
MAX_STEP = 1 << 34
MAX_SETS = 1 << 20
MAX_TILES = 0x7FFFFFFF

I32 = st.integers(-(1 << 31), (1 << 31) - 1)
I64 = st.integers(-(1 << 63), (1 << 63) - 1)


def _bins_ok(b):
    return b == 0 or (0 < b <= 4096 and b & (b - 1) == 0)


def _near(limit):
    """Values around a limit, where off-by-one mistakes live."""
    return st.integers(limit - 3, limit + 3)


BINS = st.one_of(st.sampled_from([0, 1, 2, 3, 256, 4095, 4096, 4097, 8192, -1, -256]), I32)


@settings(max_examples=1500, deadline=None)
@given(n=st.one_of(st.integers(-3, 5000), _near(MAX_PARTICLES), I64), bins=BINS)
def test_reduce_workspace_query(lib, n, bins):
    got = lib.abp_reduce_workspace_bytes(n, bins)
    if not (1 <= n <= MAX_PARTICLES and _bins_ok(bins)):
        assert got == 0
        return
    tiles = (n + 63) // 64
    need = 16 * tiles + 4 * bins  # FP64 (sum, sum of squares) per tile, u32 per bin
    assert need <= got <= need + 2 * 256 and got % 256 == 0


@settings(max_examples=1500, deadline=None)
@given(n_sets=st.one_of(st.integers(-3, 3000), _near(MAX_SETS), I32),
       extra=st.one_of(st.integers(-3, 5000), _near(MAX_TILES), I64), bins=BINS)
def test_batched_workspace_query(lib, n_sets, extra, bins):
    n_tiles = max(n_sets, 0) + extra
    if not -(1 << 63) <= n_tiles < (1 << 63):
        return
    got = lib.abp_batched_workspace_bytes(n_sets, n_tiles, bins)
    if not (1 <= n_sets <= MAX_SETS and n_sets <= n_tiles <= MAX_TILES and _bins_ok(bins)):
        assert got == 0
        return
    # per set: an 80-byte constant row, its rank (4 B), its item offset (8 B) and its bins (4 B
    # each); per tile: an 8-byte work item and two FP64 partials; 16 bytes of control words
    need = n_sets * (80 + 4 + 8 + 4 * bins) + n_tiles * (8 + 16) + 16
    assert need <= got <= need + 7 * 256 and got % 256 == 0


@settings(max_examples=2000, deadline=None)
@given(n_sets=st.one_of(st.integers(-2, 2000), I32),
       n=st.one_of(st.integers(-2, 100_000), _near(MAX_PARTICLES), I64),
       S=st.one_of(st.integers(-2, 200_000), _near(MAX_STEP), I64),
       K=st.one_of(st.integers(-2, 300), st.integers(1, 1 << 40), I64))
def test_adjoint_workspace_query(lib, n_sets, n, S, K):
    got = lib.abp_adjoint_workspace_bytes(n_sets, n, S, K)
    if not (n_sets >= 1 and n >= 1 and S >= 1 and K >= 1 and n_sets * n <= MAX_PARTICLES
            and S <= MAX_STEP):
        assert got == 0
        return
    Ke = (min(K, S) + 15) // 16 * 16  # the interval rounded up to the 16-step staging grid
    lanes = n_sets * ((n + 63) // 64) * 64
    slots = (S + Ke - 1) // Ke + Ke // 8  # checkpoints and one segment's sub-window slots
    planes = 28 * lanes * slots
    if planes >= 1 << 62:
        assert got == 0  # refused rather than wrapped
        return
    tiles = n_sets * ((n + 63) // 64)
    need = planes + 96 * n_sets + 4 + 8 * (2 + 8) * tiles  # rows, status, loss and grad partials
    assert need <= got <= need + 6 * 256 and got % 256 == 0


@pytest.mark.parametrize("status", [-(1 << 31), -1, 5, 6, 99, (1 << 31) - 1])
def test_status_string_of_any_code(lib, status):
    assert lib.abp_status_str(status) == b"unknown status"


@settings(max_examples=1500, deadline=None)
@given(n_steps=st.one_of(st.integers(-2, 1000), _near(MAX_STEP), I64),
       step0=st.one_of(st.integers(-2, 1000), _near(MAX_STEP), I64),
       win=st.one_of(st.integers(-3, 2000), I64),
       stride=st.one_of(st.integers(-2, 100), st.integers(1, 1 << 40), I64))
def test_integrate_run_checks(lib, n_steps, step0, win, stride):
    """abp_integrate's step-range checks over the whole int64 range (no sum may overflow): a run
    is accepted (ABP_E_DEVICE on this host, which has no gfx950) exactly when 0 <= n_steps,
    0 <= step0 and step0 + n_steps <= 2^34, win_begin >= -1, and a time-histogram stride >= 0
    whose sample count stays within the u32 bound; otherwise ABP_E_ARG."""
    import ctypes

    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present: a valid call would run on the placeholder pointers")
    from paper_1104_2499_amd import _lib
    from paper_1104_2499_amd.api import make_params

    p = make_params()
    state = _lib.AbpState(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 64, 0, 0)
    snap = _lib.AbpState(0x2000, 0x2000, 0x2000, 0x2000, 0x2000, 64, 0, 0)
    r = _lib.AbpRun(1e-3, n_steps, step0, win, 42, 0, 0, stride, 0x10000, 64)
    got = lib.abp_integrate(ctypes.byref(p), ctypes.byref(r), ctypes.byref(state),
                            ctypes.byref(snap), None, 0, 0, None, None)
    valid = (0 <= n_steps <= MAX_STEP and 0 <= step0 and step0 + n_steps <= MAX_STEP
             and win >= -1 and stride >= 0
             and (stride == 0 or (n_steps // stride + 1) * 256 <= 0xFFFFFFFF))
    assert got == (_lib.ABP_E_DEVICE if valid else _lib.ABP_E_ARG)
