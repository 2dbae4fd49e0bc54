"""The library under HIP graph capture. Every entry point only enqueues kernels (no host
synchronisation, no copies, no memset nodes): the single-set path (abp_init_state, abp_integrate
with its fused reduction and time-accumulated histogram, abp_reduce), the batched sweep with its
device-side plan, and the adjoint's forward and backward phases are each captured once and
replayed. Every replay is checked against the eager result, with eager work on the device
between replays."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

BASE = dict(U0=1.0, a=0.25, phi=0.0, gamma0=1.0, F0=0.0, d2=1.0, q=1.0, c=0.1, D=0.1)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_captured_run_replays_bit_identically(gpu, scheme):
    from paper_1104_2499_amd import api

    n, S, W, bins = 4000, 600, 300, 64
    st, snap = api.State.empty(n), api.State.empty(n)
    ws = api.reduce_workspace(n, bins)
    acc = torch.zeros(bins, dtype=torch.int64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    hist = torch.empty(bins, dtype=torch.int64, device="cuda")

    def run():
        api.reset_state(st, 17)
        acc.zero_()  # a fill kernel, not a memset node
        api.integrate(st, S, BASE, scheme=scheme, seed=17, win_begin=S - W, snap=snap, ws=ws,
                      n_bins=bins, hist_stride=50, hist_acc=acc)
        o, h = api.reduce(ws, n, bins, W * 1e-3)
        out.copy_(o)
        hist.copy_(h)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()  # warm-up (first calls cache the device check) outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    want = (out.clone(), hist.clone(), acc.clone(), st.xf.clone(), st.lo.clone())

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for i in range(3):
        for t in (out, hist, acc, st.xf, st.lo):
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = (out, hist, acc, st.xf, st.lo)
        for a_, b_ in zip(got, want):
            assert torch.equal(a_, b_), (i, scheme)
        assert torch.isfinite(junk)
    assert int(want[2].sum()) == n * (S // 50)
    np.testing.assert_array_equal(want[1].cpu().numpy().sum(), n)


def _replay_and_check(g, outs, want, label):
    for i in range(3):
        for t in outs:
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for a_, b_ in zip(outs, want):
            assert torch.equal(a_, b_), (label, i)
        assert torch.isfinite(junk)


def _warm(fn):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_captured_sweep_replays_bit_identically(gpu, scheme):
    """abp_integrate_batched reads device tables and plans its work list on the device, so the
    whole sweep (plan, persistent launch, finalize) is captured once and replayed; every replay
    equals the eager sweep and the sets equal their single runs."""
    from paper_1104_2499_amd import _lib, api
    from paper_1104_2499_amd.workloads import sweep_table

    table, _, _ = sweep_table(9, seed=4)
    n_traj = np.array([1, 64, 65, 300, 7, 129, 1000, 2, 513], dtype=np.int32)
    n_steps = np.array([5, 400, 1, 801, 33, 640, 250, 3, 99], dtype=np.int64)
    window = np.maximum(1, n_steps // 3)
    bins = 32
    buf = api.SweepBuffers.make(table, n_traj, n_steps, window, bins)

    def run():
        api.sweep_enqueue(buf, scheme=scheme, seed=23, bins=bins)

    _warm(run)
    assert int(buf.status.item()) == _lib.ABP_OK
    want = (buf.out.clone(), buf.hist.clone(), buf.status.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    _replay_and_check(g, (buf.out, buf.hist, buf.status), want, "sweep")
    from paper_1104_2499_amd.workloads import PARAM_KEYS

    for k in (0, 3, 8):
        params = {key: float(table[k, i]) for i, key in enumerate(PARAM_KEYS)}
        a = api.run(params, n=int(n_traj[k]), steps=int(n_steps[k]), window=int(window[k]),
                    scheme=scheme, seed=23, bins=bins, set_id=k)
        assert float(want[0][k, 0]) == a.mean_v and float(want[0][k, 1]) == a.stderr
        assert torch.equal(want[1][k], a.hist)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_captured_adjoint_replays_bit_identically(gpu, scheme):
    """abp_adjoint (forward with checkpoints, then backward) reads its parameter rows on the
    device and only enqueues: captured once, every replay gives the eager loss and gradient."""
    from paper_1104_2499_amd import _lib, adjoint
    from paper_1104_2499_amd.workloads import PARAM_KEYS

    n_sets = 3
    cfg = adjoint.AdjointConfig(n=200, steps=500, window=120, ckpt=48, seed=31, scheme=scheme)
    base = torch.tensor([[BASE[k] for k in adjoint.GRAD_KEYS]], dtype=torch.float64)
    theta = base.repeat(n_sets, 1)
    theta[:, 0] *= torch.tensor([1.0, 1.2, 0.8], dtype=torch.float64)
    rows = adjoint.param_rows(theta, cfg)
    assert rows.shape == (n_sets, len(PARAM_KEYS))
    ws = adjoint.workspace(n_sets, cfg)
    loss = torch.empty(n_sets, dtype=torch.float64, device="cuda")
    grad = torch.empty((n_sets, len(adjoint.GRAD_KEYS)), dtype=torch.float64, device="cuda")
    gloss = torch.ones(n_sets, dtype=torch.float64, device="cuda")
    status = torch.empty(1, dtype=torch.int32, device="cuda")

    def run():
        adjoint.forward(rows, cfg, ws, status=status, loss=loss, check_status=False)
        adjoint.backward(rows, cfg, ws, gloss, status=status, grad=grad, check_status=False)

    _warm(run)
    assert int(status.item()) == _lib.ABP_OK
    want = (loss.clone(), grad.clone(), status.clone())
    assert torch.isfinite(want[0]).all() and torch.isfinite(want[1]).all()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    _replay_and_check(g, (loss, grad, status), want, "adjoint")
