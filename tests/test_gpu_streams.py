"""Independent calls enqueued at once on separate streams (all of default priority) give the bits
they give one after the other on one stream: the entry points keep nothing between calls besides
the caller's buffers. Three single-set runs (both schemes, ragged sizes), a sweep and an adjoint
forward + backward are all in flight together before one synchronisation."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

RUNS = [(70_000, 3000, "em", 5), (50_000, 2000, "heun", 6), (1000, 5000, "em", 7)]


def _run(api, n, steps, scheme, seed, stream):
    with torch.cuda.stream(stream):
        st = api.init_state(n, seed, stream=stream)
        snap = api.State.empty(n)
        ws = api.reduce_workspace(n, 256)
        api.integrate(st, steps, None, 1e-3, scheme, seed, 0, 0, steps // 2, snap, ws, 256,
                      None, stream)
        out, hist = api.reduce(ws, n, 256, steps // 2 * 1e-3, stream)
    return st, out, hist, snap, ws  # every buffer stays alive until the synchronisation


def _sweep(api, adjoint, stream):
    cfg = adjoint.AdjointConfig()
    theta = torch.tensor([[1.0 + 0.1 * k, 0.05 * k, 0.1, 1.0, 1.0, 0.1, 1.0, 0.0]
                          for k in range(6)], dtype=torch.float64)
    with torch.cuda.stream(stream):
        buf = api.SweepBuffers.make(adjoint.param_rows(theta, cfg, device="cpu"),
                                    np.array([64, 100, 700, 1, 65, 3000], np.int32),
                                    np.array([1000, 2500, 800, 3000, 1200, 600], np.int64))
        api.sweep_enqueue(buf, 1e-3, "em", 11, 256, stream=stream)
    return buf


def _adjoint(adjoint, stream):
    cfg = adjoint.AdjointConfig(n=3000, steps=2000, window=500, ckpt=100, seed=9, scheme="heun")
    theta = torch.tensor([[1.0, 0.25, 0.1, 1.0, 1.0, 0.1, 1.0, 0.0],
                          [1.4, 0.10, 0.3, 0.5, 1.0, 0.1, 1.0, 0.0]], dtype=torch.float64)
    with torch.cuda.stream(stream):
        rows = adjoint.param_rows(theta, cfg)
        ws = adjoint.workspace(2, cfg)
        status = torch.empty(1, dtype=torch.int32, device="cuda")
        loss = adjoint.forward(rows, cfg, ws, stream=stream, status=status, check_status=False)
        grad = adjoint.backward(rows, cfg, ws, torch.ones(2, dtype=torch.float64),
                                stream=stream, status=status, check_status=False)
    return loss, grad, status, ws


def _host(run):
    st, out, hist = run[:3]
    return (st.cell.cpu().numpy(), st.xf.cpu().numpy(), st.v.cpu().numpy(), st.e.cpu().numpy(),
            st.lo.cpu().numpy(), out.cpu().numpy(), hist.cpu().numpy())


def test_concurrent_streams_give_sequential_bits(gpu):
    from paper_1104_2499_amd import adjoint, api

    main = torch.cuda.current_stream()
    ref_runs = []
    for case in RUNS:
        print(f"sequential run {case}", flush=True)
        ref_runs.append(_host(_run(api, *case, main)))
        torch.cuda.synchronize()
    buf = _sweep(api, adjoint, main)
    torch.cuda.synchronize()
    api.check_device_status(buf.status, "sweep")
    ref_sweep = (buf.out.cpu().numpy(), buf.hist.cpu().numpy())
    loss, grad, status, _ = _adjoint(adjoint, main)
    torch.cuda.synchronize()
    api.check_device_status(status, "adjoint")
    ref_adj = (loss.cpu().numpy(), grad.cpu().numpy())

    print("all at once on five streams", flush=True)
    streams = [torch.cuda.Stream() for _ in range(len(RUNS) + 2)]
    torch.cuda.synchronize()
    runs = [_run(api, *case, s) for case, s in zip(RUNS, streams)]
    buf2 = _sweep(api, adjoint, streams[-2])
    adj2 = _adjoint(adjoint, streams[-1])
    torch.cuda.synchronize()

    for case, got, ref in zip(RUNS, runs, ref_runs):
        for a, b in zip(_host(got), ref):
            np.testing.assert_array_equal(a, b, err_msg=str(case))
    api.check_device_status(buf2.status, "sweep")
    np.testing.assert_array_equal(buf2.out.cpu().numpy(), ref_sweep[0])
    np.testing.assert_array_equal(buf2.hist.cpu().numpy(), ref_sweep[1])
    api.check_device_status(adj2[2], "adjoint")
    np.testing.assert_array_equal(adj2[0].cpu().numpy(), ref_adj[0])
    np.testing.assert_array_equal(adj2[1].cpu().numpy(), ref_adj[1])
    assert np.isfinite(ref_adj[1]).all() and np.isfinite(ref_sweep[0]).all()
