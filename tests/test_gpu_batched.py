"""GPU checks of the persistent batched sweep: every set equals the same set run alone (bit for
bit, for every tuning), sets match the FP64 oracle, and the full 4096-set sweep is consistent."""
import numpy as np
import pytest
import torch


pytestmark = pytest.mark.gpu

KEYS = ("U0", "a", "phi", "gamma0", "F0", "d2", "q", "c", "D")


def _small_sweep():
    rng = np.random.default_rng(5)
    n_sets = 12
    from paper_1104_2499_amd.workloads import sweep_table

    table, _, _ = sweep_table(n_sets, seed=5)
    n_traj = np.array([1, 63, 64, 65, 200, 1000, 129, 7, 513, 64, 2, 300], dtype=np.int32)
    n_steps = np.array([1, 3, 4, 5, 401, 1000, 998, 17, 640, 2, 1203, 77], dtype=np.int64)
    window = np.maximum(1, n_steps // np.array([1, 2, 3, 2, 2, 5, 2, 3, 4, 1, 2, 7]))
    return table, n_traj, n_steps, window.astype(np.int64), rng


def _alone(k, table, n_traj, n_steps, window, scheme, seed, bins):
    from paper_1104_2499_amd import api

    params = {key: float(table[k, i]) for i, key in enumerate(KEYS)}
    return api.run(params, n=int(n_traj[k]), steps=int(n_steps[k]), window=int(window[k]),
                   scheme=scheme, seed=seed, bins=bins, set_id=k)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_each_set_equals_its_single_run_for_every_tuning(gpu, scheme):
    from paper_1104_2499_amd import api

    table, n_traj, n_steps, window, _ = _small_sweep()
    bins, seed = 32, 11
    alone = [_alone(k, table, n_traj, n_steps, window, scheme, seed, bins)
             for k in range(len(n_traj))]
    for block in (64, 256):
        for ppl in (1, 2):
            for unroll, la in ((1, 1), (1, 2), (2, 1)):
                for wps in (1, 8):
                    r = api.sweep(table, n_traj, n_steps, window, scheme=scheme, seed=seed,
                                  bins=bins, tune=dict(block=block, ppl=ppl, unroll=unroll,
                                                       waves_per_simd=wps, lookahead=la))
                    for k, a in enumerate(alone):
                        assert r.mean_v[k] == a.mean_v, (k, block, ppl, unroll, la, wps)
                        assert r.stderr[k] == a.stderr
                        assert torch.equal(r.hist[k], a.hist)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_sets_match_oracle(gpu, orc, scheme):
    from paper_1104_2499_amd import api

    table, n_traj, n_steps, window, _ = _small_sweep()
    r = api.sweep(table, n_traj, n_steps, window, scheme=scheme, seed=11, bins=64)
    for k in range(len(n_traj)):
        params = {key: float(table[k, i]) for i, key in enumerate(KEYS)}
        n = int(n_traj[k])
        x0, v0, e0 = orc.init_state(n, 11, k)
        x, v, e, xs, _ = orc.integrate(params, x0, v0, e0, int(n_steps[k]), seed=11, set_id=k,
                                       win_begin=int(n_steps[k] - window[k]),
                                       scheme=orc.EM if scheme == "em" else orc.HEUN)
        mean, se, hist = orc.reduce(xs, x, float(window[k]) * 1e-3, 64)
        assert abs(r.mean_v[k] - mean) <= 1e-5 * max(1.0, abs(mean)), k
        assert int(r.hist[k].sum()) == n


def test_full_sweep_4096_sets(gpu, orc):
    """The 4096-set ratchet sweep (D log-uniform, U0, a, d2 uniform; 64..4096 trajectories and
    2e4..2e5 steps per set) in one launch: sampled sets are bit-identical to their single runs,
    every histogram holds its set's trajectories, and a short set agrees with the oracle."""
    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import WORKLOADS, sweep_table

    wl = WORKLOADS["sweep-4096"]
    table, n_traj, n_steps = sweep_table(wl["n_sets"], seed=wl["seed"])
    r = api.sweep(table, n_traj, n_steps, scheme="em", seed=wl["seed"], bins=wl["bins"])
    np.testing.assert_array_equal(r.hist.sum(dim=1).cpu().numpy(), n_traj)
    assert np.all(np.isfinite(r.mean_v)) and np.all(r.stderr > 0)
    order = np.argsort(n_traj.astype(np.int64) * n_steps)
    for k in (int(order[0]), int(order[1]), 0, wl["n_sets"] - 1):
        a = _alone(k, table, n_traj, n_steps, n_steps // 2, "em", wl["seed"], wl["bins"])
        assert r.mean_v[k] == a.mean_v and r.stderr[k] == a.stderr
        assert torch.equal(r.hist[k], a.hist)
    k = int(order[0])
    params = {key: float(table[k, i]) for i, key in enumerate(KEYS)}
    n, S = int(n_traj[k]), int(n_steps[k])
    x0, v0, e0 = orc.init_state(n, wl["seed"], k)
    x, v, e, xs, _ = orc.integrate(params, x0, v0, e0, S, seed=wl["seed"], set_id=k,
                                   win_begin=S - S // 2)
    mean, se, _ = orc.reduce(xs, x, (S // 2) * 1e-3, wl["bins"])
    assert abs(r.mean_v[k] - mean) <= 4 * np.hypot(r.stderr[k], se)


def test_batched_rejects_bad_arguments(gpu):
    from paper_1104_2499_amd import api

    table, n_traj, n_steps, window, _ = _small_sweep()
    with pytest.raises(ValueError):
        api.batched_workspace(len(n_traj), len(n_traj) - 1, 32)
    # a window of zero steps is a bad table entry: found on the device
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        api.sweep(table, n_traj, n_steps, window * 0, bins=32)
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.AbpError, match="ABP_E_WORKSPACE"):
        api.sweep(table, n_traj, n_steps, window, bins=32, ws=ws)


def test_device_side_table_checks(gpu):
    """Table values are checked on the device: a set abp_integrate would reject (negative D, an
    FP32-overflowing U0, no trajectories, too many steps) or a work list longer than the
    workspace holds sets the device status; nothing is integrated, every mean becomes NaN and
    every count zero. A good sweep on the same buffers afterwards reports ABP_OK again."""
    from paper_1104_2499_amd import _lib, api

    table, n_traj, n_steps, window, _ = _small_sweep()
    col = {k: i for i, k in enumerate(KEYS)}
    bad_cases = []
    for key, val in (("D", -0.1), ("U0", 1e39), ("gamma0", float("nan"))):
        t = table.copy()
        t[5, col[key]] = val
        bad_cases.append((t, n_traj, n_steps, _lib.ABP_E_ARG))
    nt = n_traj.copy()
    nt[2] = 0
    bad_cases.append((table, nt, n_steps, _lib.ABP_E_ARG))
    ns = n_steps.copy()
    ns[7] = (1 << 34) + 1
    bad_cases.append((table, n_traj, ns, _lib.ABP_E_ARG))
    for t, nt, ns, code in bad_cases:
        buf = api.SweepBuffers.make(t, np.maximum(nt, 1), ns, None, 16)
        buf.ntraj.copy_(torch.as_tensor(nt))  # the workspace is sized for the valid counts
        api.sweep_enqueue(buf, bins=16)
        assert int(buf.status.item()) == code
        assert torch.isnan(buf.out).all()
        assert int(buf.hist.abs().sum()) == 0
    # tiles beyond the workspace: sized for the table, then one set grows
    buf = api.SweepBuffers.make(table, n_traj, n_steps, window, 16)
    big = n_traj.copy()
    big[0] = 64 * 10_000
    buf.ntraj.copy_(torch.as_tensor(big))
    api.sweep_enqueue(buf, bins=16)
    assert int(buf.status.item()) == _lib.ABP_E_WORKSPACE
    assert torch.isnan(buf.out).all()
    buf.ntraj.copy_(torch.as_tensor(n_traj))
    api.sweep_enqueue(buf, bins=16)
    assert int(buf.status.item()) == _lib.ABP_OK
    assert torch.isfinite(buf.out).all()
    assert torch.equal(buf.hist.sum(dim=1).cpu(), torch.as_tensor(n_traj, dtype=torch.int64))


def test_autotuner_picks_a_shape_that_changes_no_bits(gpu, tmp_path, monkeypatch):
    """The autotuner times every candidate launch shape on a small probe, caches the fastest per
    device, kernel and scheme, and api calls with tune="auto" use it; the results equal the
    default shape's bit for bit."""
    from paper_1104_2499_amd import api, tune

    monkeypatch.setenv("ABP_TUNE_CACHE", str(tmp_path / "tune.json"))
    best_f = tune.tune("forward", "em", force=True, probe=dict(n=65536 * 4, steps=400))
    best_s = tune.tune("forward-small", "em", force=True, probe=dict(n=16384, steps=400))
    best_b = tune.tune("batched", "em", force=True, probe=dict(n_sets=64, step_scale=0.01))
    assert best_f in list(tune.candidates("forward"))
    assert best_s in list(tune.candidates("forward"))
    assert best_b in list(tune.candidates("batched"))
    assert tune.lookup("forward", "em") == best_f and tune.lookup("batched", "em") == best_b
    # ensembles within two wavefronts per SIMD take the small band's shape
    assert tune.lookup("forward", "em", n=tune.small_band_limit()) == best_s
    assert tune.lookup("forward", "em", n=tune.small_band_limit() + 1) == best_f
    a = api.run(None, n=3000, steps=1001, scheme="em", seed=3, bins=64, tune="auto")
    b = api.run(None, n=3000, steps=1001, scheme="em", seed=3, bins=64)
    assert a.mean_v == b.mean_v and a.stderr == b.stderr and torch.equal(a.hist, b.hist)
    table, n_traj, n_steps, window, _ = _small_sweep()
    s1 = api.sweep(table, n_traj, n_steps, window, scheme="em", bins=16, tune="auto")
    s2 = api.sweep(table, n_traj, n_steps, window, scheme="em", bins=16)
    np.testing.assert_array_equal(s1.mean_v, s2.mean_v)
    assert torch.equal(s1.hist, s2.hist)


def test_many_small_sets_planned_on_the_device(gpu):
    """50000 sets of 1-70 particles and 2-40 steps in one launch: the device-side plan ranks sets
    across many blocks (step counts tie constantly; ties go in set order) and scans offsets over
    49 chunks of its scan block. Every histogram holds its set's particles, and sampled sets equal
    their single runs bit for bit."""
    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import sweep_table

    rng = np.random.default_rng(8)
    n_sets = 50_000
    table, _, _ = sweep_table(n_sets, seed=8)
    n_traj = rng.integers(1, 71, n_sets).astype(np.int32)
    n_steps = rng.integers(2, 41, n_sets).astype(np.int64)
    r = api.sweep(table, n_traj, n_steps, scheme="em", seed=19, bins=16)
    np.testing.assert_array_equal(r.hist.sum(dim=1).cpu().numpy(), n_traj)
    assert np.all(np.isfinite(r.mean_v))
    for k in [0, n_sets - 1, *rng.choice(n_sets, 10, replace=False).tolist()]:
        a = _alone(k, table, n_traj, n_steps, n_steps // 2, "em", 19, 16)
        assert r.mean_v[k] == a.mean_v and r.stderr[k] == a.stderr, k
        assert torch.equal(r.hist[k], a.hist), k
