"""GPU checks of the checkpointed adjoint against the FP64 oracle.

Readings (the pathwise gradient of a long-time average of a chaotic, dissipative system is
ill-conditioned at long horizons; see the design notes):
* G2: at S = 1e3, W = 200 the ensemble gradient matches the FP64 adjoint within 1e-3 relative;
* G3: at the full 1e4-step horizon, per-particle gradients differ from the FP64 adjoint by no more
  than twice the FP64 gradient's own change under FP32-sized path perturbations, and on the
  well-conditioned particles the summed gradient matches within 1e-3;
* G4: bit-exact invariances: the gradient does not depend on the checkpoint interval, and the
  adjoint's loss equals the integrator's mean velocity for the same set.
"""
import numpy as np
import pytest
import torch


pytestmark = pytest.mark.gpu

GRAD_KEYS = ("U0", "a", "D", "d2", "q", "c", "gamma0", "F0")


def _theta(n_sets, jitter=0.0, seed=0):
    """Base parameters, each scaled by 1 + jitter * U(-1, 1); F0 (0 at the base) is shifted by
    0.2 jitter U(-1, 1) instead."""
    from paper_1104_2499_amd.workloads import BASE_PARAMS

    base = np.array([BASE_PARAMS[k] for k in GRAD_KEYS])
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, (n_sets, len(GRAD_KEYS)))
    th = np.tile(base, (n_sets, 1)) * (1 + jitter * u)
    th[:, GRAD_KEYS.index("F0")] += 0.2 * jitter * u[:, GRAD_KEYS.index("F0")]
    return torch.tensor(th, dtype=torch.float64)


def _params(theta_row):
    from paper_1104_2499_amd.workloads import BASE_PARAMS

    p = dict(BASE_PARAMS)
    p.update({k: float(theta_row[j]) for j, k in enumerate(GRAD_KEYS)})
    return p


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_loss_equals_forward_mean_and_gradient_is_checkpoint_invariant(gpu, scheme):
    """Bit-identical gradients for every K. For Heun, K = 1203 (rounded to 1216) leaves the
    segment's noise out of LDS, so the reverse sweep recomputes the predictor's v and e instead of
    reading them from the stage: the two forms must agree bit for bit."""
    from paper_1104_2499_amd import adjoint, api

    theta = _theta(3, jitter=0.2, seed=1)
    grads = []
    for K in (100, 37, 1203, 8):
        cfg = adjoint.AdjointConfig(n=300, steps=1203, window=401, ckpt=K, seed=5, scheme=scheme)
        rows = adjoint.param_rows(theta, cfg)
        ws = adjoint.workspace(3, cfg)
        loss = adjoint.forward(rows, cfg, ws)
        g, gp = adjoint.backward(rows, cfg, ws, torch.ones(3, dtype=torch.float64),
                                 per_particle=True)
        grads.append((g.cpu().numpy(), gp.cpu().numpy()))
        for k in range(3):
            r = api.run(_params(theta[k]), n=300, steps=1203, window=401, scheme=scheme, seed=5,
                        bins=0, set_id=k)
            assert float(loss[k].cpu()) == r.mean_v
    for g, gp in grads[1:]:
        np.testing.assert_array_equal(g, grads[0][0])
        np.testing.assert_array_equal(gp, grads[0][1])
    # the set gradient is the mean of the per-particle gradients
    np.testing.assert_allclose(grads[0][0], grads[0][1].mean(axis=1), rtol=1e-12, atol=1e-15)


def test_gradient_matches_fp64_adjoint_short_horizon(gpu, orc):
    """G2: 1024 particles, S = 1e3, W = 200, K = 100."""
    from paper_1104_2499_amd import adjoint

    theta = _theta(1)
    n, S, W = 1024, 1000, 200
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=100, seed=42)
    t = theta.clone().requires_grad_(True)
    L = adjoint.mean_velocity(t, cfg)
    L.sum().backward()
    g_gpu = t.grad.numpy()[0]
    x0, v0, e0 = orc.init_state(n, 42)
    J, g = orc.adjoint(_params(theta[0]), x0, v0, e0, S, W, seed=42)
    g_ora = g.mean(axis=0)
    print("gpu", g_gpu, "\noracle", g_ora)
    # dL/dF0 nearly cancels over the ensemble (trapped particles: the equilibrium shift at both
    # window ends); FP32 sums resolve it to about 1e-6 of the largest component, hence the atol
    np.testing.assert_allclose(g_gpu, g_ora, rtol=1e-3, atol=1e-6 * np.abs(g_ora).max())
    assert abs(float(L.detach().cpu()[0]) - J.mean()) <= 1e-5


def test_gradient_matches_central_differences(gpu, orc):
    """Central differences (h = 1e-4, common random numbers) of the FP64 oracle, S = 1e3."""
    from paper_1104_2499_amd import adjoint

    theta = _theta(1)
    n, S, W = 512, 1000, 200
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=50, seed=9)
    t = theta.clone().requires_grad_(True)
    adjoint.mean_velocity(t, cfg).sum().backward()
    g_gpu = t.grad.numpy()[0]
    x0, v0, e0 = orc.init_state(n, 9)
    for j, name in enumerate(GRAD_KEYS):
        def L(val):
            p = _params(theta[0])
            p[name] = val
            x, _, _, xs, _ = orc.integrate(p, x0, v0, e0, S, seed=9, win_begin=S - W)
            return ((x - xs) / (W * 1e-3)).mean()
        c = float(theta[0, j])
        fd = (L(c + 1e-4) - L(c - 1e-4)) / 2e-4
        assert abs(g_gpu[j] - fd) <= 1e-3 * abs(fd) + 1e-8, (name, g_gpu[j], fd)


def test_batched_adjoint_sets_match_oracle(gpu, orc):
    """16 parameter sets in one launch, each against the FP64 adjoint of that set."""
    from paper_1104_2499_amd import adjoint

    n_sets, n, S, W = 16, 256, 800, 160
    theta = _theta(n_sets, jitter=0.3, seed=3)
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=64, seed=3)
    gloss = torch.linspace(-1.0, 2.0, n_sets, dtype=torch.float64)
    t = theta.clone().requires_grad_(True)
    L = adjoint.mean_velocity(t, cfg)
    (L.cpu() * gloss).sum().backward()
    for k in range(n_sets):
        x0, v0, e0 = orc.init_state(n, 3, k)
        J, g = orc.adjoint(_params(theta[k]), x0, v0, e0, S, W, seed=3, set_id=k)
        want = float(gloss[k]) * g.mean(axis=0)
        np.testing.assert_allclose(t.grad.numpy()[k], want, rtol=2e-3,
                                   atol=1e-6 * np.abs(want).max())


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_full_horizon_per_particle_gradients(gpu, orc, scheme):
    """G3 at the 65536-particle, 1e4-step, W = 2000, K = 100 configuration (the Euler-Maruyama
    workload, and the same shape through the stochastic Heun map), on 8192 sampled particles:
    (i) per particle and component, the GPU-oracle gradient difference is within twice the
    oracle's own change under FP32-sized path perturbations (2^-24 model), for >= 99% of the
    pairs; (ii) summed over the particles whose FP64 gradient is well-conditioned (every component
    changes by < 1e-4 relative under that perturbation; about 7% of the particles at this
    horizon), the GPU gradient matches within 1e-3 relative."""
    from paper_1104_2499_amd import adjoint, api

    theta = _theta(1)
    n, S, W = 65536, 10_000, 2_000
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=100, seed=42, scheme=scheme)
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(1, cfg)
    loss = adjoint.forward(rows, cfg, ws)
    g, gp = adjoint.backward(rows, cfg, ws, torch.ones(1, dtype=torch.float64), per_particle=True)
    run = api.run(_params(theta[0]), n=n, steps=S, window=W, scheme=scheme, seed=42, bins=0)
    assert float(loss[0].cpu()) == run.mean_v
    ids = np.arange(0, n, 8, dtype=np.uint64)  # 8192 sampled particles
    x0, v0, e0 = orc.init_state(ids.size, 42, ids=ids)
    p = _params(theta[0])
    sid = 0 if scheme == "em" else 1
    _, g_ora = orc.adjoint(p, x0, v0, e0, S, W, seed=42, ids=ids, scheme=sid)
    _, g_eps = orc.adjoint(p, x0, v0, e0, S, W, seed=42, ids=ids, eps=2.0**-24, scheme=sid)
    gpp = gp[0].cpu().numpy()[ids.astype(np.int64)]
    scale = np.abs(g_ora).max(axis=0)
    d_gpu = np.abs(gpp - g_ora)
    d_own = np.abs(g_eps - g_ora)
    within = d_gpu <= 2 * d_own + 1e-6 * scale
    floor = np.maximum(np.abs(g_ora), 1e-6 * scale)
    C = (d_own / floor < 1e-4).all(axis=1)
    print(f"{scheme}: pairs within 2x own sensitivity: {within.mean():.4f}; well-conditioned "
          f"particles "
          f"{C.mean():.3f}; median |gpu-ora|/|ora| {np.median(d_gpu / floor):.2e}, "
          f"median own {np.median(d_own / floor):.2e}")
    assert within.mean() >= 0.99
    assert C.sum() >= 300
    np.testing.assert_allclose(gpp[C].sum(axis=0), g_ora[C].sum(axis=0), rtol=1e-3,
                               atol=1e-6 * np.abs(g_ora[C].sum(axis=0)).max())


def test_adjoint_rejects_bad_arguments(gpu):
    from paper_1104_2499_amd import adjoint, api

    theta = _theta(1)
    theta[0, 2] = 0.0  # D = 0: d(sigma)/dD is singular
    cfg = adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=10)
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        adjoint.forward(adjoint.param_rows(theta, cfg), cfg, adjoint.workspace(1, cfg))
    cfg2 = adjoint.AdjointConfig(n=64, steps=100, window=101, ckpt=10)
    with pytest.raises(ValueError):
        adjoint.workspace(1, adjoint.AdjointConfig(n=0, steps=100, window=10, ckpt=10))
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        adjoint.forward(adjoint.param_rows(_theta(1), cfg2), cfg2, adjoint.workspace(1, cfg))


def test_adjoint_device_side_parameter_checks(gpu):
    """The parameter table is checked on the device in each phase: a set with D <= 0, with
    1 / (2D) past the FP32 range, or with an FP32-overflowing U0 sets the device status to
    ABP_E_ARG and turns that call's outputs into NaN; good rows on the same workspace then run."""
    from paper_1104_2499_amd import _lib, adjoint

    cfg = adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=16)
    ws = adjoint.workspace(2, cfg)
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    gl = torch.ones(2, dtype=torch.float64, device="cuda")
    for j, val in ((2, 0.0), (2, 1e-40), (0, 1e38)):
        theta = _theta(2)
        theta[1, j] = val
        rows = adjoint.param_rows(theta, cfg)
        loss = adjoint.forward(rows, cfg, ws, status=status, check_status=False)
        assert int(status.item()) == _lib.ABP_E_ARG
        assert torch.isnan(loss).all()
        g = adjoint.backward(rows, cfg, ws, gl, status=status, check_status=False)
        assert int(status.item()) == _lib.ABP_E_ARG
        assert torch.isnan(g).all()
    rows = adjoint.param_rows(_theta(2), cfg)
    loss = adjoint.forward(rows, cfg, ws, status=status, check_status=False)
    g = adjoint.backward(rows, cfg, ws, gl, status=status, check_status=False)
    assert int(status.item()) == _lib.ABP_OK
    assert torch.isfinite(loss).all() and torch.isfinite(g).all()


def test_decayed_estimator_matches_oracle(gpu, orc):
    """The look-back-damped estimator (lookback = 500 steps) against the FP64 oracle's, at the
    short horizon and with several sets."""
    from paper_1104_2499_amd import adjoint

    n_sets, n, S, W = 4, 512, 1000, 400
    theta = _theta(n_sets, jitter=0.2, seed=8)
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=100, seed=8, lookback=500)
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(n_sets, cfg)
    adjoint.forward(rows, cfg, ws)
    g = adjoint.backward(rows, cfg, ws, torch.ones(n_sets, dtype=torch.float64)).cpu().numpy()
    for k in range(n_sets):
        x0, v0, e0 = orc.init_state(n, 8, k)
        _, go = orc.adjoint(_params(theta[k]), x0, v0, e0, S, W, seed=8, set_id=k, lookback=500)
        want = go.mean(axis=0)
        np.testing.assert_allclose(g[k], want, rtol=1e-3, atol=1e-6 * np.abs(want).max())


def test_heun_loss_and_checkpoint_invariance(gpu):
    """G4 for the stochastic Heun adjoint: loss == the Heun integrator's mean velocity and the
    gradient does not depend on K (K rounded to 16), with 16-step (default) and 8-step staging;
    the two stagings group the FP32 sums differently and agree to FP32 rounding."""
    from paper_1104_2499_amd import adjoint, api

    theta = _theta(2, jitter=0.2, seed=6)
    by_stage = {}
    for stage in (0, 8):
        grads = []
        for K in (100, 37, 1203):
            cfg = adjoint.AdjointConfig(n=200, steps=1203, window=401, ckpt=K, seed=6,
                                        scheme="heun", stage=stage)
            rows = adjoint.param_rows(theta, cfg)
            ws = adjoint.workspace(2, cfg)
            loss = adjoint.forward(rows, cfg, ws)
            g, gp = adjoint.backward(rows, cfg, ws, torch.ones(2, dtype=torch.float64),
                                     per_particle=True)
            grads.append((g.cpu().numpy(), gp.cpu().numpy()))
            for k in range(2):
                r = api.run(_params(theta[k]), n=200, steps=1203, window=401, scheme="heun",
                            seed=6, bins=0, set_id=k)
                assert float(loss[k].cpu()) == r.mean_v
        for g, gp in grads[1:]:
            np.testing.assert_array_equal(g, grads[0][0])
            np.testing.assert_array_equal(gp, grads[0][1])
        by_stage[stage] = grads[0][0]
    np.testing.assert_allclose(by_stage[8], by_stage[0], rtol=1e-5,
                               atol=1e-7 * np.abs(by_stage[0]).max())


def test_heun_gradient_matches_fp64_adjoint(gpu, orc):
    """G2 for Heun: 3 sets x 1024 particles, S = 1e3, W = 200, against the FP64 Heun adjoint."""
    from paper_1104_2499_amd import adjoint

    n_sets, n, S, W = 3, 1024, 1000, 200
    theta = _theta(n_sets, jitter=0.2, seed=12)
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=100, seed=12, scheme="heun")
    t = theta.clone().requires_grad_(True)
    L = adjoint.mean_velocity(t, cfg)
    L.sum().backward()
    for k in range(n_sets):
        x0, v0, e0 = orc.init_state(n, 12, k)
        J, g = orc.adjoint(_params(theta[k]), x0, v0, e0, S, W, seed=12, set_id=k,
                           scheme=orc.HEUN)
        want = g.mean(axis=0)
        print("gpu", t.grad.numpy()[k], "\noracle", want)
        np.testing.assert_allclose(t.grad.numpy()[k], want, rtol=1e-3,
                                   atol=1e-6 * np.abs(want).max())
        assert abs(float(L.detach().cpu()[k]) - J.mean()) <= 1e-5


def test_heun_rejects_lookback(gpu):
    from paper_1104_2499_amd import adjoint, api

    cfg = adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=10, scheme="heun", lookback=50)
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        adjoint.forward(adjoint.param_rows(_theta(1), cfg), cfg, adjoint.workspace(1, cfg))


@pytest.mark.parametrize("scheme", ["em", "heun"])
@pytest.mark.parametrize("n,S,W,K", [(1, 1, 1, 1), (1, 5, 5, 3), (3, 17, 2, 1), (65, 40, 40, 40)])
def test_degenerate_sizes(gpu, orc, scheme, n, S, W, K):
    """Tiny ensembles and horizons (one particle, one step, windows covering the whole run, a
    partial tile) against the FP64 adjoint: at these horizons FP32 and FP64 agree closely."""
    from paper_1104_2499_amd import adjoint, api

    theta = _theta(1, jitter=0.1, seed=2)
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=K, seed=2, scheme=scheme)
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(1, cfg)
    loss = adjoint.forward(rows, cfg, ws)
    g, gp = adjoint.backward(rows, cfg, ws, torch.ones(1, dtype=torch.float64), per_particle=True)
    r = api.run(_params(theta[0]), n=n, steps=S, window=W, scheme=scheme, seed=2, bins=0)
    assert float(loss[0].cpu()) == r.mean_v
    x0, v0, e0 = orc.init_state(n, 2)
    J, go = orc.adjoint(_params(theta[0]), x0, v0, e0, S, W, seed=2,
                        scheme=orc.EM if scheme == "em" else orc.HEUN)
    want = go.mean(axis=0)
    np.testing.assert_allclose(g.cpu().numpy()[0], want, rtol=1e-4,
                               atol=1e-5 * np.abs(want).max())
    np.testing.assert_allclose(gp.cpu().numpy()[0], go, rtol=1e-3,
                               atol=1e-5 * np.abs(go).max())


def test_eight_step_staging(gpu, orc):
    """stage = 8 (the kernel that fits two wavefronts per SIMD; this small ensemble runs one, with
    the noise in LDS at K = 48 and 100 and regenerated at K = 1000): the same recursion with the
    FP32 gradient sums grouped in 8-step windows. Bit-identical loss, K-independent gradient,
    within FP32 rounding of the 16-step staging and within 1e-3 of the FP64 adjoint; invalid
    stagings are rejected."""
    from paper_1104_2499_amd import adjoint, api

    n_sets, n, S, W = 3, 700, 1000, 200
    theta = _theta(n_sets, jitter=0.2, seed=14)
    out = {}
    for stage, K in ((0, 100), (8, 100), (8, 48), (8, 1000), (8, 16)):
        cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=K, seed=14, stage=stage)
        rows = adjoint.param_rows(theta, cfg)
        ws = adjoint.workspace(n_sets, cfg)
        loss = adjoint.forward(rows, cfg, ws).cpu().numpy()
        g = adjoint.backward(rows, cfg, ws, torch.ones(n_sets, dtype=torch.float64))
        out[(stage, K)] = (loss, g.cpu().numpy())
    for key in ((8, 48), (8, 1000), (8, 16)):
        np.testing.assert_array_equal(out[key][1], out[(8, 100)][1])
    np.testing.assert_array_equal(out[(8, 100)][0], out[(0, 100)][0])
    np.testing.assert_allclose(out[(8, 100)][1], out[(0, 100)][1], rtol=1e-5,
                               atol=1e-7 * np.abs(out[(0, 100)][1]).max())
    for k in range(n_sets):
        x0, v0, e0 = orc.init_state(n, 14, k)
        _, go = orc.adjoint(_params(theta[k]), x0, v0, e0, S, W, seed=14, set_id=k)
        want = go.mean(axis=0)
        np.testing.assert_allclose(out[(8, 100)][1][k], want, rtol=1e-3,
                                   atol=1e-6 * np.abs(want).max())
    for stage, scheme in ((12, "em"), (12, "heun"), (-8, "em")):
        cfg = adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=16, stage=stage,
                                    scheme=scheme)
        with pytest.raises(api.AbpError, match="ABP_E_ARG"):
            adjoint.forward(adjoint.param_rows(_theta(1), cfg), cfg, adjoint.workspace(1, cfg))


@pytest.mark.parametrize("stage,ks", [(16, (48, 80, 1203)), (8, (48, 100, 1203))])
def test_two_wavefront_backward_matches_one_wavefront(gpu, stage, ks):
    """Euler-Maruyama ensembles of at least two wavefronts per SIMD run two backward blocks per
    CU: the 16-step kernel through its build for two wavefronts per SIMD, the 8-step kernel as it
    is, each with LDS sized for two blocks. 160 sets x 1024 particles (2560 wavefronts) select
    that; set 0 alone (16 wavefronts) runs one wavefront per SIMD with LDS sized for one block, on
    the same particles and noise, and its per-particle gradients must be the same bits. 16-step:
    the segment's sub-checkpoints in LDS (K = 48), the noise only (K = 80), neither (K = 1203).
    8-step: the noise in LDS at both sizings (K = 48), only for the lone set (K = 100), neither
    (K = 1203)."""
    from paper_1104_2499_amd import adjoint

    theta = _theta(160, jitter=0.2, seed=4)
    n, S, W = 1024, 2000, 500
    ref = None
    for K in ks:
        print(f"stage {stage}, K = {K}", flush=True)
        cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=K, seed=9, stage=stage)
        ws = adjoint.workspace(160, cfg)
        rows = adjoint.param_rows(theta, cfg)
        adjoint.forward(rows, cfg, ws)
        _, gp = adjoint.backward(rows, cfg, ws, torch.ones(160, dtype=torch.float64),
                                 per_particle=True)
        gp0 = gp[0].cpu().numpy()
        del ws, gp
        if ref is None:
            ws1 = adjoint.workspace(1, cfg)
            rows1 = adjoint.param_rows(theta[:1], cfg)
            adjoint.forward(rows1, cfg, ws1)
            _, ref = adjoint.backward(rows1, cfg, ws1, torch.ones(1, dtype=torch.float64),
                                      per_particle=True)
            ref = ref[0].cpu().numpy()
        assert np.isfinite(gp0).all()
        np.testing.assert_array_equal(gp0, ref, err_msg=f"K = {K}")


def test_batched_workload_full_size_sampled(gpu, orc):
    """The batched-adjoint workload at full size, in the launch configuration the benchmark times:
    1024 sets x 1024 particles x 5e4 EM steps, W = 1e4, K = 48, 16-step staging (a 31 GB
    workspace; the backward kernel built for two wavefronts per SIMD). Checked: the losses of
    sampled sets equal the plain forward run of the same set bit for bit; every gradient is finite;
    each set's gradient is the mean of its per-particle gradients; and on the lowest-noise set and
    on set 0 (256 sampled particles each), per-particle gradients of the particles whose FP64
    gradient moves by < 1e-3 relative under FP32-sized path perturbations (2^-24 model) agree with the FP64
    adjoint within twice that movement plus 1e-3 relative (the gradient tolerance, applied per
    particle: over 5e4 reverse steps the FP32 recursion's own rounding reaches ~1e-4 to 1e-3
    relative, more than the FP64 gradient moves for some components). At this horizon most
    trajectories decorrelate under such perturbations, so the other particles are not comparable
    one by one."""
    from paper_1104_2499_amd import adjoint, api
    from paper_1104_2499_amd.optimize import initial_theta
    from paper_1104_2499_amd.workloads import WORKLOADS

    wl = WORKLOADS["adjoint-batched-1k"]
    n_sets, n, S, W, seed = wl["n_sets"], wl["n"], wl["steps"], wl["window"], wl["seed"]
    theta = torch.tensor(initial_theta(n_sets, seed))
    cfg = adjoint.AdjointConfig(n=n, steps=S, window=W, ckpt=wl["ckpt"], seed=seed,
                                stage=wl["stage"])
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(n_sets, cfg)
    loss = adjoint.forward(rows, cfg, ws).cpu().numpy()
    g, gp = adjoint.backward(rows, cfg, ws, torch.ones(n_sets, dtype=torch.float64),
                             per_particle=True)
    del ws
    torch.cuda.empty_cache()
    g, gp = g.cpu().numpy(), gp.cpu().numpy()
    assert np.isfinite(loss).all() and np.isfinite(g).all() and np.isfinite(gp).all()
    np.testing.assert_allclose(g, gp.mean(axis=1), rtol=1e-9,
                               atol=1e-12 * np.abs(gp).sum(axis=1).max())
    low_d = int(np.argmin(theta[:, GRAD_KEYS.index("D")].numpy()))
    for k in (0, low_d, n_sets // 2, n_sets - 1):
        run = api.run(_params(theta[k]), n=n, steps=S, window=W, scheme="em", seed=seed, bins=0,
                      set_id=k)
        assert loss[k] == run.mean_v, k
    ids = np.arange(0, n, 4, dtype=np.uint64)
    n_cond = 0
    for k in (low_d, 0):
        p = _params(theta[k])
        x0, v0, e0 = orc.init_state(ids.size, seed, k, ids=ids)
        _, g_ora = orc.adjoint(p, x0, v0, e0, S, W, seed=seed, set_id=k, ids=ids)
        _, g_eps = orc.adjoint(p, x0, v0, e0, S, W, seed=seed, set_id=k, ids=ids, eps=2.0**-24)
        d_own = np.abs(g_eps - g_ora)
        C = (d_own <= 1e-3 * np.abs(g_ora)).all(axis=1)
        d_gpu = np.abs(gp[k][ids.astype(np.int64)] - g_ora)
        within = (d_gpu <= 2 * d_own + 1e-3 * np.abs(g_ora))[C]
        rel = (d_gpu / np.abs(g_ora))[C]
        print(f"set {k}: {C.sum()} well-conditioned of {ids.size}; GPU relative error median "
              f"{np.median(rel):.1e}, max {rel.max():.1e}; within bound {within.mean():.4f}")
        assert within.mean() >= 0.99, k
        n_cond += int(C.sum())
    assert n_cond >= 40
