"""GPU parity of the forward integrator and its reductions against the FP64 oracle.

Readings used for the tolerances (the dynamics amplify any rounding; see the design notes):
* per trajectory, 1e3 steps: >= 99.9% within 1e-4 and all within 1e-3 (mixed error, max over
  x, v, e of |gpu - oracle| / max(1, |oracle|));
* per trajectory, 1e4 steps: median within 1e-4, and the p50 / p90 / p99 of the GPU-oracle error
  at most twice the oracle's own divergence under FP32-sized perturbations (plus a floor);
* ensemble mean velocity: 1e-5 absolute;
* histograms: bit-exact on identical states; otherwise they differ only by particles whose
  trajectories differ.
"""
import numpy as np
import pytest
import torch

from conftest import mixed_err

pytestmark = pytest.mark.gpu

BASE = dict(U0=1.0, a=0.25, phi=0.0, gamma0=1.0, F0=0.0, d2=1.0, q=1.0, c=0.1, D=0.1)


def _np(t):
    return t.detach().cpu().numpy()


def _u32_as_i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32))


def test_philox_bit_exact(gpu, orc):
    from paper_1104_2499_amd import api

    rng = np.random.default_rng(7)
    m = 1 << 20
    ctr = rng.integers(0, 2**32, size=(m, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(m, 2), dtype=np.uint64).astype(np.uint32)
    key[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0, 0xFFFFFFFF], [0xFFFFFFFF, 0]]
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0xFFFFFFFF, 0, 0, 0], [0, 0, 0, 0xFFFFFFFF]]
    out = api.philox(_u32_as_i32(ctr).cuda(), _u32_as_i32(key).cuda())
    got = _np(out).view(np.uint32)
    np.testing.assert_array_equal(got, orc.philox(ctr, key))


def test_noise_matches_oracle_normals(gpu, orc):
    """The kernel's noise, read directly: for a force-free particle (U0 = gamma0 = d2 = F0 = q = c
    = 0) with v0 = 0 and sigma = sqrt(2 D dt) = 1 (D = 1, dt = 1/2), one Euler-Maruyama step from
    absolute step n leaves v + lv = sigma xi_n exactly (the increment lands in an empty low part,
    or in an empty high part after a block end). 2^16 particles at steps in every position of a
    Philox block and at the top of the block counter, against the FP64 oracle's normals of the
    same Philox words: the difference is the FP32 Box-Muller's rounding (v_log, v_sqrt and
    v_cos / v_sin in revolutions). Measured on MI355X: at most 2.8e-7 of max(1, |z|), about
    2.4 ulp of 1.0; the bound is 1e-6 (8 ulp)."""
    from paper_1104_2499_amd import api

    n, seed, set_id = 1 << 16, 77, 5
    free = dict(U0=0.0, a=0.0, phi=0.0, gamma0=0.0, F0=0.0, d2=0.0, q=0.0, c=0.0, D=1.0)
    worst = 0.0
    for n0 in (0, 1, 2, 3, 4 * 12345 + 2, 4 * (2**32 - 1) + 3):
        s = api.init_state(n, seed, set_id)
        api.integrate(s, 1, free, dt=0.5, scheme="em", seed=seed, set_id=set_id, step0=n0)
        z = _np(s.v.double() + s.lo[1].double())
        want = np.array([orc.normals(seed, i, set_id, n0, 1)[0] for i in range(n)])
        err = np.abs(z - want)
        rel = err / np.maximum(1.0, np.abs(want))
        print(f"step {n0}: max |dz| {err.max():.2e}, max |dz|/max(1,|z|) {rel.max():.2e}, "
              f"median {np.median(err):.1e}, max |z| {np.abs(want).max():.2f}")
        worst = max(worst, rel.max())
        assert np.isfinite(z).all()
    assert worst <= 1e-6


def test_noise_statistics_1e8_samples(gpu):
    """The kernel's normals as a sample of N(0, 1): 2^24 particles x 6 step indices = 1.0e8
    values read as in test_noise_matches_oracle_normals. Mean and variance within 5 standard
    errors, lag-one correlation between consecutive steps of a particle within 5 standard
    errors of 0, and the Kolmogorov-Smirnov distance to the standard normal CDF below 2.0e-4
    (the 0.1% critical value 1.95 / sqrt(1e8); the 2^-23 grid of the uniforms caps |z| at 5.65,
    a tail mass of 1.6e-8)."""
    from paper_1104_2499_amd import api

    n, seed = 1 << 24, 2024
    free = dict(U0=0.0, a=0.0, phi=0.0, gamma0=0.0, F0=0.0, d2=0.0, q=0.0, c=0.0, D=1.0)
    cols = []
    s = api.State.empty(n)
    for n0 in (0, 1, 2, 3, 4, 5):
        api.reset_state(s, seed)
        api.integrate(s, 1, free, dt=0.5, scheme="em", seed=seed, step0=n0)
        cols.append(s.v.double() + s.lo[1].double())
    z = torch.stack(cols)  # [6, n]
    del s, cols
    m = z.numel()
    mean, var = float(z.mean()), float(z.var())
    assert abs(mean) <= 5 / m ** 0.5, mean
    assert abs(var - 1.0) <= 5 * (2.0 / m) ** 0.5, var
    lag = float((z[1:] * z[:-1]).mean())  # consecutive steps of each particle
    assert abs(lag) <= 5 / (m * 5 / 6) ** 0.5, lag
    zs, _ = torch.sort(z.flatten())
    del z
    cdf = torch.special.ndtr(zs)
    i = torch.arange(1, m + 1, dtype=torch.float64, device=zs.device)
    d = float(torch.maximum((i / m - cdf).max(), (cdf - (i - 1) / m).max()))
    print(f"1e8 normals: mean {mean:.2e}, var-1 {var - 1:.2e}, lag-1 {lag:.2e}, KS D {d:.2e}, "
          f"max |z| {float(zs.abs().max()):.3f}")
    assert d < 2.0e-4, d


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_closed_forms_at_full_size(gpu, scheme):
    """With U0 = d2 = 0 the model decouples into closed forms that hold for any ensemble size;
    checked on 2^20 particles after 5000 steps (F0 = 0.5, gamma0 = 1, D = 0.1, q = 1, c = 0.1,
    dt = 1e-3, v0 = e0 = 0). Depot: e_n = (q/c)(1 - r^n) with r = 1 - c dt (Euler-Maruyama) or
    1 - c dt + (c dt)^2 / 2 (Heun), the same for every particle, to 1e-6 relative. Velocity: the
    discrete Ornstein-Uhlenbeck recursion v' = rho v + b + s xi with, for Euler-Maruyama,
    rho = 1 - g dt, b = F0 dt, s = sigma, and for Heun rho = 1 - g dt + (g dt)^2 / 2,
    b = F0 dt (1 - g dt / 2), s = sigma (1 - g dt / 2): mean b (1 - rho^n) / (1 - rho) and
    variance s^2 (1 - rho^(2n)) / (1 - rho^2), within 5 standard errors of the sample."""
    from paper_1104_2499_amd import api

    n, S, dt = 1 << 20, 5000, 1e-3
    g, F0, D, q, c = 1.0, 0.5, 0.1, 1.0, 0.1
    p = dict(U0=0.0, a=0.0, phi=0.0, gamma0=g, F0=F0, d2=0.0, q=q, c=c, D=D)
    res = api.run(p, n=n, steps=S, window=S // 2, scheme=scheme, seed=31, bins=0)
    v = res.state.v64().double()
    e = res.state.e64().double()
    sig = (2 * D * dt) ** 0.5
    if scheme == "em":
        r, rho, b, s_ = 1 - c * dt, 1 - g * dt, F0 * dt, sig
    else:
        r = 1 - c * dt + (c * dt) ** 2 / 2
        rho, b, s_ = 1 - g * dt + (g * dt) ** 2 / 2, F0 * dt * (1 - g * dt / 2), sig * (1 - g * dt / 2)
    e_want = q / c * (1 - r ** S)
    assert float((e - e_want).abs().max()) <= 1e-6 * e_want
    m_want = b * (1 - rho ** S) / (1 - rho)
    var_want = s_ ** 2 * (1 - rho ** (2 * S)) / (1 - rho ** 2)
    m, var = float(v.mean()), float(v.var())
    print(f"{scheme}: e err {float((e - e_want).abs().max()) / e_want:.1e}; <v> {m:.6f} vs "
          f"{m_want:.6f}; var {var:.6f} vs {var_want:.6f}")
    assert abs(m - m_want) <= 5 * (var_want / n) ** 0.5
    assert abs(var - var_want) <= 5 * var_want * (2.0 / n) ** 0.5


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_passive_ratchet_boltzmann_at_full_size(gpu, scheme):
    """A passive particle (d2 = F0 = 0) in the ratchet is in equilibrium at temperature D / gamma0:
    the density of x mod 1 is proportional to exp(-gamma0 U(x) / D) and the current vanishes.
    2^20 particles, U0 = 0.2 (barrier ~0.44), D = 0.5, dt = 1e-3, both schemes: 5000 steps
    of burn-in, then the time-accumulated histogram (64 bins) every 100 steps for 15000 steps.
    Total variation from the Boltzmann bin masses < 0.003 (measured 0.0011 with Euler-Maruyama;
    shifting the law by one bin moves it by 0.0136, so the check would see such an error) and
    the mean velocity over the sampling phase within 4 standard errors of 0."""
    from paper_1104_2499_amd import api

    n, burn, S, stride, bins, dt = 1 << 20, 5000, 20000, 100, 64, 1e-3
    U0, a, D, g = 0.2, 0.25, 0.5, 1.0
    p = dict(U0=U0, a=a, phi=0.0, gamma0=g, F0=0.0, d2=0.0, q=1.0, c=0.1, D=D)
    s = api.init_state(n, 13)
    api.integrate(s, burn, p, dt=dt, scheme=scheme, seed=13)
    x_a = s.x64().clone()
    acc = torch.zeros(bins, dtype=torch.int64, device=x_a.device)
    api.integrate(s, S - burn, p, dt=dt, scheme=scheme, seed=13, step0=burn, hist_stride=stride,
                  hist_acc=acc)
    h = acc.cpu().numpy().astype(np.float64)
    assert h.sum() == n * (S - burn) // stride
    h /= h.sum()
    fine = 256
    xs = (np.arange(bins * fine) + 0.5) / (bins * fine)
    U = U0 * (np.sin(2 * np.pi * xs) + a * np.sin(4 * np.pi * xs))
    w = np.exp(-g * U / D).reshape(bins, fine).sum(axis=1)
    w /= w.sum()
    tv = 0.5 * np.abs(h - w).sum()
    shift = 0.5 * np.abs(np.roll(w, 1) - w).sum()
    disp = (s.x64() - x_a).cpu().numpy()
    T = (S - burn) * dt
    vbar, se = disp.mean() / T, disp.std() / np.sqrt(n) / T
    print(f"{scheme}: Boltzmann TV {tv:.2e} (one-bin shift {shift:.2e}); <v> {vbar:.2e} +- "
          f"{se:.1e}")
    assert tv < 0.003 and shift > 4 * 0.003
    assert abs(vbar) <= 4 * se


@pytest.mark.parametrize("n,id0,seed,set_id", [(5000, 0, 42, 0), (77, 123456, 2**40 + 5, 9),
                                                (1, 0xFFFFFFFF, 0, 0)])
def test_init_state_bit_exact(gpu, orc, n, id0, seed, set_id):
    from paper_1104_2499_amd import api

    s = api.init_state(n, seed, set_id, id0=id0)
    x, v, e = orc.init_state(n, seed, set_id, ids=np.arange(id0, id0 + n, dtype=np.uint64))
    np.testing.assert_array_equal(_np(s.cell), 0)
    np.testing.assert_array_equal(_np(s.xf).astype(np.float64), x)
    assert not _np(s.v).any() and not _np(s.e).any()


def _run_pair(orc, params, n, steps, scheme, seed=42, window=None, dt=1e-3, bins=256, tune=None,
              set_id=0):
    from paper_1104_2499_amd import api

    window = steps // 2 if window is None else window
    res = api.run(params, n=n, steps=steps, window=window, dt=dt, scheme=scheme, seed=seed,
                  bins=bins, tune=tune, set_id=set_id)
    x0, v0, e0 = orc.init_state(n, seed, set_id)
    sid = 0 if scheme == "em" else 1
    x, v, e, xs, _ = orc.integrate(params, x0, v0, e0, steps, dt=dt, scheme=sid, seed=seed,
                                   set_id=set_id, win_begin=steps - window)
    mean, se, hist = orc.reduce(xs, x, window * dt, bins)
    return res, (x, v, e, xs), (mean, se, hist)


def _gpu_xve(res):
    return (_np(res.state.x64()), _np(res.state.v64()), _np(res.state.e64()))


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_trajectory_parity_1e3_steps(gpu, orc, scheme):
    res, (x, v, e, xs), (mean, se, hist) = _run_pair(orc, BASE, 1024, 1000, scheme)
    err = mixed_err(_gpu_xve(res), (x, v, e))
    print(f"{scheme} 1e3: p50={np.median(err):.2e} p99.9={np.quantile(err, 0.999):.2e} "
          f"max={err.max():.2e}")
    assert (err <= 1e-4).mean() >= 0.999
    assert err.max() <= 1e-3
    assert abs(res.mean_v - mean) <= 1e-5


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_ensemble_parity_1e4_steps(gpu, orc, scheme):
    """The 1024-particle, 1e4-step, dt = 1e-3 workload (EM is the parity configuration)."""
    n, steps = 1024, 10_000
    res, (x, v, e, xs), (mean, se, hist) = _run_pair(orc, BASE, n, steps, scheme)
    err = mixed_err(_gpu_xve(res), (x, v, e))
    x0, v0, e0 = orc.init_state(n, 42)
    sid = 0 if scheme == "em" else 1
    xp, vp, ep, _, _ = orc.integrate(BASE, x0, v0, e0, steps, scheme=sid, seed=42,
                                     eps=2.0**-24)
    own = mixed_err((xp, vp, ep), (x, v, e))
    q = [0.5, 0.9, 0.99]
    gq, oq = np.quantile(err, q), np.quantile(own, q)
    print(f"{scheme} 1e4: gpu-vs-oracle p50/p90/p99 = {gq}, oracle self-divergence = {oq}, "
          f"frac<=1e-4: {(err <= 1e-4).mean():.3f}; <v> gpu={res.mean_v:.6e} ora={mean:.6e}")
    assert np.median(err) <= 1e-4
    assert np.all(gq <= 2 * oq + 1e-6)
    assert abs(res.mean_v - mean) <= 1e-5
    assert res.stderr == pytest.approx(se, rel=0.05)
    # histogram: identical bins wherever the trajectories agree (and are off bin edges)
    hg = _np(res.hist).astype(np.int64)
    assert hg.sum() == n
    xg = _np(res.state.x64())
    bg = np.minimum(np.floor((xg - np.floor(xg)) * 256), 255).astype(np.int64)
    bo = np.minimum(np.floor((x - np.floor(x)) * 256), 255).astype(np.int64)
    np.testing.assert_array_equal(np.bincount(bg, minlength=256), hg)
    frac = x - np.floor(x)
    edge = np.minimum(np.abs(frac * 256 - np.round(frac * 256)), 1.0) / 256
    agree = (np.abs(xg - x) < 1e-6) & (edge > 1e-6)
    assert np.array_equal(bg[agree], bo[agree])
    # where trajectories do not agree, the bins move no more than the oracle's own under 2^-24
    # rounding perturbations: the count of particles in a different bin, and the L1 distance of
    # the histograms, are within twice the oracle's self-divergence (plus a few particles)
    bp = np.minimum(np.floor((xp - np.floor(xp)) * 256), 255).astype(np.int64)
    hp = np.bincount(bp, minlength=256)
    ho = hist.astype(np.int64)
    moved, moved_own = int((bg != bo).sum()), int((bp != bo).sum())
    l1, l1_own = int(np.abs(hg - ho).sum()), int(np.abs(hp - ho).sum())
    print(f"{scheme} 1e4 histogram: particles in another bin {moved} (oracle self {moved_own}), "
          f"L1 {l1} (oracle self {l1_own})")
    assert moved <= 2 * moved_own + 4
    assert l1 <= 2 * l1_own + 8


@pytest.mark.parametrize("scheme,order", [("em", 1), ("heun", 2)])
def test_convergence_order_in_the_deterministic_limit(gpu, orc, scheme, order):
    """D = 0: the kernel's error at t = 1 against an FP64 RK4 solution (step dt / 100) falls by
    2^order when dt halves (dt = 1e-2, 5e-3, 2.5e-3): first order for Euler-Maruyama, second
    for Heun. 256 particles of the base physics from the workload initial condition."""
    from paper_1104_2499_amd import api

    n, T = 256, 1.0
    p = dict(BASE, D=0.0)
    x0, v0, e0 = orc.init_state(n, 3)
    errs = []
    for dt in (1e-2, 5e-3, 2.5e-3):
        S = int(round(T / dt))
        xr, vr, er = orc.rk4(p, x0, v0, e0, 100 * S, dt / 100)
        s = api.init_state(n, 3)
        api.integrate(s, S, p, dt=dt, scheme=scheme, seed=3)
        err = mixed_err((_np(s.x64()), _np(s.v64()), _np(s.e64())), (xr, vr, er))
        errs.append(float(np.median(err)))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    print(f"{scheme}: median errors {errs}, ratios {ratios}")
    for r in ratios:
        assert 0.75 * 2 ** order <= r <= 1.3 * 2 ** order, ratios


def test_deterministic_limit_matches_oracle(gpu, orc):
    p = dict(BASE, D=0.0)
    res, (x, v, e, xs), _ = _run_pair(orc, p, 256, 2000, "heun")
    err = mixed_err(_gpu_xve(res), (x, v, e))
    assert err.max() <= 1e-4


@pytest.mark.parametrize("params", [dict(U0=0.0, d2=0.0, F0=0.5, D=0.3),
                                    dict(U0=0.3, a=0.4, phi=0.1903, F0=-0.2, d2=1.7, c=0.3,
                                         q=0.8, gamma0=1.3, D=0.02),
                                    # no energy input: the depot stays empty (passive limit)
                                    dict(q=0.0, c=0.0, a=0.0, d2=2.0, D=0.2),
                                    # no friction: only the depot coupling limits the speed
                                    dict(gamma0=0.0, d2=1.0, q=2.0, c=0.5, D=0.05)])
def test_other_parameters(gpu, orc, params):
    res, (x, v, e, xs), (mean, se, hist) = _run_pair(orc, params, 2048, 1000, "em", seed=5)
    err = mixed_err(_gpu_xve(res), (x, v, e))
    assert (err <= 1e-4).mean() >= 0.999 and err.max() <= 1e-3
    assert abs(res.mean_v - mean) <= 1e-5


@pytest.mark.parametrize("phi", [0.1903 + 1000.0, -0.1903 - 517.0, 0.1903 - 1.0])
def test_large_and_negative_phase(gpu, orc, phi):
    """The potential is periodic in its phase: a phase far outside [0, 1), or negative, gives the
    trajectories of its reduction to [0, 1) (the FP64 oracle evaluates the phase as given)."""
    params = dict(BASE, phi=phi, U0=0.7, a=0.4)
    for scheme in ("em", "heun"):
        res, (x, v, e, xs), (mean, se, hist) = _run_pair(orc, params, 2048, 1000, scheme, seed=13)
        err = mixed_err(_gpu_xve(res), (x, v, e))
        assert (err <= 1e-4).mean() >= 0.999 and err.max() <= 1e-3, (scheme, err.max())
        assert abs(res.mean_v - mean) <= 1e-5
    # the library reduces the phase before it reaches FP32: the same bits as the reduced phase
    from paper_1104_2499_amd import api

    red = dict(params, phi=phi - np.floor(phi))
    a = api.run(params, n=2048, steps=1000, scheme="heun", seed=13, bins=0)
    b = api.run(red, n=2048, steps=1000, scheme="heun", seed=13, bins=0)
    assert torch.equal(a.state.xf, b.state.xf) and torch.equal(a.state.lo, b.state.lo)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_chunked_equals_unchunked_bitwise(gpu, scheme):
    from paper_1104_2499_amd import api

    n, bins = 3001, 64
    one = api.run(BASE, n=n, steps=1003, window=502, scheme=scheme, seed=9, bins=bins)
    s = api.init_state(n, 9)
    snap = api.State.empty(n)
    ws = api.reduce_workspace(n, bins)
    for step0, k in ((0, 333), (333, 170), (503, 497), (1000, 3)):
        last = step0 + k == 1003
        api.integrate(s, k, BASE, scheme=scheme, seed=9, step0=step0, win_begin=501, snap=snap,
                      ws=ws if last else None, n_bins=bins)
    out, hist = api.reduce(ws, n, bins, 502e-3)
    for a_, b_ in zip(one.state.tensors() + one.snap.tensors(), s.tensors() + snap.tensors()):
        assert torch.equal(a_, b_)
    assert float(out[0].cpu()) == one.mean_v and float(out[1].cpu()) == one.stderr
    assert torch.equal(hist, one.hist)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_every_tuning_gives_identical_results(gpu, scheme):
    """Every launch shape -- block size, particles per lane, and the loop form (one or two noise
    blocks per trip, or the next block's noise ahead of the steps) -- gives the same bits."""
    from paper_1104_2499_amd import api

    ref = None
    for block in (64, 128, 256):
        for ppl in (1, 2):
            for unroll, lookahead in ((1, 1), (1, 2), (2, 1), (1, 0)):
                r = api.run(BASE, n=5000, steps=403, window=201, scheme=scheme, seed=3, bins=128,
                            tune=dict(block=block, ppl=ppl, unroll=unroll, lookahead=lookahead))
                got = tuple(_np(t) for t in r.state.tensors()) + (r.mean_v, r.stderr,
                                                                   _np(r.hist))
                if ref is None:
                    ref = got
                    continue
                for a_, b_ in zip(ref, got):
                    np.testing.assert_array_equal(a_, b_)


def test_reduce_state_histogram_bit_exact(gpu, orc):
    from paper_1104_2499_amd import api

    rng = np.random.default_rng(4)
    n = 100_003
    cell = rng.integers(-1000, 1000, n).astype(np.int32)
    xf = rng.random(n).astype(np.float32)
    edges = (np.arange(256) / 256).astype(np.float32)
    xf[:256] = edges                                        # exactly on bin edges
    xf[256:512] = np.nextafter(edges, np.float32(-1))       # just below them
    xf[512:520] = [0.0, -0.0, 1.0, -1e-30, 1.0 - 2**-24, -0.5, 1.5, -2**-26]
    lx = (rng.standard_normal(n) * 1e-8).astype(np.float32)
    lx[:512] = 0.0
    scell = rng.integers(-10, 10, n).astype(np.int32)
    sxf = rng.random(n).astype(np.float32)
    slx = (rng.standard_normal(n) * 1e-8).astype(np.float32)
    z = torch.zeros(n, device="cuda")

    def state(c, x, l):
        lo = torch.zeros((3, n), device="cuda")
        lo[0] = torch.from_numpy(l).cuda()
        return api.State(torch.from_numpy(c).cuda(), torch.from_numpy(x).cuda(), z, z, lo)

    end, snap = state(cell, xf, lx), state(scell, sxf, slx)
    for bins in (256, 4096, 1):
        ws = api.reduce_workspace(n, bins)
        api.reduce_state(snap, end, bins, ws)
        out, hist = api.reduce(ws, n, bins, 3.5)
        xe = (cell.astype(np.float64) + xf.astype(np.float64)) + lx.astype(np.float64)
        xs = (scell.astype(np.float64) + sxf.astype(np.float64)) + slx.astype(np.float64)
        mean, se, h = orc.reduce(xs, xe, 3.5, bins)
        np.testing.assert_array_equal(_np(hist).astype(np.uint64), h)
        assert float(out[0].cpu()) == pytest.approx(mean, rel=1e-12)
        assert float(out[1].cpu()) == pytest.approx(se, rel=1e-9)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129])
def test_ragged_sizes(gpu, orc, n):
    res, (x, v, e, xs), (mean, se, hist) = _run_pair(orc, BASE, n, 401, "em", seed=1, window=7)
    err = mixed_err(_gpu_xve(res), (x, v, e))
    assert err.max() <= 1e-4
    assert abs(res.mean_v - mean) <= 1e-5 * max(1.0, abs(mean))
    assert int(_np(res.hist).sum()) == n


def test_zero_steps_and_partial_blocks(gpu, orc):
    from paper_1104_2499_amd import api

    n = 100
    s = api.init_state(n, 2)
    before = s.clone()
    snap = api.State.empty(n)
    ws = api.reduce_workspace(n, 16)
    api.integrate(s, 0, BASE, step0=6, win_begin=6, snap=snap, ws=ws, n_bins=16)
    out, hist = api.reduce(ws, n, 16, 1.0)
    assert torch.equal(s.xf, before.xf) and torch.equal(snap.xf, before.xf)
    assert float(out[0].cpu()) == 0.0 and int(hist.sum().cpu()) == n
    # 2 steps inside one Philox block, starting mid-block
    api.integrate(s, 2, BASE, step0=5, seed=2)
    x0, v0, e0 = orc.init_state(n, 2)
    x, v, e, _, _ = orc.integrate(BASE, x0, v0, e0, 2, step0=5, seed=2)
    err = mixed_err((_np(s.x64()), _np(s.v64()), _np(s.e64())), (x, v, e))
    assert err.max() <= 1e-6


def test_invalid_arguments_raise(gpu):
    from paper_1104_2499_amd import api

    s = api.init_state(64, 1)
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        api.integrate(s, 10, dict(BASE, D=-1.0))
    with pytest.raises(api.AbpError, match="ABP_E_WORKSPACE"):
        api.integrate(s, 10, BASE, win_begin=0, snap=api.State.empty(64),
                      ws=torch.empty(16, dtype=torch.uint8, device="cuda"), n_bins=256)


def test_full_size_heun_sampled(gpu, orc):
    """2^20 particles, stochastic Heun, in the launch shape the benchmark times: sampled particles
    (first, last, spread) match the oracle one by one after 1e3 steps, and the long-run ensemble
    mean agrees statistically with an oracle sub-ensemble."""
    from paper_1104_2499_amd import api

    n = 1 << 20
    res = api.run(BASE, n=n, steps=1000, window=500, scheme="heun", seed=7, bins=256)
    ids = np.unique(np.concatenate([[0, 1, 63, 64, n - 65, n - 1],
                                    np.random.default_rng(0).integers(0, n, 250)]))
    x0, v0, e0 = orc.init_state(ids.size, 7, ids=ids)
    x, v, e, _, _ = orc.integrate(BASE, x0, v0, e0, 1000, scheme=1, seed=7, ids=ids)
    idx = torch.from_numpy(ids.astype(np.int64)).cuda()
    g = (_np(res.state.x64()[idx]), _np(res.state.v64()[idx]), _np(res.state.e64()[idx]))
    err = mixed_err(g, (x, v, e))
    assert err.max() <= 1e-3 and np.median(err) <= 1e-5
    assert int(_np(res.hist).sum()) == n

    steps, window = 20_000, 10_000
    big = api.run(BASE, n=n, steps=steps, window=window, scheme="heun", seed=7, bins=256)
    m = 4096
    sub = np.arange(m, dtype=np.uint64) * (n // m)
    x0, v0, e0 = orc.init_state(m, 7, ids=sub)
    x, v, e, xs, _ = orc.integrate(BASE, x0, v0, e0, steps, scheme=1, seed=7, ids=sub,
                                   win_begin=steps - window)
    mean, se, _ = orc.reduce(xs, x, window * 1e-3, 256)
    assert abs(big.mean_v - mean) <= 4 * np.hypot(big.stderr, se)
    assert int(_np(big.hist).sum()) == n


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_time_histogram(gpu, orc, scheme):
    """Time-accumulated histogram of x mod 1 (every 100 steps over 1000 steps, 1000 particles,
    64 bins): (i) equal bit for bit to the sum of the final-position histograms of runs stopped
    at each sample step; (ii) chunked calls accumulate like one call; (iii) against the FP64
    oracle, counts differ only by particles whose trajectories differ (here < 1e-3 of all)."""
    from paper_1104_2499_amd import api

    n, S, stride, bins, seed = 1000, 1000, 100, 64, 21
    r = api.run(BASE, n=n, steps=S, window=S, scheme=scheme, seed=seed, bins=bins,
                hist_stride=stride)
    occ = _np(r.occupancy)
    assert occ.sum() == n * (S // stride)
    # (i) by definition, from plain runs and final-position histograms
    st = api.init_state(n, seed)
    snap = api.State.empty(n)
    ws = api.reduce_workspace(n, bins)
    want = np.zeros(bins, dtype=np.int64)
    for k in range(S // stride):
        api.integrate(st, stride, BASE, scheme=scheme, seed=seed, step0=k * stride,
                      win_begin=k * stride, snap=snap, ws=ws, n_bins=bins)
        want += _np(api.reduce(ws, n, bins, 1.0)[1])
    np.testing.assert_array_equal(occ, want)
    # (ii) chunked (boundaries off the sample grid and on it)
    st = api.init_state(n, seed)
    acc = torch.zeros(bins, dtype=torch.int64, device="cuda")
    for a, b in ((0, 370), (370, 400), (400, 1000)):
        api.integrate(st, b - a, BASE, scheme=scheme, seed=seed, step0=a, hist_stride=stride,
                      hist_acc=acc)
    np.testing.assert_array_equal(_np(acc), occ)
    # (iii) oracle
    x0, v0, e0 = orc.init_state(n, seed)
    h, _, _, _ = orc.occupancy(BASE, x0, v0, e0, S, stride, n_bins=bins, seed=seed,
                               scheme=0 if scheme == "em" else 1)
    assert np.abs(occ - h.astype(np.int64)).sum() <= 1e-3 * occ.sum()


def test_time_histogram_edges(gpu):
    """No sample step in range: nothing is added; the counts add to what the array holds;
    invalid arguments are rejected before any launch."""
    from paper_1104_2499_amd import api

    st = api.init_state(300, 3)
    acc = torch.full((16,), 5, dtype=torch.int64, device="cuda")
    api.integrate(st, 99, BASE, seed=3, step0=0, hist_stride=100, hist_acc=acc)
    assert _np(acc).tolist() == [5] * 16
    api.integrate(st, 1, BASE, seed=3, step0=99, hist_stride=100, hist_acc=acc)
    assert _np(acc).sum() == 5 * 16 + 300
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        api.integrate(st, 10, BASE, seed=3, hist_stride=-1, hist_acc=acc)
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        api.integrate(st, 10, BASE, seed=3, hist_stride=5,
                      hist_acc=torch.zeros(12, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        api.integrate(st, 10, BASE, seed=3, hist_stride=5, hist_acc=None)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_largest_step_index(gpu, orc, scheme):
    """The last steps the ABI allows (step0 + n_steps = 2^34: the Philox block counter n/4 at its
    top 32-bit values) against the oracle, starting mid-block; one step more is rejected."""
    from paper_1104_2499_amd import api

    n, top = 333, 1 << 34
    s = api.init_state(n, 6, set_id=3)
    api.integrate(s, 11, BASE, scheme=scheme, seed=6, set_id=3, step0=top - 11)
    x0, v0, e0 = orc.init_state(n, 6, 3)
    x, v, e, _, _ = orc.integrate(BASE, x0, v0, e0, 11, scheme=0 if scheme == "em" else 1,
                                  seed=6, set_id=3, step0=top - 11)
    err = mixed_err((_np(s.x64()), _np(s.v64()), _np(s.e64())), (x, v, e))
    assert err.max() <= 1e-6
    with pytest.raises(api.AbpError, match="ABP_E_ARG"):
        api.integrate(s, 1, BASE, scheme=scheme, seed=6, step0=top)


def test_benchmark_configuration_full_size(gpu, orc):
    """The exact configuration bench.py times (2^20 particles x 1e5 Heun steps, W = 5e4, 256
    bins, default launch shape). After 1e5 steps single trajectories have decorrelated from the
    FP64 path (the dynamics amplify rounding), so the check is by properties that hold at any
    size: a repeat is bit-identical, the histogram holds every particle, and the mean velocity
    agrees within 4 sigma with the oracle's over 8192 evenly spaced particles of the same run."""
    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import WORKLOADS

    wl = WORKLOADS["ensemble-1m-heun"]
    n, S, W = wl["n"], wl["steps"], wl["window"]
    a = api.run(BASE, n=n, steps=S, window=W, scheme="heun", seed=wl["seed"], bins=wl["bins"])
    b = api.run(BASE, n=n, steps=S, window=W, scheme="heun", seed=wl["seed"], bins=wl["bins"])
    assert a.mean_v == b.mean_v and a.stderr == b.stderr and torch.equal(a.hist, b.hist)
    assert int(_np(a.hist).sum()) == n
    m = 8192
    sub = np.arange(m, dtype=np.uint64) * (n // m)
    x0, v0, e0 = orc.init_state(m, wl["seed"], ids=sub)
    x, v, e, xs, _ = orc.integrate(BASE, x0, v0, e0, S, scheme=1, seed=wl["seed"], ids=sub,
                                   win_begin=S - W)
    mean, se, _ = orc.reduce(xs, x, W * wl["dt"], wl["bins"])
    print(f"gpu {a.mean_v:.6e} +- {a.stderr:.2e}; oracle subset {mean:.6e} +- {se:.2e}")
    assert abs(a.mean_v - mean) <= 4 * np.hypot(a.stderr, se)


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_sharding_by_particle_ids(gpu, scheme):
    """What a multi-GPU run would do, on one GPU: two shards holding particle ids [0, n_a) and
    [n_a, n) (abp_state.id0) give, bit for bit, the states of the unsharded run; their histograms
    add up to its histogram and their tile sums to its mean velocity."""
    from paper_1104_2499_amd import api

    n, n_a, S, W, bins = 5000, 2048, 3001, 1000, 64
    full = api.run(BASE, n=n, steps=S, window=W, scheme=scheme, seed=13, bins=bins)
    parts = []
    for id0, m in ((0, n_a), (n_a, n - n_a)):
        st = api.init_state(m, 13, id0=id0)
        snap = api.State.empty(m, id0=id0)
        ws = api.reduce_workspace(m, bins)
        api.integrate(st, S, BASE, scheme=scheme, seed=13, win_begin=S - W, snap=snap, ws=ws,
                      n_bins=bins)
        out, hist = api.reduce(ws, m, bins, W * 1e-3)
        parts.append((st, _np(out), _np(hist), m))
    for name in ("cell", "xf", "v", "e"):
        joined = torch.cat([getattr(p[0], name) for p in parts])
        assert torch.equal(joined, getattr(full.state, name)), name
    assert torch.equal(torch.cat([p[0].lo for p in parts], dim=1), full.state.lo)
    np.testing.assert_array_equal(parts[0][2] + parts[1][2], _np(full.hist))
    combined = sum(p[1][0] * p[3] for p in parts) / n
    assert abs(combined - full.mean_v) <= 1e-14 * max(1.0, abs(full.mean_v))


def test_largest_ensemble(gpu, orc):
    """The largest ensemble the ABI takes (2^31 particles, 60 GB of state plus a 60 GB window
    snapshot in HBM), a few Heun steps: sampled particles (tile edges, the last one, random ids)
    match the oracle and the histogram holds every particle (one particle more is refused before
    any launch: tests/test_abi.py)."""
    from paper_1104_2499_amd import api

    n = 1 << 31
    S, W = 8, 4
    res = api.run(BASE, n=n, steps=S, window=W, scheme="heun", seed=23, bins=256)
    assert int(_np(res.hist).sum()) == n
    assert np.isfinite(res.mean_v) and res.stderr > 0
    ids = np.unique(np.concatenate([[0, 63, 64, (1 << 30) - 1, 1 << 30, n - 65, n - 64, n - 1],
                                    np.random.default_rng(1).integers(0, n, 200)]))
    x0, v0, e0 = orc.init_state(ids.size, 23, ids=ids.astype(np.uint64))
    x, v, e, _, _ = orc.integrate(BASE, x0, v0, e0, S, scheme=1, seed=23, ids=ids)
    idx = torch.from_numpy(ids.astype(np.int64)).cuda()
    st = res.state
    lo = st.lo[:, idx].double()  # gather first: float64 copies of the whole state would be 51 GB
    g = (_np((st.cell[idx].double() + st.xf[idx].double()) + lo[0]),
         _np(st.v[idx].double() + lo[1]), _np(st.e[idx].double() + lo[2]))
    assert mixed_err(g, (x, v, e)).max() <= 1e-6
    del res, st
    torch.cuda.empty_cache()
