"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle by mathematics or by an independent implementation:
published Philox known-answer vectors and rocRAND's Philox, the normal law of the Box-Muller
output, exact discrete closed forms of the linear sub-models, conserved energy of the frictionless
limit, the fixed point of the depot model, convergence orders against RK4, equilibrium statistics
of the passive ratchet, and complex-step derivatives for the adjoint.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import optimize, stats

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------------------------
# Philox4x32-10
# ----------------------------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answer_vectors(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    ctr = np.array([r[0] for r in rows], dtype=np.uint32)
    key = np.array([r[1] for r in rows], dtype=np.uint32)
    want = np.array([r[2] for r in rows], dtype=np.uint32)
    np.testing.assert_array_equal(orc.philox(ctr, key), want)


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "rocrand_philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    """rocRAND's Philox (run as a black box on the host): key = seed; the state after
    rocrand_init(seed, subsequence, offset) has counter words (offset/4 as 64 bits,
    subsequence as 64 bits), which reaches every counter with c1 < 2^30."""
    rng = np.random.default_rng(20110411)
    m = 4000
    ctr = rng.integers(0, 2**32, size=(m, 4), dtype=np.uint64)
    ctr[:, 1] >>= 2
    key = rng.integers(0, 2**32, size=(m, 2), dtype=np.uint64)
    # edge cases: zero and all-ones keys, counter words at their extremes
    ctr[0] = [0, 0, 0, 0]
    key[0] = [0, 0]
    ctr[1] = [0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]
    key[1] = [0xFFFFFFFF, 0xFFFFFFFF]
    lines = []
    for c, k in zip(ctr, key):
        seed = int(k[0]) | (int(k[1]) << 32)
        sub = int(c[2]) | (int(c[3]) << 32)
        off = 4 * (int(c[0]) | (int(c[1]) << 32))
        lines.append(f"{seed} {sub} {off}")
    out = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split()
    ref = np.array([int(w, 16) for w in out], dtype=np.uint32).reshape(m, 4)
    np.testing.assert_array_equal(orc.philox(ctr.astype(np.uint32), key.astype(np.uint32)), ref)


# ----------------------------------------------------------------------------------------------
# Box-Muller normals and the initial condition
# ----------------------------------------------------------------------------------------------
def test_normals_are_standard_normal(orc):
    z = np.concatenate([orc.normals(7, pid, 3, 0, 4096) for pid in range(64)])
    assert z.shape == (262144,)
    ks = stats.kstest(z, "norm")
    assert ks.pvalue > 1e-3, ks
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    # consecutive normals (same Philox block and across blocks) are uncorrelated
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / np.sqrt(z.size)


def test_noise_stream_is_counter_addressed(orc):
    """Any window of a stream is the same slice of the whole stream (counter-based RNG)."""
    full = orc.normals(42, 5, 0, 0, 1000)
    for s0 in (1, 3, 4, 257, 998):
        np.testing.assert_array_equal(orc.normals(42, 5, 0, s0, 1000 - s0), full[s0:])
    assert not np.array_equal(orc.normals(42, 6, 0, 0, 16), full[:16])
    assert not np.array_equal(orc.normals(43, 5, 0, 0, 16), full[:16])
    assert not np.array_equal(orc.normals(42, 5, 1, 0, 16), full[:16])


def test_initial_positions_uniform_on_24bit_grid(orc):
    x, v, e = orc.init_state(1 << 16, seed=42)
    assert np.all(v == 0) and np.all(e == 0)
    assert x.min() >= 0 and x.max() < 1
    np.testing.assert_array_equal(x * 2**24, np.floor(x * 2**24))
    assert stats.kstest(x, "uniform").pvalue > 1e-3
    xs, _, _ = orc.init_state(8, seed=42, ids=np.arange(100, 108))
    np.testing.assert_array_equal(xs, x[100:108])


# ----------------------------------------------------------------------------------------------
# Drift: potential gradient, friction, load, depot (Eqs. 1-3)
# ----------------------------------------------------------------------------------------------
def _U(x, U0, a, phi=0.0):
    """Eq. (3), two-harmonic ratchet (the model definition, not the oracle's derivative)."""
    return U0 * (np.sin(2 * np.pi * (x + phi)) + a * np.sin(4 * np.pi * (x + phi)))


def test_potential_matches_definition_and_paper_shape(orc):
    for x in (0.0, 0.1, 0.37, 0.9):
        assert orc.potential(dict(U0=1.3, a=0.25, phi=0.1903), x) == pytest.approx(
            _U(x, 1.3, 0.25, 0.1903), abs=1e-14)
    # With the paper's amplitude -0.453 h, a = 1/4, phi = 0.1903 and offset 0.499 h, the ratchet
    # spans [0, h] to within 3e-3 h with its minimum at x = 0 (second harmonic read as 4 pi x).
    xs = np.linspace(0, 1, 200001)
    u = 0.499 + np.array([_U(x, -0.453, 0.25, 0.1903) for x in xs[::1000]])
    assert -3e-3 < u.min() < 3e-3 and 1 - 3e-3 < u.max() < 1 + 3e-3
    assert abs(xs[::1000][np.argmin(u)]) < 6e-3 or abs(xs[::1000][np.argmin(u)] - 1) < 6e-3


@pytest.mark.parametrize("U0,a,phi", [(1.0, 0.25, 0.0), (0.7, 0.4, 0.1903), (2.0, 0.0, 0.3)])
def test_energy_conserved_without_friction(orc, U0, a, phi):
    """gamma0 = d2 = D = F0 = 0: Hamiltonian flow, H = v^2/2 + U(x) is conserved. A wrong sign,
    factor or phase in the oracle's U'(x) breaks this."""
    p = dict(U0=U0, a=a, phi=phi, gamma0=0.0, d2=0.0, D=0.0, F0=0.0)
    x0 = np.linspace(0.05, 0.95, 7)
    v0 = np.linspace(-1.5, 1.5, 7)
    e0 = np.zeros(7)
    H0 = v0**2 / 2 + _U(x0, U0, a, phi)
    x, v, _ = orc.rk4(p, x0, v0, e0, 20000, 1e-3)
    H = v**2 / 2 + _U(x, U0, a, phi)
    np.testing.assert_allclose(H, H0, atol=1e-9)
    assert np.abs(x - x0).max() > 0.1  # particles actually moved


def test_damped_particle_settles_in_potential_minimum(orc):
    """gamma0 = 1, D = d2 = F0 = 0: the particle stops where U' = 0 and U'' > 0."""
    U0, a = 1.0, 0.25
    xmin = optimize.minimize_scalar(lambda x: _U(x, U0, a), bounds=(0.5, 1.0), method="bounded",
                                    options=dict(xatol=1e-12)).x
    x0 = np.array([xmin - 0.2, xmin - 0.05, xmin + 0.1])
    x, v, _ = orc.rk4(dict(U0=U0, a=a, gamma0=1.0, d2=0.0, D=0.0), x0, np.zeros(3), np.zeros(3),
                      40000, 1e-3)
    np.testing.assert_allclose(x, xmin, atol=1e-8)
    np.testing.assert_allclose(v, 0.0, atol=1e-8)


def test_load_force_mobility(orc):
    """U0 = d2 = 0: the velocity relaxes to the mobility value F0/gamma0 (EM fixed point)."""
    n = 4096
    x, v, e = orc.init_state(n, 3)
    p = dict(U0=0.0, d2=0.0, F0=0.7, gamma0=2.0, D=0.05)
    x, v, e, xs, vs = orc.integrate(p, x, v, e, 10000, win_begin=2000, seed=3)
    mean, se, _ = orc.reduce(xs, x, 8.0)
    assert abs(mean - 0.35) < 4 * se + 1e-12
    assert se < 5e-3


@pytest.mark.parametrize("scheme", [0, 1])
def test_depot_closed_form(orc, scheme):
    """d2 = 0 decouples Eq. (1): EM gives e_n = (q/c)(1 - (1 - c dt)^n); Heun gives the same with
    the factor 1 - c dt + (c dt)^2/2."""
    q, c, dt, n = 1.3, 0.1, 1e-3, 12345
    x, v, e = orc.init_state(4, 1)
    _, _, e, _, _ = orc.integrate(dict(q=q, c=c, d2=0.0), x, v, e, n, dt=dt, scheme=scheme)
    rho = 1 - c * dt if scheme == 0 else 1 - c * dt + (c * dt) ** 2 / 2
    np.testing.assert_allclose(e, q / c * (1 - rho**n), rtol=1e-12)


def test_active_fixed_point(orc):
    """U0 = F0 = D = 0: the depot drives self-propulsion at v*^2 = q/gamma0 - c/d2 with
    e* = gamma0/d2 (set dv/dt = 0 with v != 0 and de/dt = 0)."""
    g0, d2, q, c = 1.0, 1.0, 1.0, 0.1
    p = dict(U0=0.0, F0=0.0, D=0.0, gamma0=g0, d2=d2, q=q, c=c)
    x, v, e = orc.rk4(p, np.zeros(2), np.array([0.1, -0.2]), np.zeros(2), 60000, 1e-3)
    vstar = np.sqrt(q / g0 - c / d2)
    np.testing.assert_allclose(v, [vstar, -vstar], rtol=1e-7)
    np.testing.assert_allclose(e, g0 / d2, rtol=1e-7)
    # EM has the same fixed points
    x2, v2, e2, _, _ = orc.integrate(p, np.zeros(2), np.array([0.1, -0.2]), np.zeros(2), 60000)
    np.testing.assert_allclose(v2, [vstar, -vstar], rtol=1e-6)


@pytest.mark.parametrize("scheme", [0, 1])
def test_ou_stationary_variance(orc, scheme):
    """Free particle (U0 = d2 = F0 = 0): v follows the AR(1) map v' = rho v + s xi with
    EM: rho = 1 - g dt, s = sigma;  Heun: rho = 1 - g dt + (g dt)^2/2, s = sigma (1 - g dt/2),
    so Var v_n = s^2 (1 - rho^(2n)) / (1 - rho^2) (-> D/gamma0 as dt -> 0)."""
    n, S, dt, g, D = 1 << 15, 6000, 1e-3, 1.0, 0.3
    x, v, e = orc.init_state(n, 11)
    _, v, _, _, _ = orc.integrate(dict(U0=0.0, d2=0.0, gamma0=g, D=D), x, v, e, S, dt=dt,
                                  scheme=scheme, seed=11)
    sig = np.sqrt(2 * D * dt)
    if scheme == 0:
        rho, s = 1 - g * dt, sig
    else:
        rho, s = 1 - g * dt + (g * dt) ** 2 / 2, sig * (1 - g * dt / 2)
    want = s**2 * (1 - rho ** (2 * S)) / (1 - rho**2)
    assert abs(v.var() / want - 1) < 4 * np.sqrt(2 / n)
    assert abs(v.mean()) < 4 * np.sqrt(want / n)
    assert want == pytest.approx(D / g, rel=5e-3)


@pytest.mark.parametrize("scheme,order", [(0, 1.0), (1, 2.0)])
def test_deterministic_limit_convergence_order(orc, scheme, order):
    """D = 0: EM converges to RK4 (dt/100) with global order 1, Heun with order 2."""
    p = dict(D=0.0)
    x0, v0, e0 = np.array([0.13, 0.61]), np.array([0.5, -0.3]), np.array([0.2, 1.0])
    T = 1.0
    xr, vr, er = orc.rk4(p, x0, v0, e0, 100000, 1e-5)
    errs = []
    for dt in (1e-2, 5e-3, 2.5e-3):
        x, v, e, _, _ = orc.integrate(p, x0, v0, e0, int(round(T / dt)), dt=dt, scheme=scheme)
        errs.append(max(np.abs(x - xr).max(), np.abs(v - vr).max(), np.abs(e - er).max()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    np.testing.assert_allclose(rates, order, atol=0.15)


def test_passive_ratchet_zero_current_and_boltzmann(orc):
    """d2 = F0 = 0: detailed balance. The mean current vanishes and x mod 1 follows the
    Boltzmann law exp(-gamma0 U(x) / D) (temperature D/gamma0)."""
    n, S, dt = 16384, 20000, 1e-3
    U0, a, D, g = 0.2, 0.25, 0.5, 1.0
    p = dict(U0=U0, a=a, D=D, gamma0=g, d2=0.0, F0=0.0)
    x, v, e = orc.init_state(n, 5)
    x, v, e, xs, _ = orc.integrate(p, x, v, e, S, dt=dt, seed=5, win_begin=5000)
    mean, se, hist = orc.reduce(xs, x, (S - 5000) * dt, n_bins=32)
    assert abs(mean) < 4 * se
    edges = np.linspace(0, 1, 33)
    fine = np.linspace(0, 1, 32 * 64 + 1)[:-1] + 0.5 / (32 * 64)
    w = np.exp(-g * _U(fine, U0, a) / D).reshape(32, 64).sum(axis=1)
    expected = n * w / w.sum()
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, 31) > 1e-3, (chi2, hist, expected)
    assert edges.size == 33


def test_occupancy_time_average_is_boltzmann(orc):
    """The time-accumulated histogram of passive particles (d2 = F0 = 0) after a burn-in follows
    the same Boltzmann law as the snapshot: total-variation distance below 0.015 with 4096
    particles x 30 samples (measured 0.006; the histogram shifted by one bin gives 0.028, a flat
    one 0.125)."""
    n, dt = 4096, 1e-3
    U0, a, D, g = 0.2, 0.25, 0.5, 1.0
    p = dict(U0=U0, a=a, D=D, gamma0=g, d2=0.0, F0=0.0)
    x, v, e = orc.init_state(n, 8)
    x, v, e, _, _ = orc.integrate(p, x, v, e, 5000, dt=dt, seed=8)
    occ, _, _, _ = orc.occupancy(p, x, v, e, 15000, 500, n_bins=32, dt=dt, seed=8, step0=5000)
    assert occ.sum() == n * 30
    fine = np.linspace(0, 1, 32 * 64 + 1)[:-1] + 0.5 / (32 * 64)
    w = np.exp(-g * _U(fine, U0, a) / D).reshape(32, 64).sum(axis=1)
    tv = 0.5 * np.abs(occ / occ.sum() - w / w.sum()).sum()
    assert tv < 0.015, tv


def test_occupancy_definition_cases(orc):
    """One sample at the end equals the final-position histogram; the sample count is the number
    of multiples of the stride in (step0, step0 + n_steps]; sampling leaves the state unchanged;
    chunked accumulation equals one call."""
    x0, v0, e0 = orc.init_state(300, 4)
    occ, x, v, e = orc.occupancy(None, x0, v0, e0, 400, 400, n_bins=64, seed=4)
    xf, vf, ef, _, _ = orc.integrate(None, x0, v0, e0, 400, seed=4)
    np.testing.assert_array_equal(occ, orc.reduce(xf, xf, 1.0, 64)[2])
    for a_, b_ in zip((x, v, e), (xf, vf, ef)):
        np.testing.assert_array_equal(a_, b_)
    occ, _, _, _ = orc.occupancy(None, x0, v0, e0, 100, 10, n_bins=16, seed=4, step0=7)
    assert occ.sum() == 300 * 10
    full, xa, _, _ = orc.occupancy(None, x0, v0, e0, 300, 20, n_bins=64, seed=4)
    h1, x1, v1, e1 = orc.occupancy(None, x0, v0, e0, 130, 20, n_bins=64, seed=4)
    h2, x2, _, _ = orc.occupancy(None, x1, v1, e1, 170, 20, n_bins=64, seed=4, step0=130)
    np.testing.assert_array_equal(full, h1 + h2)
    np.testing.assert_array_equal(xa, x2)


def test_em_displacement_equals_time_average(orc):
    """For EM, x_S - x_(S-W) = dt * sum of v_n over the window exactly (x uses the old v)."""
    x, v, e = orc.init_state(256, 42)
    x, v, e, xs, vs = orc.integrate(None, x, v, e, 4000, win_begin=1500)
    np.testing.assert_allclose((x - xs) / (2500 * 1e-3), vs / 2500, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("scheme", [0, 1])
def test_chunked_equals_unchunked(orc, scheme):
    x0, v0, e0 = orc.init_state(64, 9)
    full = orc.integrate(None, x0, v0, e0, 1003, scheme=scheme, seed=9, win_begin=501)
    x, v, e, xs, vs = orc.integrate(None, x0, v0, e0, 333, scheme=scheme, seed=9, win_begin=501)
    x, v, e, xs, vs = orc.integrate(None, x, v, e, 170, scheme=scheme, seed=9, step0=333,
                                    win_begin=501, x_snap=xs, v_sum=vs)
    x, v, e, xs, vs = orc.integrate(None, x, v, e, 500, scheme=scheme, seed=9, step0=503,
                                    win_begin=501, x_snap=xs, v_sum=vs)
    for a_, b_ in zip(full, (x, v, e, xs, vs)):
        np.testing.assert_array_equal(a_, b_)


# ----------------------------------------------------------------------------------------------
# Reductions
# ----------------------------------------------------------------------------------------------
def test_reduce_statistics_and_histogram_fixture(orc):
    rng = np.random.default_rng(0)
    xs = rng.normal(size=1000) * 3
    xe = xs + rng.normal(size=1000) * 0.5 + 0.2
    mean, se, hist = orc.reduce(xs, xe, 2.0, n_bins=256)
    d = xe - xs
    assert mean == pytest.approx(d.mean() / 2.0, rel=1e-13)
    assert se == pytest.approx(d.std(ddof=1) / np.sqrt(1000) / 2.0, rel=1e-10)
    assert hist.sum() == 1000 and hist.dtype == np.uint64
    # hand-placed points: bin k of 256 holds x with k/256 <= x mod 1 < (k+1)/256
    pts = np.array([0.0, 1.0 / 256, 0.5, -0.5, 3.999, -1e-9, 7.25 + 1e-12, -2.0])
    _, _, h = orc.reduce(np.zeros(8), pts, 1.0, n_bins=256)
    want = np.zeros(256, np.uint64)
    for b in (0, 1, 128, 128, 255, 255, 64, 0):
        want[b] += 1
    np.testing.assert_array_equal(h, want)


# ----------------------------------------------------------------------------------------------
# Adjoint
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [0, 1])
def test_complex_step_real_part_is_the_forward(orc, scheme):
    x0, v0, e0 = orc.init_state(32, 42)
    x, v, e, xs, _ = orc.integrate(None, x0, v0, e0, 800, win_begin=600, scheme=scheme)
    J = (x - xs) / (200 * 1e-3)
    for k in range(8):
        _, Jre = orc.complex_step(None, k, x0, v0, e0, 800, 200, scheme=scheme)
        np.testing.assert_allclose(Jre, J, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("scheme", [0, 1])
def test_adjoint_matches_complex_step(orc, scheme):
    """Reverse mode (adjoint) and forward mode (complex step) on the same FP64 path, for all
    eight parameters and both schemes."""
    n, S, W = 64, 1000, 200
    x0, v0, e0 = orc.init_state(n, 42)
    p = dict(F0=0.1, phi=0.07)
    J, g = orc.adjoint(p, x0, v0, e0, S, W, scheme=scheme)
    assert g.shape == (n, 8)
    for k in range(8):
        cs, Jre = orc.complex_step(p, k, x0, v0, e0, S, W, scheme=scheme)
        np.testing.assert_allclose(Jre, J, rtol=1e-12, atol=1e-12)
        scale = np.abs(cs).max()
        np.testing.assert_allclose(g[:, k], cs, rtol=1e-8, atol=1e-10 * scale)


@pytest.mark.parametrize("scheme", [0, 1])
def test_adjoint_matches_central_differences(orc, scheme):
    """Ensemble gradient vs central differences with common random numbers (h = 1e-4)."""
    n, S, W = 256, 1000, 200
    x0, v0, e0 = orc.init_state(n, 42)
    _, g = orc.adjoint(None, x0, v0, e0, S, W, scheme=scheme)
    base = dict(orc.DEFAULTS)
    for k, name in enumerate(orc.GRAD_KEYS):
        def L(val):
            p = dict(base)
            p[name] = val
            x, _, _, xs, _ = orc.integrate(p, x0, v0, e0, S, win_begin=S - W, scheme=scheme)
            return ((x - xs) / (W * 1e-3)).mean()
        h = 1e-4
        fd = (L(base[name] + h) - L(base[name] - h)) / (2 * h)
        assert abs(g[:, k].mean() - fd) <= 1e-3 * abs(fd) + 1e-9, (name, g[:, k].mean(), fd)


def test_adjoint_rejects_zero_noise(orc):
    x0, v0, e0 = orc.init_state(4, 1)
    with pytest.raises(ValueError):
        orc.adjoint(dict(D=0.0), x0, v0, e0, 100, 10)


def test_decayed_adjoint_limits_and_ou_closed_form(orc):
    """The decayed estimator: (i) with an effectively infinite look-back it is the exact gradient
    (for EM the velocity-sum form of J equals the displacement form); (ii) for the free particle
    (U0 = d2 = 0) v_n = sum_m r^(n-1-m) sigma xi_m with r = 1 - gamma0 dt, and the damping acts
    once per step between v_(m+1) and v_n, so the decayed
    dJ/dD = (1/W) sum_{n>=wb} sum_{m<n} (r rho)^(n-1-m) xi_m dsigma/dD in closed form, and J does
    not depend on q or c."""
    n, S, W = 16, 600, 200
    x0, v0, e0 = orc.init_state(n, 4)
    J, g = orc.adjoint(None, x0, v0, e0, S, W, seed=4)
    J2, g2 = orc.adjoint(None, x0, v0, e0, S, W, seed=4, lookback=10**15)
    np.testing.assert_allclose(g2, g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
    D, T, dt = 0.3, 50, 1e-3
    p = dict(U0=0.0, d2=0.0, D=D, gamma0=1.0)
    _, gd = orc.adjoint(p, x0, v0, e0, S, W, seed=4, lookback=T)
    r, rho = 1 - dt, 1 - 1 / T
    dsig = np.sqrt(dt / (2 * D))
    for i in range(n):
        xi = orc.normals(4, i, 0, 0, S)
        total = 0.0
        for k in range(S - W, S):
            m = np.arange(k)
            total += np.sum((r * rho) ** (k - 1 - m) * xi[m]) * dsig
        assert gd[i, 2] == pytest.approx(total / W, rel=1e-9, abs=1e-12)
        assert abs(gd[i, 4]) < 1e-15 and abs(gd[i, 5]) < 1e-15


def test_thread_count_does_not_change_results(orc):
    """The oracle's OpenMP split is over independent particles: one thread and all threads give
    the same bits (the single-core timings rely on it)."""
    x, v, e = orc.init_state(96, 5)
    ref = orc.integrate(None, x, v, e, 300, scheme=orc.HEUN, seed=5, win_begin=100)
    J0, g0 = orc.adjoint(None, x, v, e, 200, 50, seed=5)
    n = orc.num_threads()
    orc.set_num_threads(1)
    try:
        one = orc.integrate(None, x, v, e, 300, scheme=orc.HEUN, seed=5, win_begin=100)
        J1, g1 = orc.adjoint(None, x, v, e, 200, 50, seed=5)
    finally:
        orc.set_num_threads(n)
    for a, b in zip(ref, one):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(J0, J1)
    np.testing.assert_array_equal(g0, g1)


# ----------------------------------------------------------------------------------------------
# Rounding-sensitivity model (eps != 0): x += eps u0, v *= 1 + eps u1, e *= 1 + eps u2 after
# every step, u uniform on [-1, 1) and independent across steps and coordinates. It sets the
# tolerance of the long-horizon trajectory and gradient gates, so its placement and scale are
# fixed here by closed forms of sub-models where the perturbation is the only thing that moves.
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("eps", [2.0**-24, 1e-3])
def test_perturbation_is_an_unbiased_random_walk_in_x(orc, scheme, eps):
    """U0 = F0 = q = c = D = 0 with v0 = e0 = 0: the drift and the noise vanish, v and e stay
    exactly 0, and x_n - x_0 = eps * sum of n independent U[-1, 1) draws: mean 0, variance
    n eps^2 / 3 (a wrong scale, a bias, a relative instead of an absolute placement in x, or a
    draw reused across steps fails this)."""
    n, S = 8192, 1000
    p = dict(U0=0.0, F0=0.0, q=0.0, c=0.0, D=0.0)
    x0, v0, e0 = orc.init_state(n, 21)
    x, v, e, _, _ = orc.integrate(p, x0, v0, e0, S, scheme=scheme, seed=21, eps=eps)
    assert not v.any() and not e.any()
    z = (x - x0) / (eps * np.sqrt(S / 3.0))
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # without the model nothing moves at all
    x1, _, _, _, _ = orc.integrate(p, x0, v0, e0, S, scheme=scheme, seed=21)
    np.testing.assert_array_equal(x1, x0)


@pytest.mark.parametrize("scheme", [0, 1])
def test_perturbation_is_relative_in_v_and_e(orc, scheme):
    """Free damped particle with an empty-input depot (U0 = F0 = d2 = q = D = 0, v0 = e0 = 1):
    v and e decay geometrically, v_n = r_v^n prod(1 + eps u1), e_n = r_e^n prod(1 + eps u2), so
    log(v_n / v_n^0) and log(e_n / e_n^0) are sums of n independent log(1 + eps u) terms:
    variance n eps^2 / 3 to first order, and the two are uncorrelated (different Philox
    words)."""
    n, S, eps = 8192, 1000, 1e-3
    p = dict(U0=0.0, F0=0.0, d2=0.0, q=0.0, c=0.5, gamma0=2.0, D=0.0)
    x0, _, _ = orc.init_state(n, 22)
    v0, e0 = np.ones(n), np.ones(n)
    _, v, e, _, _ = orc.integrate(p, x0, v0, e0, S, scheme=scheme, seed=22, eps=eps)
    _, vr, er, _, _ = orc.integrate(p, x0, v0, e0, S, scheme=scheme, seed=22)
    np.testing.assert_allclose(vr, vr[0], rtol=1e-15)  # unperturbed: deterministic decay
    # E log(1 + eps u) = -eps^2/6 + O(eps^4); Var = eps^2/3 + O(eps^4)
    for lr in (np.log(v / vr), np.log(e / er)):
        z = (lr + S * eps**2 / 6) / (eps * np.sqrt(S / 3.0))
        assert abs(z.mean()) < 5 / np.sqrt(n)
        assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    c = np.corrcoef(np.log(v / vr), np.log(e / er))[0, 1]
    assert abs(c) < 5 / np.sqrt(n)


@pytest.mark.parametrize("scheme", [0, 1])
def test_one_perturbed_step_is_bounded_by_eps(orc, scheme):
    """After one step from any state the perturbed and unperturbed results differ by at most
    eps in x (absolute) and by a factor within [1 - eps, 1 + eps] in v and e; over many particles
    the bound is nearly reached on both sides (the scale is eps, not a fraction of it)."""
    n, eps = 1 << 14, 1e-3
    rng = np.random.default_rng(5)
    x0 = rng.uniform(-3, 3, n)
    v0 = rng.uniform(0.2, 2.0, n) * rng.choice([-1, 1], n)
    e0 = rng.uniform(0.1, 3.0, n)
    for step0 in (0, 7, 12345):
        x, v, e, _, _ = orc.integrate(None, x0, v0, e0, 1, scheme=scheme, step0=step0, eps=eps)
        xr, vr, er, _, _ = orc.integrate(None, x0, v0, e0, 1, scheme=scheme, step0=step0)
        dx = (x - xr) / eps
        rv = (v / vr - 1) / eps
        re = (e / er - 1) / eps
        for d in (dx, rv, re):
            assert np.abs(d).max() <= 1.0 + 1e-9
            assert d.max() > 0.99 and d.min() < -0.99


def test_linearised_adjoint_follows_the_perturbed_path(orc):
    """With eps != 0 the adjoint is the exact gradient evaluated along the perturbed path. For
    the linear free particle (U0 = d2 = 0, EM) the adjoint lambda is path-independent and known in
    closed form: lambda_x(n+1) = 1/(W dt) for n >= S - W, else 0, and
    lambda_v(n) = lambda_x(n+1) dt + (1 - gamma0 dt) lambda_v(n+1); hence
    dJ/dgamma0 = -dt sum_n lambda_v(n+1) v_n with v_n the perturbed velocities (recovered from the
    oracle's integrator one step at a time), while the F0, q and D components do not depend on
    the path at all."""
    n, S, W, eps, dt, g0 = 16, 400, 150, 1e-3, 1e-3, 1.3
    p = dict(U0=0.0, d2=0.0, gamma0=g0, D=0.2, F0=0.1)
    x0, v0, e0 = orc.init_state(n, 31)
    J, g = orc.adjoint(p, x0, v0, e0, S, W, seed=31, eps=eps)
    J0, g0_ = orc.adjoint(p, x0, v0, e0, S, W, seed=31)
    # J is the perturbed path's displacement
    xe, _, _, xs, _ = orc.integrate(p, x0, v0, e0, S, seed=31, win_begin=S - W, eps=eps)
    np.testing.assert_allclose(J, (xe - xs) / (W * dt), rtol=1e-12)
    # path-independent components are unchanged by the perturbation
    for k in (2, 4, 7):  # D, q, F0
        np.testing.assert_array_equal(g[:, k], g0_[:, k])
    lam_x = np.where(np.arange(S) >= S - W, 1.0 / (W * dt), 0.0)  # lambda_x(n+1) for n = 0..S-1
    lam_v = np.zeros(S + 1)
    for m in range(S - 1, -1, -1):
        lam_v[m] = lam_x[m] * dt + (1 - g0 * dt) * lam_v[m + 1]
    vs = np.empty((S, n))
    x, v, e = x0.copy(), v0.copy(), e0.copy()
    for m in range(S):
        vs[m] = v
        x, v, e, _, _ = orc.integrate(p, x, v, e, 1, seed=31, step0=m, eps=eps)
    want = -dt * (lam_v[1:, None] * vs).sum(axis=0)
    np.testing.assert_allclose(g[:, 6], want, rtol=1e-10)
    # the check has teeth: the unperturbed gradient is measurably different
    assert np.all(np.abs(g0_[:, 6] - want) > 1e-6 * np.abs(want))


@pytest.mark.parametrize("scheme", [0, 1])
def test_adjoint_matches_complex_step_at_the_full_horizon(orc, scheme):
    """G1 at the gradient workload's horizon (S = 1e4, W = 2000) on 1024 evenly spaced particles
    of the 65536-particle ensemble, all eight components: reverse mode (adjoint) and forward mode
    (complex step) on the same FP64 path agree to <= 1e-8 relative for >= 99.9% of the particles
    (measured max 5e-11) and to 1e-6 for all."""
    n_all, n, S, W = 65536, 1024, 10_000, 2_000
    ids = (np.arange(n, dtype=np.uint64) * (n_all // n)).astype(np.uint32)
    x0, v0, e0 = orc.init_state(n, 42, ids=ids)
    J, g = orc.adjoint(None, x0, v0, e0, S, W, seed=42, ids=ids, scheme=scheme)
    worst = 0.0
    for k in range(8):
        cs, Jre = orc.complex_step(None, k, x0, v0, e0, S, W, seed=42, ids=ids, scheme=scheme)
        np.testing.assert_allclose(Jre, J, rtol=1e-12, atol=1e-12)
        rel = np.abs(g[:, k] - cs) / np.abs(cs)
        assert (rel <= 1e-8).mean() >= 0.999, (orc.GRAD_KEYS[k], np.quantile(rel, 0.999))
        assert rel.max() <= 1e-6, (orc.GRAD_KEYS[k], rel.max())
        worst = max(worst, rel.max())
    print(f"scheme {scheme}: max relative |adjoint - complex step| = {worst:.2e}")
