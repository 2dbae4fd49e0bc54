"""GPU checks of the paper's own workloads: the load-force curve and the scaling measurement."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_load_force_curve_passive_limit(gpu):
    """Passive particles (d2 = 0) in the tilted ratchet: no current without load, and the mean
    velocity grows with the force."""
    from paper_1104_2499_amd import experiments

    F0 = np.array([-1.5, -0.75, 0.0, 0.75, 1.5])
    out = experiments.load_force_curve(F0, params=dict(d2=0.0, U0=0.2, D=0.5), n=4096,
                                       steps=20_000, window=10_000, scheme="heun", seed=2)
    v, se = out["mean_v"], out["stderr"]
    assert abs(v[2]) <= 4 * se[2]
    assert np.all(np.diff(v) > 0)
    np.testing.assert_allclose(out["load_power"], -F0 * v)
    np.testing.assert_allclose(out["efficiency"], -F0 * v / 1.0)  # q = 1 in the base parameters


def test_load_force_curve_sets_equal_single_runs(gpu):
    from paper_1104_2499_amd import api, experiments

    F0 = np.array([-0.3, 0.0, 0.2])
    out = experiments.load_force_curve(F0, n=300, steps=2003, window=1000, scheme="em", seed=4)
    for k, f in enumerate(F0):
        r = api.run(dict(F0=float(f)), n=300, steps=2003, window=1000, scheme="em", seed=4,
                    bins=0, set_id=k)
        assert r.mean_v == out["mean_v"][k] and r.stderr == out["stderr"][k]


def test_scaling_measurement_shape(gpu):
    from paper_1104_2499_amd import experiments

    rows = experiments.scaling([1, 64, 4096], steps=(0, 200, 400), repeats=4, keep=3)
    assert [r["n"] for r in rows] == [1, 64, 4096]
    for r in rows:
        assert r["t0_us"] > 0 and r["t400_us"] > r["t0_us"]
        assert r["us_per_step"] > 0


def test_density_cost_measurement_shape(gpu):
    """The density-sampling measurement: every sampled histogram holds n x samples counts,
    including a stride that ends calls inside Philox blocks."""
    from paper_1104_2499_amd import experiments

    rows = experiments.density_cost(strides=(0, 100, 7), n=4096, steps=700, repeats=2)
    assert [r["stride"] for r in rows] == [0, 100, 7]
    assert [r["samples"] for r in rows] == [0, 7, 100]
    assert all(r["counts_ok"] for r in rows)
    assert all("extra_us_per_sample" in r for r in rows[1:])
