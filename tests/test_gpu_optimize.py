"""GPU check of the batched adjoint + Adam loop on a reduced size of the ratchet-design workload."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_adam_loop_small(gpu):
    """8 sets x 256 particles x 2000 steps, 3 Adam iterations: the final adjoint loss equals the
    plain batched integrator's current at the final parameters (bit for bit), the free parameters
    stay inside their bounds and the fixed ones do not move."""
    from paper_1104_2499_amd import optimize
    from paper_1104_2499_amd.adjoint import GRAD_KEYS

    r = optimize.adam_ratchet(n_sets=8, n=256, steps=2000, window=500, ckpt=100, iters=3, seed=5)
    assert r.history.shape == (4,) and np.all(np.isfinite(r.history))
    np.testing.assert_array_equal(r.final_loss, r.verify_mean_v)
    theta0 = optimize.initial_theta(8, 5)
    for j, key in enumerate(GRAD_KEYS):
        if key in optimize.FREE:
            lo, hi = optimize.BOUNDS[key]
            assert np.all(r.theta[:, j] >= lo) and np.all(r.theta[:, j] <= hi)
        else:
            np.testing.assert_array_equal(r.theta[:, j], theta0[:, j])
    assert not np.array_equal(r.theta, theta0)


def test_adam_loop_with_lookback(gpu):
    from paper_1104_2499_amd import optimize

    r = optimize.adam_ratchet(n_sets=4, n=128, steps=1500, window=500, ckpt=64, iters=2, seed=6,
                              lookback=200)
    assert np.all(np.isfinite(r.history))
    np.testing.assert_array_equal(r.final_loss, r.verify_mean_v)
