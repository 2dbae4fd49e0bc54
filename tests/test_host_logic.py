"""Host-side marshalling logic (no GPU): parameter rows, configurations, projections."""
import numpy as np
import pytest
import torch


def test_param_rows_places_theta_in_abi_order():
    from paper_1104_2499_amd import adjoint
    from paper_1104_2499_amd.workloads import BASE_PARAMS, PARAM_KEYS

    theta = torch.arange(16, dtype=torch.float64).reshape(2, 8) + 1.0
    cfg = adjoint.AdjointConfig(fixed={"phi": 0.25})
    rows = adjoint.param_rows(theta, cfg)
    assert rows.shape == (2, len(PARAM_KEYS)) and rows.flags["C_CONTIGUOUS"]
    for j, key in enumerate(adjoint.GRAD_KEYS):
        np.testing.assert_array_equal(rows[:, PARAM_KEYS.index(key)], theta[:, j].numpy())
    np.testing.assert_array_equal(rows[:, PARAM_KEYS.index("phi")], [0.25, 0.25])
    assert set(PARAM_KEYS) == set(adjoint.GRAD_KEYS) | {"phi"}
    assert BASE_PARAMS.keys() == set(PARAM_KEYS)


def test_param_rows_rejects_wrong_width():
    from paper_1104_2499_amd import adjoint

    with pytest.raises(ValueError):
        adjoint.param_rows(torch.zeros(2, 6, dtype=torch.float64), adjoint.AdjointConfig())


def test_adjoint_config_abi_fields():
    from paper_1104_2499_amd import _lib, adjoint

    c = adjoint.AdjointConfig(n=10, steps=100, window=20, ckpt=16, dt=2e-3, seed=9, lookback=5,
                              scheme="heun").abi()
    assert (c.dt, c.n_steps, c.window, c.ckpt_every, c.seed, c.lookback) == (2e-3, 100, 20, 16, 9, 5)
    assert c.scheme == _lib.ABP_HEUN
    with pytest.raises(ValueError):
        adjoint.AdjointConfig(scheme="rk4").abi()


def test_initial_theta_follows_sweep_table():
    from paper_1104_2499_amd import optimize
    from paper_1104_2499_amd.adjoint import GRAD_KEYS
    from paper_1104_2499_amd.workloads import PARAM_KEYS, sweep_table

    th = optimize.initial_theta(16, 3)
    table, _, _ = sweep_table(16, seed=3)
    for j, key in enumerate(GRAD_KEYS):
        np.testing.assert_array_equal(th[:, j], table[:, PARAM_KEYS.index(key)])
