"""Host-side marshalling logic (no GPU): parameter rows, configurations, projections."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch


def test_param_rows_places_theta_in_abi_order():
    from paper_1104_2499_amd import adjoint
    from paper_1104_2499_amd.workloads import BASE_PARAMS, PARAM_KEYS

    theta = torch.arange(16, dtype=torch.float64).reshape(2, 8) + 1.0
    cfg = adjoint.AdjointConfig(fixed={"phi": 0.25})
    rows = adjoint.param_rows(theta, cfg, device="cpu")
    assert rows.shape == (2, len(PARAM_KEYS)) and rows.is_contiguous()
    assert rows.dtype == torch.float64
    rows = rows.numpy()
    for j, key in enumerate(adjoint.GRAD_KEYS):
        np.testing.assert_array_equal(rows[:, PARAM_KEYS.index(key)], theta[:, j].numpy())
    np.testing.assert_array_equal(rows[:, PARAM_KEYS.index("phi")], [0.25, 0.25])
    assert set(PARAM_KEYS) == set(adjoint.GRAD_KEYS) | {"phi"}
    assert BASE_PARAMS.keys() == set(PARAM_KEYS)


def test_param_rows_rejects_wrong_width():
    from paper_1104_2499_amd import adjoint

    with pytest.raises(ValueError):
        adjoint.param_rows(torch.zeros(2, 6, dtype=torch.float64), adjoint.AdjointConfig(),
                           device="cpu")


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


def test_tuner_candidates_are_valid_launch_shapes(lib):
    """Every shape the autotuner may pick passes the library's validation (on a host without a
    gfx950 device the call then stops at the device check, not at the arguments)."""
    import ctypes

    from paper_1104_2499_amd import _lib, tune
    from paper_1104_2499_amd.api import make_params, make_tuning

    ptr = 0x10000
    s = _lib.AbpState(ptr, ptr, ptr, ptr, ptr, 64, 0, 0)
    r = _lib.AbpRun(1e-3, 100, 0, -1, 42, 0, 0)
    p = make_params()
    shapes = list(tune.candidates("forward")) + list(tune.candidates("batched"))
    assert len(shapes) == 18 + 36  # 3 blocks x 2 ppl x 3 loop forms (x 2 residencies)
    for shape in shapes:
        t = make_tuning(shape)
        rc = lib.abp_integrate(ctypes.byref(p), ctypes.byref(r), ctypes.byref(s), None, None, 0, 0,
                               ctypes.byref(t), None)
        assert rc != _lib.ABP_E_ARG, shape


def test_tuner_cache_roundtrip(tmp_path, monkeypatch):
    from paper_1104_2499_amd import _lib, tune
    from paper_1104_2499_amd.api import make_tuning

    monkeypatch.setenv("ABP_TUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    monkeypatch.setattr(tune, "device_key", lambda kind, scheme: f"gfx950:256:{kind}:{scheme}")
    assert tune.lookup("batched", "em") is None
    assert make_tuning("auto", "batched", "em") is None
    shape = dict(block=128, ppl=2, unroll=1, waves_per_simd=4)
    assert tune._store_cache({"gfx950:256:batched:em": {"tune": shape}})
    assert tune.lookup("batched", "em") == shape
    t = make_tuning("auto", "batched", _lib.ABP_EM)
    assert (t.block, t.ppl, t.unroll, t.waves_per_simd) == (128, 2, 1, 4)
    assert make_tuning("auto", "forward", "heun") is None
    with pytest.raises(ValueError):
        make_tuning("fastest")
    # an unwritable cache location is not an error: nothing is cached
    blocker = tmp_path / "file"
    blocker.write_text("x")
    monkeypatch.setenv("ABP_TUNE_CACHE", str(blocker / "tune.json"))
    assert tune._store_cache({"k": {}}) is False


def _fresh_python(code: str) -> subprocess.CompletedProcess:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root,
                          timeout=300)


def test_missing_library_fails_loudly():
    """Without libabp.so the product path raises LibraryMissing; there is no CPU or torch
    fallback that would compute something instead."""
    code = (
        "import paper_1104_2499_amd._lib as L\n"
        "L._lib = None\n"
        "L.load.__defaults__ = ('/nonexistent/libabp.so',)\n"
        "from paper_1104_2499_amd import api\n"
        "try:\n"
        "    api.run(None, n=64, steps=10, window=5, device='cpu')\n"
        "except L.LibraryMissing as e:\n"
        "    print('raised', type(e).__name__)\n"
        "else:\n"
        "    print('computed')\n")
    res = _fresh_python(code)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "raised LibraryMissing" in res.stdout


def test_package_never_imports_the_oracle():
    """The oracle is test infrastructure: importing every module of the package leaves it
    unimported."""
    code = (
        "import glob, importlib, os, sys\n"
        "import paper_1104_2499_amd as P\n"
        "for f in sorted(glob.glob(os.path.join(P.__path__[0], '*.py'))):\n"
        "    name = os.path.basename(f)[:-3]\n"
        "    if name != '__init__':\n"
        "        importlib.import_module('paper_1104_2499_amd.' + name)\n"
        "print('oracle' in sys.modules)\n")
    res = _fresh_python(code)
    assert res.returncode == 0, res.stderr[-2000:]
    assert res.stdout.strip().splitlines()[-1] == "False"


def test_python_layer_rejects_bad_arguments_before_any_device_call():
    """Argument errors the binding itself catches (the C ABI validates the rest): they raise
    before anything touches a device, so they are checked here without one."""
    from paper_1104_2499_amd import adjoint, api
    from paper_1104_2499_amd.workloads import sweep_table

    with pytest.raises(KeyError):
        api.make_params(dict(U1=1.0))
    with pytest.raises(ValueError):
        api.make_tuning("fastest")
    with pytest.raises(ValueError):
        api.params_table(np.zeros((3, 8)))
    with pytest.raises(ValueError):
        api.run(None, n=64, steps=10, window=11)
    table, n_traj, n_steps = sweep_table(4, seed=1)
    with pytest.raises(ValueError):
        api.sweep(table, n_traj[:3], n_steps)
    with pytest.raises(ValueError):
        api.sweep(table, n_traj, n_steps, window=n_steps[:3] // 2)  # one window per set
    with pytest.raises(ValueError):
        adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=16, scheme="rk4").abi()
    with pytest.raises(ValueError):
        adjoint.param_rows(torch.zeros((2, 6), dtype=torch.float64),
                           adjoint.AdjointConfig(n=64, steps=100, window=10, ckpt=16),
                           device="cpu")
