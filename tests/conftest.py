import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def lib():
    """The HIP library (built here if missing); its entry points validate arguments without a
    device."""
    import os

    from paper_1104_2499_amd import _lib, build

    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0. GPU tests fail (never skip) if the device or library is absent."""
    import torch

    assert torch.cuda.is_available(), "gpu-marked test needs a HIP device"
    from paper_1104_2499_amd import _lib

    lib = _lib.load()
    assert lib.abp_abi_version() == _lib.ABI_VERSION
    return lib


def mixed_err(gpu_xyz, ora_xyz):
    """Per-trajectory max over (x, v, e) of |gpu - oracle| / max(1, |oracle|)."""
    import numpy as np

    errs = [np.abs(np.asarray(g, np.float64) - o) / np.maximum(1.0, np.abs(o))
            for g, o in zip(gpu_xyz, ora_xyz)]
    return np.max(np.stack(errs), axis=0)
