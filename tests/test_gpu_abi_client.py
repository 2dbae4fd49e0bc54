"""The C ABI from a plain host program (tests/c_client/abi_client.cpp: include/abp.h and the HIP
runtime's C API, no Python binding, no torch): its results equal the Python binding's bit for bit
and invalid calls are rejected with the documented statuses: the single-set integrator and
reduction, the batched sweep and the adjoint's two phases over device parameter tables. The client
runs as a child process, started before this process touches the GPU."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "abi_client")


@pytest.mark.parametrize("scheme", ["em", "heun"])
def test_c_client_equals_python_binding(scheme):
    n, steps, window, seed = 5000, 3000, 1000, 11
    assert os.path.exists(CLIENT), "the C ABI client is built by build()"
    print(f"abi_client {n} {steps} {window} {scheme} {seed}", flush=True)
    proc = subprocess.run([CLIENT, str(n), str(steps), str(window),
                           "0" if scheme == "em" else "1", str(seed)],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stderr
    got = json.loads(proc.stdout.strip().splitlines()[-1])

    import torch

    assert torch.cuda.is_available(), "gpu-marked test needs a HIP device"
    from paper_1104_2499_amd import api
    from paper_1104_2499_amd.workloads import BASE_PARAMS

    res = api.run(BASE_PARAMS, n=n, steps=steps, window=window, scheme=scheme, seed=seed,
                  bins=256)
    assert got["abi_version"] == 4
    assert got["mean_v"] == res.mean_v and got["stderr"] == res.stderr
    assert got["hist_total"] == n and got["hist_first"] == int(res.hist[0])
    assert got["rejected"] == "invalid argument"
    assert got["short_workspace"] == "workspace too small"
    # the batched sweep over device tables: each set equals its single run
    assert got["sweep_status"] == 0
    assert got["sweep_short_workspace"] == "workspace too small"
    sets = [(dict(BASE_PARAMS), n, steps, window), (dict(BASE_PARAMS, U0=1.5), 100, 500, 250),
            (dict(BASE_PARAMS, U0=0.7), 65, 1001, 400)]
    for k, (params, n_k, s_k, w_k) in enumerate(sets):
        r = api.run(params, n=n_k, steps=s_k, window=w_k, scheme=scheme, seed=seed, bins=256,
                    set_id=k)
        assert got["sweep_mean_v"][k] == r.mean_v and got["sweep_stderr"][k] == r.stderr
    # the adjoint over a device table: loss and weighted gradient equal the binding's bit for bit
    from paper_1104_2499_amd import adjoint

    assert got["adjoint_status"] == 0
    assert got["adjoint_rejected"] == "invalid argument"
    cfg = adjoint.AdjointConfig(n=700, steps=steps, window=window, ckpt=100, seed=seed,
                                scheme=scheme)
    theta = torch.tensor([[BASE_PARAMS[k] for k in adjoint.GRAD_KEYS]] * 2, dtype=torch.float64)
    theta[1, adjoint.GRAD_KEYS.index("U0")] = 1.5
    rows = adjoint.param_rows(theta, cfg)
    ws = adjoint.workspace(2, cfg)
    loss = adjoint.forward(rows, cfg, ws).cpu().numpy()
    grad = adjoint.backward(rows, cfg, ws, torch.tensor([1.0, 0.5], dtype=torch.float64))
    assert got["adjoint_loss"] == loss.tolist()
    assert got["adjoint_grad"] == grad.cpu().numpy().reshape(-1).tolist()
