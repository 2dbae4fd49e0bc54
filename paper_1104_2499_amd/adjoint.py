"""Pathwise gradients of the window mean velocity as a torch.autograd.Function.

theta [n_sets, 8] float64 holds (U0, a, D, d2, q, c, gamma0, F0) per parameter set; the phase phi
of the potential, Eq. (3), is fixed by the config. The forward pass runs abp_adjoint phase 0
(integrate with checkpoints, loss L_k = mean velocity of set k over the last W steps); backward
runs phase 1 (checkpointed discrete adjoint of the Euler-Maruyama or Heun map, with regenerated
noise). All arithmetic is in the HIP
library; torch provides the buffers and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from .api import SCHEMES, _ptr, _stream, check, check_device_status
from .workloads import BASE_PARAMS, PARAM_KEYS

GRAD_KEYS = ("U0", "a", "D", "d2", "q", "c", "gamma0", "F0")


@dataclass
class AdjointConfig:
    n: int = 65536            # particles per set
    steps: int = 10_000       # S
    window: int = 2_000       # W
    ckpt: int = 100           # K
    dt: float = 1e-3
    seed: int = 42
    lookback: int = 0         # 0 = exact gradient; T > 0 = sensitivities damped by (1 - 1/T)/step
    scheme: str = "em"        # "em" or "heun" (lookback > 0 needs "em")
    stage: int = 0            # backward register staging: 0 = default (16); 8 = two EM wavefronts/SIMD
    fixed: dict = field(default_factory=lambda: {"phi": BASE_PARAMS["phi"]})

    def abi(self) -> _lib.AbpAdjointCfg:
        if self.scheme not in SCHEMES:
            raise ValueError(f"scheme must be one of {sorted(SCHEMES)}")
        return _lib.AbpAdjointCfg(self.dt, self.steps, self.window, self.ckpt, self.seed,
                                  self.lookback, SCHEMES[self.scheme], self.stage)


def param_rows(theta: torch.Tensor, cfg: AdjointConfig, device="cuda") -> torch.Tensor:
    """[n_sets, 9] float64 device rows in PARAM_KEYS order from theta [n_sets, 8]: the fixed
    parameters from the config, the rest copied from theta on the device (no host round trip)."""
    th = theta.detach()
    if th.ndim != 2 or th.shape[1] != len(GRAD_KEYS):
        raise ValueError("theta must be [n_sets, 8] = (U0, a, D, d2, q, c, gamma0, F0)")
    th = th.to(device=device, dtype=torch.float64)
    base = dict(BASE_PARAMS, **cfg.fixed)
    row = torch.tensor([base[k] for k in PARAM_KEYS], dtype=torch.float64, device=device)
    rows = row.repeat(th.shape[0], 1)
    rows[:, [PARAM_KEYS.index(k) for k in GRAD_KEYS]] = th
    return rows.contiguous()


def workspace(n_sets: int, cfg: AdjointConfig, device="cuda") -> torch.Tensor:
    nbytes = int(_lib.load().abp_adjoint_workspace_bytes(n_sets, cfg.n, cfg.steps, cfg.ckpt))
    if nbytes == 0:
        raise ValueError("invalid adjoint sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _check_rows(rows: torch.Tensor) -> None:
    if (rows.dtype != torch.float64 or rows.ndim != 2 or rows.shape[1] != len(PARAM_KEYS)
            or not rows.is_contiguous() or not rows.is_cuda):
        raise ValueError("rows must be a contiguous [n_sets, 9] float64 device tensor")


def _finish(status: torch.Tensor, check_status: bool, stream, where: str) -> None:
    if check_status:
        if stream is not None:
            stream.synchronize()
        check_device_status(status, where)


def forward(rows: torch.Tensor, cfg: AdjointConfig, ws: torch.Tensor, stream=None,
            status: torch.Tensor | None = None, loss: torch.Tensor | None = None,
            check_status: bool = True) -> torch.Tensor:
    """Phase 0 (abp_adjoint): the loss per set; enqueue-only when check_status is False (the
    device-side status then lands in `status` for the caller to read)."""
    _check_rows(rows)
    n_sets = rows.shape[0]
    loss = torch.empty(n_sets, dtype=torch.float64, device=ws.device) if loss is None else loss
    status = torch.empty(1, dtype=torch.int32, device=ws.device) if status is None else status
    c = cfg.abi()
    check(_lib.load().abp_adjoint(0, n_sets, _ptr(rows), cfg.n, ctypes.byref(c), _ptr(ws),
                                  ws.numel(), _ptr(loss), None, None, None, _ptr(status),
                                  _stream(stream)), "abp_adjoint(forward)")
    _finish(status, check_status, stream, "abp_adjoint(forward)")
    return loss


def backward(rows: torch.Tensor, cfg: AdjointConfig, ws: torch.Tensor, gloss: torch.Tensor,
             per_particle: bool = False, stream=None, status: torch.Tensor | None = None,
             grad: torch.Tensor | None = None, check_status: bool = True):
    """Phase 1 (abp_adjoint): gloss[k] * dL_k/dtheta, and optionally the per-particle gradients."""
    _check_rows(rows)
    n_sets = rows.shape[0]
    gloss = gloss.detach().to(ws.device, torch.float64).contiguous()
    ng = len(GRAD_KEYS)
    grad = (torch.empty((n_sets, ng), dtype=torch.float64, device=ws.device)
            if grad is None else grad)
    gp = (torch.empty((n_sets, cfg.n, ng), dtype=torch.float64, device=ws.device)
          if per_particle else None)
    status = torch.empty(1, dtype=torch.int32, device=ws.device) if status is None else status
    c = cfg.abi()
    check(_lib.load().abp_adjoint(1, n_sets, _ptr(rows), cfg.n, ctypes.byref(c), _ptr(ws),
                                  ws.numel(), None, _ptr(gloss), _ptr(grad), _ptr(gp),
                                  _ptr(status), _stream(stream)), "abp_adjoint(backward)")
    _finish(status, check_status, stream, "abp_adjoint(backward)")
    return (grad, gp) if per_particle else grad


class MeanVelocity(torch.autograd.Function):
    """L = MeanVelocity.apply(theta, cfg): theta [n_sets, 8] -> L [n_sets] (float64, cuda).
    The parameters stay on the device: the rows the library reads are assembled there."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, cfg: AdjointConfig):
        rows = param_rows(theta, cfg)
        ws = workspace(rows.shape[0], cfg)
        loss = forward(rows, cfg, ws)
        ctx.rows, ctx.cfg, ctx.ws = rows, cfg, ws
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return loss

    @staticmethod
    def backward(ctx, gloss: torch.Tensor):
        grad = backward(ctx.rows, ctx.cfg, ctx.ws, gloss)
        return grad.to(ctx.theta_device, ctx.theta_dtype), None


def mean_velocity(theta: torch.Tensor, cfg: AdjointConfig) -> torch.Tensor:
    return MeanVelocity.apply(theta, cfg)
