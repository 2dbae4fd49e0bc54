"""Pathwise gradients of the window mean velocity as a torch.autograd.Function.

theta [n_sets, 8] float64 holds (U0, a, D, d2, q, c, gamma0, F0) per parameter set; the phase phi
of the potential, Eq. (4), is fixed by the config. The forward pass runs abp_adjoint phase 0
(integrate with checkpoints, loss L_k = mean velocity of set k over the last W steps); backward
runs phase 1 (checkpointed discrete adjoint of the Euler-Maruyama or Heun map, with regenerated
noise). All arithmetic is in the HIP
library; torch provides the buffers and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .api import SCHEMES, _stream, check
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


def param_rows(theta: torch.Tensor, cfg: AdjointConfig) -> np.ndarray:
    """[n_sets, 9] float64 host rows in PARAM_KEYS order from theta [n_sets, 8]."""
    th = theta.detach().to("cpu", torch.float64).numpy()
    if th.ndim != 2 or th.shape[1] != len(GRAD_KEYS):
        raise ValueError("theta must be [n_sets, 8] = (U0, a, D, d2, q, c, gamma0, F0)")
    rows = np.empty((th.shape[0], len(PARAM_KEYS)), dtype=np.float64)
    col = {k: i for i, k in enumerate(PARAM_KEYS)}
    base = dict(BASE_PARAMS, **cfg.fixed)
    for k in PARAM_KEYS:
        rows[:, col[k]] = base[k]
    for j, k in enumerate(GRAD_KEYS):
        rows[:, col[k]] = th[:, j]
    return np.ascontiguousarray(rows)


def workspace(n_sets: int, cfg: AdjointConfig, device="cuda") -> torch.Tensor:
    nbytes = int(_lib.load().abp_adjoint_workspace_bytes(n_sets, cfg.n, cfg.steps, cfg.ckpt))
    if nbytes == 0:
        raise ValueError("invalid adjoint sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def forward(rows: np.ndarray, cfg: AdjointConfig, ws: torch.Tensor, stream=None) -> torch.Tensor:
    n_sets = rows.shape[0]
    loss = torch.empty(n_sets, dtype=torch.float64, device=ws.device)
    c = cfg.abi()
    check(_lib.load().abp_adjoint(0, n_sets, rows.ctypes.data, cfg.n, ctypes.byref(c),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                  ctypes.c_void_p(loss.data_ptr()), None, None, None,
                                  _stream(stream)), "abp_adjoint(forward)")
    return loss


def backward(rows: np.ndarray, cfg: AdjointConfig, ws: torch.Tensor, gloss: torch.Tensor,
             per_particle: bool = False, stream=None):
    n_sets = rows.shape[0]
    gloss = gloss.detach().to(ws.device, torch.float64).contiguous()
    ng = len(GRAD_KEYS)
    grad = torch.empty((n_sets, ng), dtype=torch.float64, device=ws.device)
    gp = (torch.empty((n_sets, cfg.n, ng), dtype=torch.float64, device=ws.device)
          if per_particle else None)
    c = cfg.abi()
    check(_lib.load().abp_adjoint(1, n_sets, rows.ctypes.data, cfg.n, ctypes.byref(c),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), None,
                                  ctypes.c_void_p(gloss.data_ptr()),
                                  ctypes.c_void_p(grad.data_ptr()),
                                  None if gp is None else ctypes.c_void_p(gp.data_ptr()),
                                  _stream(stream)), "abp_adjoint(backward)")
    return (grad, gp) if per_particle else grad


class MeanVelocity(torch.autograd.Function):
    """L = MeanVelocity.apply(theta, cfg): theta [n_sets, 8] -> L [n_sets] (float64, cuda)."""

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
