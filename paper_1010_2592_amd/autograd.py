"""torch.autograd.Function over the C-ABI: y = f(A) b (or sign(H) b) with
gradients for b, the PFE weights w_s, the shifts sigma_s and the gauge links.

forward calls ``mshift_bicgstabl`` (or ``pfe_sign_apply``); backward calls
``pfe_sign_backward`` with eta = grad_output, i.e. the gradient of a real loss
in PyTorch's convention dL/dRe + i dL/dIm.  a_scale is held constant.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from . import msb


@dataclass(frozen=True)
class FAConfig:
    dims: Sequence[int]
    mass: float
    mu: float
    bc_t: int
    a_scale: float
    l: int = 4
    tol: float = 1e-8
    max_outer: int = 2000
    pass_: int = 1
    mixed: bool = False
    sign: bool = False          # y = sign(H) b instead of f(A) b


class FA(torch.autograd.Function):
    """y = FA.apply(b, w, sigma, links, cfg); b (nrhs, 12, V) complex128 CUDA,
    w and sigma (N_s,) float64 (CPU), links (4, 3, 3, V) complex128 CUDA."""

    @staticmethod
    def forward(ctx, b, w, sigma, links, cfg: FAConfig):
        c = msb.Context(msb.Lattice(cfg.dims, cfg.mass, cfg.mu, cfg.bc_t), links.detach())
        wn = w.detach().cpu().numpy().astype(np.float64)
        sn = sigma.detach().cpu().numpy().astype(np.float64)
        flags = msb.MIXED if cfg.mixed else 0
        if cfg.sign:
            y, _ = c.pfe_sign_apply(b.detach(), cfg.a_scale, sn, wn, cfg.l, cfg.tol, cfg.max_outer,
                                    cfg.pass_, flags=flags)
        else:
            y, _, _ = c.mshift_bicgstabl(b.detach(), cfg.a_scale, sn, wn, cfg.l, cfg.tol, cfg.max_outer,
                                         cfg.pass_, flags=flags)
        c.close()
        ctx.save_for_backward(b, w, sigma, links)
        ctx.cfg = cfg
        return y

    @staticmethod
    def backward(ctx, gy):
        b, w, sigma, links = ctx.saved_tensors
        cfg = ctx.cfg
        c = msb.Context(msb.Lattice(cfg.dims, cfg.mass, cfg.mu, cfg.bc_t), links.detach())
        gb, gw, gs, gl, _ = c.pfe_sign_backward(
            b.detach(), gy.contiguous(), cfg.a_scale, sigma.detach().cpu().numpy(),
            w.detach().cpu().numpy(), cfg.l, cfg.tol, cfg.max_outer, mode=1 if cfg.sign else 0,
            flags=msb.MIXED if cfg.mixed else 0)
        c.close()
        return (gb, torch.from_numpy(gw).to(w.device, w.dtype), torch.from_numpy(gs).to(sigma.device, sigma.dtype),
                gl, None)
