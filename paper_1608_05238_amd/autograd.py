"""The radiance Monte Carlo as a differentiable PyTorch function.

`absorbed_energy(mua, mus, ...)` returns the absorbed energy density
H = mua Phi (Sec. 2) from the forward Monte Carlo; its backward is the
adjoint Monte Carlo and the harmonic-product gradient kernels (Sec. 4-6):
for an upstream gradient G = dL/dH the adjoint source is q* = -mua G / A
(`mc_adjoint_source`), the adjoint field comes from `mc_adjoint`, and
`mc_gradient_h` forms dL/dmua and dL/dmus.  For L = eps of eq.
error_function3 this is exactly the gradient of Sec. 5.

Every step runs in librmc.so; this module only sequences the calls.  The
forward and adjoint runs use counter-based random numbers, so a fixed seed
gives common random numbers across evaluations (what finite differences and
line searches of a Monte Carlo functional need).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import rmc


@dataclass
class MCConfig:
    """Packets per forward run, harmonic order N, seed (stream tags 0 and 1
    for the forward and adjoint runs) and packets per adjoint run (default:
    as many as the forward run)."""
    n_packets: int
    n_harm: int = 16
    seed: int = 0
    n_adjoint: Optional[int] = None


class _AbsorbedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mua, mus, g, dx, sources, cfg: MCConfig):
        med = rmc.Medium(mua.detach().to(torch.float32).contiguous(), mus.detach().to(torch.float32).contiguous(),
                         g.detach().to(torch.float32).contiguous(), float(dx))
        fwd, _ = rmc.mc_forward(med, sources, rmc.make_run(cfg.n_packets, cfg.n_harm, seed=cfg.seed), ledger=False)
        h = rmc.mc_absorbed(med, fwd)
        ctx.save_for_backward(fwd)
        ctx.med, ctx.cfg = med, cfg
        ctx.dtypes = (mua.dtype, mus.dtype)
        return h

    @staticmethod
    def backward(ctx, grad_h):
        (fwd,) = ctx.saved_tensors
        med, cfg = ctx.med, ctx.cfg
        grad_h = grad_h.to(torch.float64).contiguous()
        q = rmc.mc_adjoint_source(med, grad_h)
        n_adj = cfg.n_adjoint or cfg.n_packets
        adj, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)],
                                rmc.make_run(n_adj, cfg.n_harm, seed=cfg.seed, stream_tag=1), ledger=False)
        dmua, dmus = rmc.mc_gradient_h(med, cfg.n_harm, fwd, adj, grad_h)
        ga = dmua.to(ctx.dtypes[0]) if ctx.needs_input_grad[0] else None
        gs = dmus.to(ctx.dtypes[1]) if ctx.needs_input_grad[1] else None
        return ga, gs, None, None, None, None


def absorbed_energy(mua: torch.Tensor, mus: torch.Tensor, g: torch.Tensor, dx: float, sources: Sequence,
                    cfg: MCConfig) -> torch.Tensor:
    """H = mua Phi (float64 [nz][nx]) from the forward Monte Carlo; differentiable
    in mua and mus through the adjoint Monte Carlo."""
    return _AbsorbedEnergy.apply(mua, mus, g, dx, sources, cfg)


def error_functional(h: torch.Tensor, hmeas: torch.Tensor, dx: float) -> torch.Tensor:
    """eps = (A/2) sum (Hmeas - H)^2 over pixels (eq. error_function3, A = dx^2)."""
    return 0.5 * dx * dx * ((hmeas - h) ** 2).sum()
