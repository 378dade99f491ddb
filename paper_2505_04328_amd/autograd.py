"""J(u) as a torch.autograd.Function whose backward is the hand-written adjoint.

forward:  jd_forward on the engine (trajectory or checkpoints kept in the
          engine's buffer), returns the Monte Carlo cost J (0-d FP64 tensor).
backward: jd_adjoint on the same (u, iteration word) -- in the recompute mode
          each checkpoint segment is regenerated with the same counters -- and
          returns grad_J * dJ/du = grad_J * dt * g (the Euclidean gradient of
          the discrete functional; g is the L2(0,T) representative the ABI
          returns, Section 4, eq. definition_Gradient).

The engine holds one trajectory buffer: if another forward on the same engine
ran between this forward and its backward, the backward first re-runs this
forward (same u, same counters, so bit-identical) before sweeping back.
"""
from __future__ import annotations

import torch

from .binding import Engine


class JdCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, engine: Engine, it: int):
        J = engine.forward(u.detach(), it=it)
        engine._generation = getattr(engine, "_generation", 0) + 1
        ctx.engine = engine
        ctx.it = it
        ctx.generation = engine._generation
        ctx.save_for_backward(u.detach())
        return J

    @staticmethod
    def backward(ctx, grad_J):
        (u,) = ctx.saved_tensors
        eng = ctx.engine
        if getattr(eng, "_generation", None) != ctx.generation:
            eng.forward(u, it=ctx.it)
            eng._generation += 1
        g = eng.adjoint(u, it=ctx.it)
        grad_u = (grad_J * eng.p.dt) * g
        return grad_u.to(u.dtype), None, None


def jd_cost(u: torch.Tensor, engine: Engine, it: int = 0) -> torch.Tensor:
    """Differentiable Monte Carlo cost J(u) for control u (N x d, FP64 on the
    engine's device) under iteration word `it`."""
    return JdCost.apply(u, engine, it)
