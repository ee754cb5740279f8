"""torch.autograd.Function over the finite-time flow: forward = rd_step with
checkpoints, backward = rd_vjp (recomputation between checkpoints)."""
from __future__ import annotations

import dataclasses

import torch

from . import _binding as B


class RDFlow(torch.autograd.Function):
    """(u0, v0, ...) -> state after prob.nsteps steps; differentiable."""

    @staticmethod
    def forward(ctx, prob: B.Problem, *fields):
        p = dataclasses.replace(prob)
        if p.checkpoint_every <= 0:
            p.checkpoint_every = 64
        z = [f.detach().contiguous().clone() for f in fields]
        nck = B.checkpoint_count(p)
        ck = torch.empty(max(nck, 1) * p.nfields * p.cells, dtype=torch.float64,
                         device=z[0].device)
        B.step(p, z, ck)
        ctx.save_for_backward(ck)
        ctx.prob = p
        return tuple(z)

    @staticmethod
    def backward(ctx, *grads):
        (ck,) = ctx.saved_tensors
        p = ctx.prob
        lam = [torch.zeros(p.shape, dtype=torch.float64, device=ck.device) if g is None
               else g.detach().contiguous().clone() for g in grads]
        B.vjp(p, ck, lam)
        return (None, *lam)


def flow(prob: B.Problem, *fields):
    """Differentiable finite-time flow (see RDFlow)."""
    return RDFlow.apply(prob, *fields)
