"""torch.autograd wrapper: homogenized stress as a differentiable function of F.

forward  = rve_batch_solve (relaxation + boundary-reaction stress)
backward = rve_batch_vjp   (one adjoint conjugate-gradient solve per RVE on
                            the converged network)

The backward pass uses the state of the most recent solve of the batch, so a
second solve between forward and backward invalidates the gradient; the
function records the solve count and refuses such a backward.
"""
from __future__ import annotations

import torch


class RVEStress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, F, batch):
        sig, st = batch.solve(F)
        batch._solve_count = getattr(batch, "_solve_count", 0) + 1
        ctx.batch = batch
        ctx.count = batch._solve_count
        ctx.mark_non_differentiable(st)
        return sig, st

    @staticmethod
    def backward(ctx, g_sigma, g_status):
        b = ctx.batch
        if getattr(b, "_solve_count", 0) != ctx.count:
            raise RuntimeError("the batch was solved again after this forward pass; its adjoint state is gone")
        gF, st = b.vjp(g_sigma.contiguous())
        return gF, None


def rve_stress(F, batch):
    """sigma[R,3,3], status[R] = RVEStress.apply(F, batch)."""
    return RVEStress.apply(F, batch)
