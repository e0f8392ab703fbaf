"""torch.autograd wrapper: homogenized stress as a differentiable function of F.

forward  = rve_batch_solve (relaxation + boundary-reaction stress)
backward = rve_batch_vjp   (one adjoint conjugate-gradient solve per RVE on
                            the converged network)

The backward pass uses the state the batch holds when it runs.  The library
counts every change of that state (solve, state import, option change) in
rve_batch_generation; forward records the count after its solve and backward
refuses to run when it has changed, so a VJP is never taken at another
state than the one forward returned.
"""
from __future__ import annotations

import torch


class RVEStress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, F, batch):
        sig, st = batch.solve(F)
        ctx.batch = batch
        ctx.generation = batch.generation()
        ctx.mark_non_differentiable(st)
        return sig, st

    @staticmethod
    def backward(ctx, g_sigma, g_status):
        b = ctx.batch
        if b.generation() != ctx.generation:
            raise RuntimeError("the batch's state changed after this forward pass (solve, import or option "
                               "change); its adjoint state is gone")
        gF, st = b.vjp(g_sigma.contiguous())
        return gF, None


def rve_stress(F, batch):
    """sigma[R,3,3], status[R] = RVEStress.apply(F, batch)."""
    return RVEStress.apply(F, batch)
