"""torch.autograd.Function over the FLUX5 forward and adjoint kernels."""

from __future__ import annotations

import torch


class EdgeFluxFn(torch.autograd.Function):
    """r = flux(q) on a Plan; backward runs the adjoint kernel on the same
    partition.  Geometry is a plan constant and gets no gradient."""

    @staticmethod
    def forward(ctx, q, plan):
        q = q.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(q)
        return plan.forward(q)

    @staticmethod
    def backward(ctx, g_r):
        (q,) = ctx.saved_tensors
        return ctx.plan.backward(q, g_r.contiguous()), None


def edge_flux(q, plan):
    return EdgeFluxFn.apply(q, plan)
