"""Differentiable products: torch.autograd.Function wrappers of the C ABI.

``bttb_matvec(plan, m)`` computes d = G m with ``bttb_forward``; its backward
is ``bttb_transpose`` (the exact adjoint: for a linear map the gradient of
<g, G m> with respect to m is G^T g), which is what an inverse problem needs
(the paper's transpose product, Sec. 3, used in the inverse problem of its
conclusions).  ``bttb_rmatvec(plan, r)`` is the reverse pair.  Both run on
torch's current stream; gradients are produced by the same hand-written
kernels as the products.
"""
from __future__ import annotations

import torch


class BTTBForward(torch.autograd.Function):
    """d = G m; backward: grad_m = G^T grad_d."""

    @staticmethod
    def forward(ctx, m, plan):
        ctx.plan = plan
        return plan.forward(m.contiguous())

    @staticmethod
    def backward(ctx, grad_d):
        return ctx.plan.transpose(grad_d.contiguous()), None


class BTTBTranspose(torch.autograd.Function):
    """m = G^T r; backward: grad_r = G grad_m."""

    @staticmethod
    def forward(ctx, r, plan):
        ctx.plan = plan
        return plan.transpose(r.contiguous())

    @staticmethod
    def backward(ctx, grad_m):
        return ctx.plan.forward(grad_m.contiguous()), None


def bttb_matvec(plan, m: torch.Tensor) -> torch.Tensor:
    """Differentiable d = G m for m of shape [..., nz, ny, nx]."""
    return BTTBForward.apply(m, plan)


def bttb_rmatvec(plan, r: torch.Tensor) -> torch.Tensor:
    """Differentiable G^T r for r of shape [..., sy, sx]."""
    return BTTBTranspose.apply(r, plan)
