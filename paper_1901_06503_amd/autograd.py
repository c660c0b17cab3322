"""torch.autograd bridge: the forward operator A = X W_T as a differentiable op.

forward  g = A h        (ffpat_forward)
backward dh = A^T dg    (ffpat_adjoint, the exact transpose of the discrete A)

A is linear in h, so the backward needs no saved tensors; the gradient with
respect to the sound speed c is not provided (c lives in the plan).
"""
from __future__ import annotations

import torch


class XWFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, plan):
        ctx.plan = plan
        return plan.forward(h.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.adjoint(grad_g.contiguous()), None


def xw(plan, h):
    """g = X W_T h with autograd support (backward = W_T^T X^T)."""
    return XWFunction.apply(h, plan)


class XW(torch.nn.Module):
    """Module form of the forward operator for use inside larger torch models."""

    def __init__(self, plan):
        super().__init__()
        self.plan = plan

    def forward(self, h):
        return xw(self.plan, h)
