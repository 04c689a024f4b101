"""torch.autograd.Function over the butterfly apply.

The operator is C-linear, u = K f.  For a real loss, PyTorch's convention for
complex inputs makes the gradient with respect to f equal to K^H times the
gradient with respect to u, so the backward pass is one call of the
library's adjoint kernels (tb_apply_adjoint).
"""
from __future__ import annotations

import torch


class TBApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan, dtype="c64"):
        ctx.plan = plan
        ctx.dtype = dtype
        return plan.apply(f, dtype=dtype)

    @staticmethod
    def backward(ctx, grad_u):
        grad_f = ctx.plan.apply_adjoint(grad_u.contiguous(), dtype=ctx.dtype)
        return grad_f, None, None
