"""torch.autograd wrappers around the library's transforms.

NfftFunction       f = A~ fhat with A~ = B(x) F D (the NFFT); gradients with respect to the
                   coefficients (the adjoint NFFT) and to the node positions (window derivative).
InfftApplyFunction fcheck = D^* F^* B_opt^* f (the modified adjoint NFFT, (3.32)); gradient with
                   respect to f is B_opt F D applied to the incoming gradient (Remark 3.24); when
                   the nodes x are passed, also the gradient with respect to x through B_opt(x)
                   (implicit differentiation of the local problems of Algorithm 3.17).

The modified adjoint runs on its own plan (loading new nodes into a plan invalidates its B_opt),
whose B_opt must have been computed for the nodes passed as x.
Gradients follow PyTorch's convention for complex tensors (dL/dx = sum Re(conj(g) df/dx)).
"""
from __future__ import annotations

import torch

from ._lib import InfftError
from .plan import NfftBatchPlan, NfftPlan


class NfftFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan):
        plan.set_nodes(x.detach())
        ctx.plan = plan
        ctx.save_for_backward(fhat)
        f = plan.trafo(fhat)
        ctx.trafo = (getattr(plan, "_trafo_seq", None), getattr(plan, "_slot", 0))
        return f

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        (fhat,) = ctx.saved_tensors
        plan = ctx.plan
        g = grad_f.contiguous()
        gx = None
        if ctx.needs_input_grad[1]:
            # the node gradient first: if this forward's trafo was the plan's last and its slot is
            # current, the grid may still hold F D fhat (the library checks that no other call
            # wrote it since); otherwise it is recomputed from fhat
            if not isinstance(plan, NfftBatchPlan) and ctx.trafo[0] is not None and \
                    ctx.trafo == (getattr(plan, "_trafo_seq", None), getattr(plan, "_slot", 0)):
                try:
                    gx = plan.grad_x_after_trafo(g)
                except InfftError:
                    gx = None
            if gx is None:
                gx = plan.grad_x(fhat, g)
        gfh = plan.adjoint(g) if ctx.needs_input_grad[0] else None
        return gfh, gx, None


class InfftApplyFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, plan: NfftPlan, x=None):
        ctx.plan = plan
        ctx.with_x = x is not None
        ctx.save_for_backward(f)
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_h: torch.Tensor):
        (f,) = ctx.saved_tensors
        g = grad_h.contiguous()
        gf = ctx.plan.apply_adjoint(g) if ctx.needs_input_grad[0] else None
        gx = None
        if ctx.with_x and ctx.needs_input_grad[2]:
            gx = ctx.plan.grad_x_bopt(f.detach().contiguous(), g)
        return gf, None, gx


def nfft(fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan) -> torch.Tensor:
    """Differentiable NFFT (nodes x are loaded into `plan`)."""
    return NfftFunction.apply(fhat, x, plan)


def infft(f: torch.Tensor, plan: NfftPlan, x: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable modified adjoint NFFT with the plan's B_opt (call plan.precompute_B first).
    Pass the plan's nodes as x to differentiate through B_opt(x) as well."""
    return InfftApplyFunction.apply(f, plan, x)
