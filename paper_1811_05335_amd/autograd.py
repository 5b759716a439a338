"""torch.autograd wrappers around the library's transforms.

NfftFunction       f = A~ fhat with A~ = B(x) F D (the NFFT); gradients with respect to the
                   coefficients (the adjoint NFFT) and to the node positions (window derivative).
InfftApplyFunction fcheck = D^* F^* B_opt^* f (the modified adjoint NFFT, (3.32)); gradient with
                   respect to f is B_opt F D applied to the incoming gradient (Remark 3.24); when
                   the nodes x are passed, also the gradient with respect to x through B_opt(x)
                   (implicit differentiation of the local problems of Algorithm 3.17).

The modified adjoint runs on its own plan (loading new nodes into a plan invalidates its B_opt),
whose B_opt must have been computed for the nodes passed as x.

A plan holds one node set at a time.  The NFFT's backward reloads the nodes of its own forward
when another forward has loaded different nodes into the plan since; the modified adjoint's
forward and backward raise if the plan's B_opt is not the one computed for its current nodes.
Gradients follow PyTorch's convention for complex tensors (dL/dx = sum Re(conj(g) df/dx)).
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import InfftError
from .plan import NfftBatchPlan, NfftPlan


class NfftFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan):
        xd = x.detach()
        plan.set_nodes(xd)
        ctx.plan = plan
        ctx.save_for_backward(fhat, xd)
        ctx.nodes_version = plan.nodes_version
        f = plan.trafo(fhat)
        ctx.trafo = (getattr(plan, "_trafo_seq", None), getattr(plan, "_slot", 0))
        return f

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        fhat, xd = ctx.saved_tensors
        plan = ctx.plan
        if plan.nodes_version != ctx.nodes_version:
            # another forward loaded other nodes into the plan since: reload this forward's
            plan.set_nodes(xd)
            ctx.nodes_version = plan.nodes_version
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
        _check_bopt(plan, x)
        ctx.plan = plan
        ctx.with_x = x is not None
        ctx.nodes_version = plan.nodes_version
        ctx.save_for_backward(f)
        return plan.apply(f)

    @staticmethod
    def backward(ctx, grad_h: torch.Tensor):
        (f,) = ctx.saved_tensors
        if ctx.plan.nodes_version != ctx.nodes_version or ctx.plan.bopt_version != ctx.nodes_version:
            raise InfftError(_lib.INFFT_ESTATE, "the plan's nodes or B_opt changed between the modified "
                             "adjoint's forward and its backward")
        g = grad_h.contiguous()
        gf = ctx.plan.apply_adjoint(g) if ctx.needs_input_grad[0] else None
        gx = None
        if ctx.with_x and ctx.needs_input_grad[2]:
            gx = ctx.plan.grad_x_bopt(f.detach().contiguous(), g)
        return gf, None, gx


def _check_bopt(plan: NfftPlan, x) -> None:
    if plan.bopt_version != plan.nodes_version:
        raise InfftError(_lib.INFFT_ESTATE, "the plan's B_opt was not computed for its current nodes "
                         "(call precompute_B after set_nodes)")
    if x is not None and x.data_ptr() != plan._x.data_ptr():
        xp = plan._x.reshape(x.shape) if plan._x.numel() == x.numel() else None
        if xp is None or not torch.equal(x.detach(), xp):
            raise InfftError(_lib.INFFT_EINVAL, "x is not the node set whose B_opt the plan holds")


def nfft(fhat: torch.Tensor, x: torch.Tensor, plan: NfftPlan) -> torch.Tensor:
    """Differentiable NFFT (nodes x are loaded into `plan`)."""
    return NfftFunction.apply(fhat, x, plan)


def infft(f: torch.Tensor, plan: NfftPlan, x: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable modified adjoint NFFT with the plan's B_opt (call plan.precompute_B first).
    Pass the plan's nodes as x to differentiate through B_opt(x) as well."""
    return InfftApplyFunction.apply(f, plan, x)
