"""torch.autograd.Function over the C ABI.

rho = solve(q, logD, logmua, plan) is differentiable with respect to all
three inputs, in reverse mode (backward = dmgs_vjp: the transposed
V-cycles, then the coefficient gradients) and in forward mode (jvp =
dmgs_jvp).  Only the forward solution rho is saved for the backward pass:
the analytic adjoint needs no per-level iterates, so the memory of a
forward + backward pair is the plan's hierarchy plus a handful of fields.

The plan keeps the coefficient hierarchy of the last coefficients it was
given; every call records which coefficients the plan holds, and the
backward / forward-mode pass re-sets them if another solve on the same plan
changed them in between.
"""
import itertools

import torch

from .solver import Options, Plan

_token = itertools.count(1)


def _set_coefficients(plan, logD, logmua, token):
    if getattr(plan, "_coef_token", None) != token:
        plan.set_log_coefficients(logD, logmua)
        plan._coef_token = token


class DMGSSolve(torch.autograd.Function):
    """rho = S(q; log D, log mua) on a resident plan."""

    @staticmethod
    def forward(q, logD, logmua, plan):
        token = next(_token)
        _set_coefficients(plan, logD.detach().contiguous(), logmua.detach().contiguous(), token)
        rho, info = plan.forward(q.detach().contiguous())
        plan._last_forward = (token, info)
        return rho

    @staticmethod
    def setup_context(ctx, inputs, output):
        q, logD, logmua, plan = inputs
        ctx.plan = plan
        ctx.token, ctx.info = plan._last_forward
        ctx.save_for_backward(output, logD, logmua)
        ctx.save_for_forward(output, logD, logmua)

    @staticmethod
    def backward(ctx, rhobar):
        rho, logD, logmua = ctx.saved_tensors
        plan = ctx.plan
        _set_coefficients(plan, logD.detach().contiguous(), logmua.detach().contiguous(), ctx.token)
        need_coef = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        (qbar, gD, gmu), _ = plan.vjp(rho.detach(), rhobar.contiguous(), coef_grads=need_coef)
        return (qbar if ctx.needs_input_grad[0] else None,
                gD if ctx.needs_input_grad[1] else None,
                gmu if ctx.needs_input_grad[2] else None,
                None)

    @staticmethod
    def jvp(ctx, dq, dlogD, dlogmua, _plan_tangent):
        rho, logD, logmua = ctx.saved_tensors
        plan = ctx.plan
        _set_coefficients(plan, logD.detach().contiguous(), logmua.detach().contiguous(), ctx.token)
        c = lambda t: None if t is None else t.contiguous()
        drho, _ = plan.jvp(rho.detach(), c(dq), c(dlogD), c(dlogmua))
        return drho


def solve(q, logD, logmua, plan):
    """Differentiable forward solve on `plan` (see DMGSSolve)."""
    return DMGSSolve.apply(q, logD, logmua, plan)


class DMGSSolveUnrolled(torch.autograd.Function):
    """rho = S_n(q; log D, log mua), the fixed-cycle map of a float64 3D plan
    with fixed_cycles = n, differentiated exactly through every step
    (backward = dmgs_vjp_unrolled, which recomputes the cycles from q, so q
    is saved instead of per-level iterates).  Reverse mode only."""

    @staticmethod
    def forward(q, logD, logmua, plan):
        token = next(_token)
        _set_coefficients(plan, logD.detach().contiguous(), logmua.detach().contiguous(), token)
        rho, info = plan.forward(q.detach().contiguous())
        plan._last_forward = (token, info)
        return rho

    @staticmethod
    def setup_context(ctx, inputs, output):
        q, logD, logmua, plan = inputs
        ctx.plan = plan
        ctx.token, ctx.info = plan._last_forward
        ctx.save_for_backward(q, logD, logmua)

    @staticmethod
    def backward(ctx, rhobar):
        q, logD, logmua = ctx.saved_tensors
        plan = ctx.plan
        _set_coefficients(plan, logD.detach().contiguous(), logmua.detach().contiguous(), ctx.token)
        need_coef = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        (_, (qbar, gD, gmu)), _ = plan.vjp_unrolled(q.detach().contiguous(), rhobar.contiguous(), coef_grads=need_coef)
        return (qbar if ctx.needs_input_grad[0] else None,
                gD if ctx.needs_input_grad[1] else None,
                gmu if ctx.needs_input_grad[2] else None,
                None)


def solve_unrolled(q, logD, logmua, plan):
    """Forward solve on a fixed-cycle float64 3D `plan` whose backward is
    the unrolled adjoint (see DMGSSolveUnrolled)."""
    return DMGSSolveUnrolled.apply(q, logD, logmua, plan)


class Solver:
    """A plan plus the differentiable call, for one grid size."""

    def __init__(self, N, device=None, **opts):
        self.plan = Plan(Options(N, **opts), device=device)

    def __call__(self, q, logD, logmua):
        return solve(q, logD, logmua, self.plan)

    def close(self):
        self.plan.close()
