"""torch.autograd.Function over the library's evaluation.

Forward (Eq. 1): one hawkes_eval with the log-likelihood and the
hyperparameter gradient -- the row pass, its finalisation and the integral
term.  Backward: the rate gradient of Eq. 4 is the library's column pass,
launched on the intensities the forward left in the plan
(hawkes_grad_theta_from_last); if the plan has evaluated anything else in
between, the backward runs a fresh hawkes_grad instead.  The hyperparameter
gradient comes from the forward's reductions.  No autograd graph is recorded
through the kernels: the backward is hand-written.
"""
from __future__ import annotations

import torch

from .hawkes import Plan

HYPER_NAMES = ("mu0", "tau_x", "tau_t", "theta0", "omega", "h")


class HawkesLoglik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, hyper: torch.Tensor, plan: Plan):
        if hyper.dtype != torch.float64 or hyper.shape != (6,):
            raise ValueError("hyper must be a float64 tensor of 6 values (mu0, tau_x, tau_t, theta0, omega, h)")
        hy = tuple(float(v) for v in hyper.detach().cpu())
        out = plan.eval(theta.detach(), hy, loglik=True, grad_hyper=True)
        ctx.plan = plan
        ctx.hyper = hy
        ctx.hyper_device = hyper.device
        ctx.epoch = plan.epoch()
        ctx.grad_hyper = out["grad_hyper"]
        ctx.save_for_backward(theta)
        return out["loglik"].reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (theta,) = ctx.saved_tensors
        g_theta = g_hyper = None
        if ctx.needs_input_grad[0]:
            r = ctx.plan.grad_theta_from_last(ctx.hyper, ctx.epoch)
            if r is None:  # the plan was used in between: evaluate afresh
                g = ctx.plan.eval(theta.detach(), ctx.hyper, loglik=False, grad_theta=True)["grad_theta"]
            else:
                g = r[0]
            g_theta = grad_out * g
        if ctx.needs_input_grad[1]:
            g_hyper = (grad_out * ctx.grad_hyper).to(ctx.hyper_device)
        return g_theta, g_hyper, None


def loglik(theta: torch.Tensor, hyper: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable log-likelihood (Eq. 1) of the plan's events at rates theta
    (float64 [n], caller order, on the plan's device) and hyperparameters hyper
    (float64 [6], any device)."""
    return HawkesLoglik.apply(theta, hyper, plan)
