"""``torch.autograd.Function`` wrappers of the state solve and its adjoint.

``StateSolve``  gamma -> x*: forward runs ``newton_solve``; backward solves
    J(x*)^T lambda = x_bar with ``fe_adjoint_solve`` and returns
    gamma_bar = -lambda^T dR/dgamma (``fe_dR_dgamma``), since R(x*(gamma), gamma) = 0
    gives dx*/dgamma = -J^{-1} dR/dgamma.
``Compliance``  gamma -> f = integral over the source of s T(x*(gamma)) (the
    thermal-compliance objective of Sec. "Optimisation problem"); backward solves
    J^T lambda = df/dx and returns -f_bar lambda^T dR/dgamma (consistent adjoint
    sensitivities, appendix "Stabilisation parameters").

Element quantities are recomputed by the kernels in the backward pass; only
the converged state is kept between forward and backward.
"""
from __future__ import annotations

import torch

from . import fe


class StateSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, prob, s, opts=None, adj_opts=None, x0=None):
        x = torch.zeros(prob.n_dof, dtype=torch.float64, device=gamma.device) if x0 is None \
            else x0.detach().clone()
        rep = fe.newton_solve(prob, gamma.detach().contiguous(), s, x, opts)
        ctx.prob, ctx.adj_opts, ctx.report = prob, adj_opts, rep
        ctx.save_for_backward(gamma.detach(), x, s)
        return x

    @staticmethod
    def backward(ctx, x_bar):
        gamma, x, s = ctx.saved_tensors
        lam, _ = fe.fe_adjoint_solve(ctx.prob, x, gamma, s, x_bar.contiguous(), opts=ctx.adj_opts)
        g = fe.fe_dR_dgamma(ctx.prob, x, gamma, s, lam)
        return -g, None, None, None, None, None


class Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, prob, s, opts=None, adj_opts=None, x0=None):
        x = torch.zeros(prob.n_dof, dtype=torch.float64, device=gamma.device) if x0 is None \
            else x0.detach().clone()
        rep = fe.newton_solve(prob, gamma.detach().contiguous(), s, x, opts)
        dfdx = torch.empty_like(x)
        f = fe.fe_compliance(prob, x, s, dfdx)
        ctx.prob, ctx.adj_opts, ctx.report, ctx.x = prob, adj_opts, rep, x
        ctx.save_for_backward(gamma.detach(), x, s, dfdx)
        return torch.tensor(f, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, f_bar):
        gamma, x, s, dfdx = ctx.saved_tensors
        lam, _ = fe.fe_adjoint_solve(ctx.prob, x, gamma, s, dfdx, opts=ctx.adj_opts)
        g = fe.fe_dR_dgamma(ctx.prob, x, gamma, s, lam)
        return -f_bar * g, None, None, None, None, None


def state_solve(gamma, prob, s, opts=None, adj_opts=None, x0=None):
    return StateSolve.apply(gamma, prob, s, opts, adj_opts, x0)


def compliance(gamma, prob, s, opts=None, adj_opts=None, x0=None):
    return Compliance.apply(gamma, prob, s, opts, adj_opts, x0)
