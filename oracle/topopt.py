"""Oracle design-loop evaluation (test infrastructure only): objective,
volume constraint and their gradients with respect to the design values, by
the chain blend -> PDE filter -> blend -> Newton -> thermal compliance ->
adjoint -> lambda^T dR/dgamma -> filter transpose (Sec. "Optimisation
problem"), with exact sparse solves."""
from __future__ import annotations

import numpy as np

from . import solve as osolve
from .filter import Filter


def physical_design(p, filt: Filter, rho, design, gamma_fixed):
    gin = np.where(design, rho, gamma_fixed)
    return np.where(design, filt.apply(gin), gamma_fixed)


def evaluate(p, filt: Filter, rho, design, gamma_fixed, vf, rtol=1e-12, grads=True):
    gt = physical_design(p, filt, rho, design, gamma_fixed)
    x, _, rel = osolve.newton(p, gamma=gt, mask="solve", rtol=rtol)
    f = osolve.compliance(p, x)
    nd = int(design.sum())
    g = float(np.sum(np.where(design, 1.0 - gt, 0.0)) / nd - vf)
    if not grads:
        return f, g, None, None, x
    _, dfdg = osolve.adjoint_gradient(p, x, gamma=gt, mask="solve")
    df = np.where(design, filt.apply_transpose(np.where(design, dfdg, 0.0)), 0.0)
    dg = np.where(design, filt.apply_transpose(np.where(design, -1.0 / nd, 0.0)), 0.0)
    return f, g, df, dg, x
