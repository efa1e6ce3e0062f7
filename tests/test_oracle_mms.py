"""Manufactured-solution pin of the oracle's discretisation (second-order L2 error).

A smooth divergence-free velocity that vanishes with its gradient on the walls,
a smooth pressure and temperature are inserted into Eqs. BoussDimless-a..c; the
resulting forcing enters the oracle's Galerkin and stabilised residuals.  The
discrete solution on n^3 grids must converge to the exact fields at second order
in the L2 norm for velocity and temperature (trilinear elements).  Pressure is
reported only.
"""
import numpy as np
import pytest
import sympy as sy

import oracle
from oracle import solve as osolve
from paper_1508_04596_amd import inputs

PR, GR = 1.0, 100.0
EG = (0.0, 0.0, -1.0)


def _exact():
    X, Y, Z = sy.symbols("x y z")
    pi = sy.pi
    psi = (sy.sin(pi * X) * sy.sin(pi * Y) * sy.sin(pi * Z)) ** 2
    u = [sy.diff(psi, Y) - sy.diff(psi, Z), sy.diff(psi, Z) - sy.diff(psi, X), sy.diff(psi, X) - sy.diff(psi, Y)]
    p = sy.cos(pi * X) * sy.cos(pi * Y) * sy.cos(pi * Z)
    T = sy.sin(pi * X) * sy.sin(pi * Y) * sy.sin(pi * Z)
    xs = (X, Y, Z)
    B = GR * PR ** 2
    fM = []
    for i in range(3):
        conv = sum(u[j] * sy.diff(u[i], xs[j]) for j in range(3))
        visc = sum(sy.diff(sy.diff(u[i], xs[j]) + sy.diff(u[j], xs[i]), xs[j]) for j in range(3))
        fM.append(conv - PR * visc + sy.diff(p, xs[i]) + B * EG[i] * T)  # alpha = 0 (gamma = 1)
    fT = sum(u[j] * sy.diff(T, xs[j]) for j in range(3)) - sum(sy.diff(T, xs[j], 2) for j in range(3))
    lam = lambda e: sy.lambdify((X, Y, Z), e, "numpy")
    return [lam(c) for c in u], lam(p), lam(T), [lam(c) for c in fM], lam(fT)


def _problem(n):
    p = inputs.tiny_problem(n, n, n, Gr=GR)
    p.Pr, p.eg = PR, EG
    p.gamma[:] = 1.0
    p.s[:] = 0.0
    return p


def _l2_errors(p, x, uex, pex, Tex):
    """L2 errors of u, T and mean-free p with a 3x3x3 Gauss rule per element."""
    q = np.sqrt(3.0 / 5.0)
    pts = np.array([-q, 0.0, q])
    wts = np.array([5.0, 8.0, 5.0]) / 9.0
    xs = x.reshape(p.nz + 1, p.ny + 1, p.nx + 1, 5)
    errs = {"u": 0.0, "T": 0.0}
    pvals, pex_vals, wv = [], [], []
    for gz, wz in zip(pts, wts):
        for gy, wy in zip(pts, wts):
            for gx, wx in zip(pts, wts):
                w = wx * wy * wz * (p.h / 2) ** 3
                val = 0.0
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    Na = (1 + (2 * ax - 1) * gx) * (1 + (2 * ay - 1) * gy) * (1 + (2 * az - 1) * gz) / 8
                    val = val + Na * xs[az:az + p.nz, ay:ay + p.ny, ax:ax + p.nx, :]
                K, J, I = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
                X = (I + 0.5 * (1 + gx)) * p.h
                Y = (J + 0.5 * (1 + gy)) * p.h
                Z = (K + 0.5 * (1 + gz)) * p.h
                for i in range(3):
                    errs["u"] += np.sum(w * (val[..., i] - uex[i](X, Y, Z)) ** 2)
                errs["T"] += np.sum(w * (val[..., 4] - Tex(X, Y, Z)) ** 2)
                pvals.append(val[..., 3])
                pex_vals.append(pex(X, Y, Z))
                wv.append(w)
    P = np.array(pvals)
    PE = np.array(pex_vals)
    W = np.array(wv)[:, None, None, None]
    P = P - np.sum(W * P) / np.sum(W * np.ones_like(P))
    PE = PE - np.sum(W * PE) / np.sum(W * np.ones_like(PE))
    errs["p"] = np.sum(W * (P - PE) ** 2)
    return {k: float(np.sqrt(v)) for k, v in errs.items()}


def test_manufactured_solution_converges_at_second_order():
    uex, pex, Tex, fM, fT = _exact()
    errs = []
    for n in (4, 8, 16):
        p = _problem(n)
        xg = oracle.gauss_points(p)  # [n_el, 8, 3]
        forc = np.empty((p.n_el, 8, 4))
        X, Y, Z = xg[..., 0], xg[..., 1], xg[..., 2]
        for i in range(3):
            forc[..., i] = fM[i](X, Y, Z)
        forc[..., 3] = fT(X, Y, Z)
        x0 = np.zeros(p.n_dof)
        x0[3] = pex(0.0, 0.0, 0.0)  # pinned pressure value
        x, it, rr = osolve.newton(p, x0=x0, rtol=1e-12, forcing=forc.reshape(-1))
        assert rr <= 1e-12
        errs.append(_l2_errors(p, x, uex, pex, Tex))
    ou = [np.log2(errs[k]["u"] / errs[k + 1]["u"]) for k in range(2)]
    oT = [np.log2(errs[k]["T"] / errs[k + 1]["T"]) for k in range(2)]
    print("L2 errors", errs, "orders u", ou, "T", oT)
    assert ou[-1] > 1.8 and oT[-1] > 1.8
    assert errs[-1]["u"] < errs[0]["u"] and errs[-1]["T"] < errs[0]["T"]
