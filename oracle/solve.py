"""Oracle solves (test infrastructure only).

* ``assemble`` -- the global Jacobian as a scipy sparse matrix, summed from the
  oracle's element Jacobians, with prescribed DOFs eliminated symmetrically
  (prescribed rows and columns replaced by the identity).
* ``newton`` -- the damped Newton method of Sec. "Solving the non-linear system":
  each step solves J delta = -R exactly (sparse direct solve), then picks the
  damping factor as the minimiser of a quadratic fitted to the squared L2 norm
  of the residual at 0, 1/2 and 1 times the step; it stops when the L2 norm of
  the residual has fallen by ``rtol`` relative to the initial one.
* ``adjoint_gradient`` -- thermal compliance f = integral over the source region
  of s T (Sec. "Optimisation problem"), its adjoint J^T lambda = df/dx and
  df/dgamma = -lambda^T dR/dgamma.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import core

NF = 5


def element_dofs(p) -> np.ndarray:
    """Global DOF numbers [n_el, 40] of every element (row = 5*local node + field)."""
    i = np.arange(p.nx)
    j = np.arange(p.ny)
    k = np.arange(p.nz)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    I, J, K = I.reshape(-1), J.reshape(-1), K.reshape(-1)
    out = np.empty((p.n_el, 40), dtype=np.int64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        n = (I + ax) + (p.nx + 1) * ((J + ay) + (p.ny + 1) * (K + az))
        for f in range(NF):
            out[:, NF * a + f] = NF * n + f
    return out


def assemble(p, x, gamma=None, mask="solve", forcing=None, s=None) -> sp.csr_matrix:
    Ke = core.element_jacobians(p, x, gamma=gamma, forcing=forcing, s=s)
    dofs = element_dofs(p)
    rows = np.repeat(dofs, 40, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 40)).reshape(-1)
    J = sp.csr_matrix((Ke.reshape(-1), (rows, cols)), shape=(p.n_dof, p.n_dof))
    m = _mask(p, mask)
    if m is not None:
        free = sp.diags((~m).astype(np.float64))
        fixed = sp.diags(m.astype(np.float64))
        J = (free @ J @ free + fixed).tocsr()
    return J


def _mask(p, mask):
    if mask is None:
        return None
    if isinstance(mask, str):
        return (p.mask_walls if mask == "walls" else p.mask_solve).astype(bool)
    return np.asarray(mask).astype(bool)


def line_search_lambda(phi0: float, phi_half: float, phi1: float, lam_min: float = 0.05) -> float:
    """Minimiser of the quadratic through (0, phi0), (1/2, phi_half), (1, phi1)."""
    c2 = 2.0 * (phi1 - 2.0 * phi_half + phi0)
    c1 = phi1 - phi0 - c2
    if c2 > 0.0:
        return float(min(1.0, max(lam_min, -c1 / (2.0 * c2))))
    return 0.5 if phi_half < phi1 else 1.0


def newton(p, x0=None, gamma=None, mask="solve", rtol=1e-8, max_newton=50, forcing=None,
           s=None, history=None):
    m = _mask(p, mask)
    x = np.zeros(p.n_dof) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    R = core.residual(p, x, gamma=gamma, mask=m.astype(np.uint8), forcing=forcing, s=s)
    r0 = np.linalg.norm(R)
    if history is not None:
        history.append(r0)
    it = 0
    while np.linalg.norm(R) > rtol * r0 and it < max_newton:
        J = assemble(p, x, gamma=gamma, mask=m, forcing=forcing, s=s)
        delta = spla.spsolve(J.tocsc(), -R)
        def phi(lam):
            Rl = core.residual(p, x + lam * delta, gamma=gamma, mask=m.astype(np.uint8),
                               forcing=forcing, s=s)
            return float(Rl @ Rl), Rl
        phi0 = float(R @ R)
        ph, Rh = phi(0.5)
        p1, R1 = phi(1.0)
        lam = line_search_lambda(phi0, ph, p1)
        if lam == 1.0:
            R = R1
        elif lam == 0.5:
            R = Rh
        else:
            _, R = phi(lam)
        x = x + lam * delta
        it += 1
        if history is not None:
            history.append(np.linalg.norm(R))
    return x, it, float(np.linalg.norm(R) / r0 if r0 > 0 else 0.0)


def compliance(p, x, s=None) -> float:
    """f = sum over source elements of s_e (h^3/8) sum_a T_a (exact integral of s T)."""
    ss = p.s if s is None else s
    dofs = element_dofs(p)
    T = x[dofs[:, 4::NF]]  # [n_el, 8]
    return float(np.sum(ss * (p.h ** 3 / 8.0) * T.sum(axis=1)))


def compliance_gradient_x(p, mask="solve", s=None) -> np.ndarray:
    ss = p.s if s is None else s
    dofs = element_dofs(p)
    c = np.zeros(p.n_dof)
    np.add.at(c, dofs[:, 4::NF].reshape(-1), np.repeat(ss * p.h ** 3 / 8.0, 8))
    m = _mask(p, mask)
    if m is not None:
        c[m] = 0.0
    return c


def adjoint_gradient(p, x, gamma=None, mask="solve"):
    """(lambda, df/dgamma) at a converged state x (exact sparse adjoint solve)."""
    m = _mask(p, mask)
    J = assemble(p, x, gamma=gamma, mask=m)
    c = compliance_gradient_x(p, mask=m)
    lam = spla.spsolve(J.T.tocsc(), c)
    g = core.dR_dgamma(p, x, lam, gamma=gamma, mask=m.astype(np.uint8))
    return lam, -g
