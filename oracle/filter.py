"""Oracle PDE (Helmholtz) density filter (test infrastructure only).

Sec. "Optimisation problem": the design field is regularised with a PDE-based
density filter.  The filter equation itself is in the cited references, which
are not part of the paper's text; the reading used here (and by the HIP path):

    -r^2 lap(psi) + psi = gamma   in the box grid,   d psi / dn = 0 on its boundary,

with r = R / (2 sqrt 3), R the filter radius (2.5 element sizes in the paper's
examples).  psi is trilinear on the nodes of the element grid; gamma is
constant per element, so the load of node a is the sum over its elements of
gamma_e times the integral of the shape function (h^3 / 8).  The filtered
element value is the mean of psi over the element's 8 nodes.  Hence

    F gamma = A K^-1 T gamma,     F^T g = T^T K^-1 A^T g      (K symmetric)

with K = r^2 K_lap + M assembled from element matrices that this module
integrates with the 2x2x2 Gauss rule (exact for trilinear products), A the
element-mean and T the element-to-node load.  Exact sparse solves.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def element_matrices(h: float):
    """(K_lap_e, M_e), 8x8, by Gauss quadrature of the trilinear shape functions
    on the cube [0, h]^3; local node a = ax + 2 ay + 4 az."""
    gp = [(1 - 1 / np.sqrt(3)) / 2, (1 + 1 / np.sqrt(3)) / 2]  # Gauss points on [0, 1]
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for qx, qy, qz in itertools.product(gp, gp, gp):
        N = np.empty(8)
        dN = np.empty((8, 3))
        for a in range(8):
            c = [(a >> d) & 1 for d in range(3)]
            f = [q if ci else 1 - q for q, ci in zip((qx, qy, qz), c)]
            df = [1.0 if ci else -1.0 for ci in c]
            N[a] = f[0] * f[1] * f[2]
            dN[a, 0] = df[0] * f[1] * f[2] / h
            dN[a, 1] = f[0] * df[1] * f[2] / h
            dN[a, 2] = f[0] * f[1] * df[2] / h
        w = h ** 3 / 8.0  # weight 1/8 of the unit cube times h^3
        K += w * dN @ dN.T
        M += w * np.outer(N, N)
    return K, M


def _elem_nodes(nx, ny, nz):
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    I, J, K = I.reshape(-1), J.reshape(-1), K.reshape(-1)
    out = np.empty((nx * ny * nz, 8), dtype=np.int64)
    for a in range(8):
        out[:, a] = (I + (a & 1)) + (nx + 1) * ((J + ((a >> 1) & 1)) + (ny + 1) * (K + (a >> 2)))
    return out


class Filter:
    def __init__(self, nx: int, ny: int, nz: int, h: float, radius: float):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, h
        self.r = radius / (2.0 * np.sqrt(3.0))
        Ke, Me = element_matrices(h)
        self.Ee = self.r ** 2 * Ke + Me
        en = _elem_nodes(nx, ny, nz)
        nn = (nx + 1) * (ny + 1) * (nz + 1)
        ne = nx * ny * nz
        rows = np.repeat(en, 8, axis=1).reshape(-1)
        cols = np.tile(en, (1, 8)).reshape(-1)
        vals = np.tile(self.Ee.reshape(-1), ne)
        self.K = sp.csc_matrix((vals, (rows, cols)), shape=(nn, nn))
        eidx = np.repeat(np.arange(ne), 8)
        self.T = sp.csr_matrix((np.full(8 * ne, h ** 3 / 8.0), (en.reshape(-1), eidx)),
                               shape=(nn, ne))
        self.A = sp.csr_matrix((np.full(8 * ne, 1.0 / 8.0), (eidx, en.reshape(-1))),
                               shape=(ne, nn))
        self._lu = spla.splu(self.K)

    def solve_nodal(self, b: np.ndarray) -> np.ndarray:
        return self._lu.solve(np.asarray(b, dtype=np.float64))

    def apply(self, gamma: np.ndarray) -> np.ndarray:
        """F gamma (element values in, element values out)."""
        return self.A @ self.solve_nodal(self.T @ gamma)

    def apply_transpose(self, g: np.ndarray) -> np.ndarray:
        """F^T g."""
        return self.T.T @ self.solve_nodal(self.A.T @ g)
