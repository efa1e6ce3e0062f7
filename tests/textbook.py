"""Textbook 1-D linear-element integrals and their tensor products.

Every trilinear element integral of a product of shape functions and first
derivatives on a cube of edge h factors into three 1-D integrals over [0, h]
of the two linear shape functions N_0 = 1 - t/h, N_1 = t/h.  These are the
standard 2x2 element matrices of linear finite elements; the tests build the
closed forms of the oracle's element Jacobians from them.
"""
import numpy as np


def one_d(h):
    """(M, S, C, D): int N_a N_b, int N_a' N_b', int N_a N_b', int N_a' N_b."""
    M1 = h / 6 * np.array([[2.0, 1.0], [1.0, 2.0]])
    S1 = 1 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    C1 = 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])
    D1 = C1.T
    return M1, S1, C1, D1


def tp(fx, fy, fz):
    """8x8 tensor-product matrix, local node a = ax + 2 ay + 4 az."""
    return np.kron(fz, np.kron(fy, fx))


class Integrals:
    """Element integrals on a cube of edge h (row a = test, column b = trial)."""

    def __init__(self, h):
        self.M1, self.S1, self.C1, self.D1 = one_d(h)
        self.M = tp(self.M1, self.M1, self.M1)

    def dd(self, i, j):
        """int d_i N_a d_j N_b"""
        f = [self.M1, self.M1, self.M1]
        if i == j:
            f[i] = self.S1
        else:
            f[i], f[j] = self.D1, self.C1
        return tp(*f)

    def nd(self, j):
        """int N_a d_j N_b"""
        f = [self.M1, self.M1, self.M1]
        f[j] = self.C1
        return tp(*f)

    def dn(self, i):
        """int d_i N_a N_b"""
        f = [self.M1, self.M1, self.M1]
        f[i] = self.D1
        return tp(*f)

    def lap(self):
        return self.dd(0, 0) + self.dd(1, 1) + self.dd(2, 2)
