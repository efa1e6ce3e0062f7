"""Pins of the oracle's PDE density filter (reading of Sec. "Optimisation
problem": Helmholtz filter, Neumann boundary, trilinear nodal field, element
mean).  Closed forms: the trilinear element matrices, the constant field, and
the cosine modes of the Neumann problem on a uniform grid."""
import itertools

import numpy as np
import pytest

from oracle import filter as ofilter


def test_element_matrices_are_the_textbook_trilinear_ones():
    h = 0.3
    K, M = ofilter.element_matrices(h)
    kap = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}
    mu = {0: 8, 1: 4, 2: 2, 3: 1}
    for a, b in itertools.product(range(8), range(8)):
        d = bin(a ^ b).count("1")
        assert K[a, b] == pytest.approx(h * kap[d], abs=1e-15)
        assert M[a, b] == pytest.approx(h ** 3 / 216 * mu[d], abs=1e-16)


def test_constant_field_is_preserved():
    f = ofilter.Filter(7, 5, 6, 0.1, radius=0.25)
    out = f.apply(np.full(7 * 5 * 6, 0.37))
    assert np.abs(out - 0.37).max() <= 1e-13


@pytest.mark.parametrize("modes", [(1, 0, 0), (2, 3, 1), (4, 1, 5)])
def test_cosine_modes_of_the_neumann_problem(modes):
    """K c = lambda (w * c) for nodal c = prod_d cos(pi k_d i_d / n_d), w the
    product of the per-axis end-node halvings and lambda from the 1-D mass and
    stiffness symbols m = h (4 + 2 cos t) / 6, k = (2 - 2 cos t) / h."""
    nx, ny, nz, h, R = 6, 5, 7, 0.2, 0.5
    f = ofilter.Filter(nx, ny, nz, h, radius=R)
    r2 = (R / (2 * np.sqrt(3))) ** 2
    c, w, m, k = [], [], [], []
    for n, kd in zip((nx, ny, nz), modes):
        i = np.arange(n + 1)
        t = np.pi * kd / n
        c.append(np.cos(t * i))
        wd = np.ones(n + 1)
        wd[0] = wd[-1] = 0.5
        w.append(wd)
        m.append(h * (4 + 2 * np.cos(t)) / 6)
        k.append((2 - 2 * np.cos(t)) / h)
    cc = np.einsum("k,j,i->kji", c[2], c[1], c[0]).reshape(-1)
    ww = np.einsum("k,j,i->kji", w[2], w[1], w[0]).reshape(-1)
    lam = r2 * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) + m[0] * m[1] * m[2]
    psi = f.solve_nodal(lam * ww * cc)
    assert np.abs(psi - cc).max() <= 1e-12


def test_transpose_identity():
    f = ofilter.Filter(5, 4, 6, 0.2, radius=0.5)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(120), rng.standard_normal(120)
    assert abs(f.apply(a) @ b - a @ f.apply_transpose(b)) <= 1e-13 * np.abs(a).sum() * np.abs(b).max()


def test_filter_smooths_and_keeps_the_mean_weighting():
    """A single solid element spreads to its neighbours (values in (0, 1)),
    and the element-sum of the filtered field equals that of the input
    (T^T K^-1 T preserves the integral because K 1 = M 1 = T 1)."""
    f = ofilter.Filter(6, 6, 6, 1 / 6, radius=2.5 / 6)
    g = np.ones(216)
    g[3 + 6 * (3 + 6 * 3)] = 0.0
    out = f.apply(g)
    assert out.min() > 0.0 and out.max() <= 1.0 + 1e-14
    assert np.sum(out) == pytest.approx(np.sum(g), rel=1e-12)
