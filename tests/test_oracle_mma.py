"""Pins of the oracle MMA (Sec. "Optimisation problem": MMA with one volume
constraint; algorithm as published by Svanberg, see the oracle's header)."""
import numpy as np
import pytest

from oracle.mma import MMA


def test_approximation_interpolates_value_and_gradient():
    rng = np.random.default_rng(0)
    n = 50
    x = rng.uniform(0.2, 0.8, n)
    df0, df1 = rng.standard_normal(n), rng.standard_normal(n)
    m = MMA(n)
    sp = m.subproblem(x, 0.3, df0, df1)
    # f1~(x) = f1 and d f_i~ / dx_j (x) = df_ij
    assert m.g_of(sp, x) == pytest.approx(0.3, abs=1e-14)
    for p, q, df in ((sp["p0"], sp["q0"], df0), (sp["p1"], sp["q1"], df1)):
        grad = p / (sp["upp"] - x) ** 2 - q / (x - sp["low"]) ** 2
        assert np.abs(grad - df).max() <= 1e-13


def test_subproblem_solution_is_stationary():
    """x(lam) minimises the Lagrangian of the subproblem over the box: central
    differences of the Lagrangian vanish at interior components, and point
    inward at active bounds; the constraint is active when lam > 0."""
    rng = np.random.default_rng(1)
    n = 40
    x = rng.uniform(0.3, 0.7, n)
    df0 = rng.uniform(-2.0, -0.1, n)  # objective decreases with x
    df1 = np.full(n, 1.0 / n)  # volume-like constraint, active
    m = MMA(n, move=0.5)
    xn, lam = m.update(x, 1.0, df0, 0.02, df1)
    m2 = MMA(n, move=0.5)
    s = m2.subproblem(x, 0.02, df0, df1)
    assert lam > 0.0
    assert abs(m2.g_of(s, xn)) <= 1e-12
    L = lambda z: ((s["p0"] + lam * s["p1"]) / (s["upp"] - z) + (s["q0"] + lam * s["q1"]) / (z - s["low"]))
    eps = 1e-7
    dL = (L(xn + eps) - L(xn - eps)) / (2 * eps)
    inner = (xn > s["alpha"] + 1e-9) & (xn < s["beta"] - 1e-9)
    assert inner.any()
    assert np.abs(dL[inner]).max() <= 1e-5 * np.abs(dL).max() + 1e-8
    assert np.all(dL[xn <= s["alpha"] + 1e-12] >= -1e-8)
    assert np.all(dL[xn >= s["beta"] - 1e-12] <= 1e-8)


def test_converges_to_the_analytic_optimum():
    """min sum c_j / x_j s.t. mean(x) <= V, 0 <= x <= 1: the KKT point is
    x_j = n V sqrt(c_j) / sum sqrt(c) when that lies inside the box."""
    rng = np.random.default_rng(2)
    n, V = 30, 0.4
    c = rng.uniform(0.5, 1.5, n)
    xs = n * V * np.sqrt(c) / np.sqrt(c).sum()
    assert xs.max() < 1.0
    m = MMA(n, move=0.2)
    x = np.full(n, V)
    for _ in range(150):
        f0, df0 = np.sum(c / x), -c / x ** 2
        f1, df1 = x.mean() - V, np.full(n, 1.0 / n)
        x, _ = m.update(x, f0, df0, f1, df1)
    assert np.abs(x - xs).max() <= 1e-6
