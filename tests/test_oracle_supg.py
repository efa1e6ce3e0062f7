"""Pins of the oracle's streamline-upwind (SUPG) terms and of the tau variations.

At rest (u = 0) the SUPG weights tau (u . grad N_a) and tauT (u . grad N_a)
vanish, so the closed forms at rest cannot see them.  Here the element Jacobian
is taken in a uniform flow: every node of the element carries the same velocity
c, with p = 0, T = 0 and s = 0.  Then u_h = c and grad u_h = 0 everywhere in the
element, the strong thermal residual r_T = c . grad T - s vanishes and the
strong momentum residual is r_M = alpha c (zero in fluid), so the Jacobian is a
sum of integrals of products of shape functions and their first derivatives:
exactly the 1-D linear-element integrals in tensor products (Sec. "Finite
element formulation": Galerkin + SUPG/PSPG with the single element parameter
tau of the appendix "Stabilisation parameters").  A sign, index or factor
mistake in any SUPG term (momentum or thermal), in the PSPG or Brinkman terms,
or in the variation of tau with the element velocity changes that Jacobian by
far more than rounding.

The last test reproduces the closing comparison of the appendix: dropping
d tau / d u_e and d tau / d gamma_e from the derivatives degrades the agreement
of the adjoint design sensitivities with finite differences by more than an
order of magnitude.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from oracle import solve as osolve
from paper_1508_04596_amd import inputs

import textbook

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "fe_oracle.c")


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build_oracle(force=False)


def _phys(Pr, Gr, eg, Ck=0.1, qf=0.881, amax=1e4, qa=1.0):
    return np.array([Pr, Gr, Ck, qf, amax, qa, *eg], dtype=np.float64)


def taus_by_definition(h, Pr, U2, alpha, K):
    """tau and tauT from the inverse-square combination of the convective
    limit 4h/|u_e| (|u_e|^2 over the 24 nodal velocities), the viscous limit
    h^2/(4 Pr) and the Brinkman limit 1/alpha; thermal: convective and h^2/(4K)."""
    tau = (U2 / (4 * h) ** 2 + (4 * Pr / h ** 2) ** 2 + alpha ** 2) ** -0.5
    tauT = (U2 / (4 * h) ** 2 + (4 * K / h ** 2) ** 2) ** -0.5
    return tau, tauT


def textbook_jacobian_uniform_flow(h, Pr, B, eg, alpha, K, c):
    """Element Jacobian at u_a = c for all 8 nodes, p = T = s = 0.

    Row blocks (test function N_a), column blocks (trial N_b):
      u_i-u_k : delta_ik [ int N_a c.grad N_b + Pr L + alpha M + tau int (c.grad N_a) c.grad N_b
                           + tau alpha int (c.grad N_a) N_b ]
                + Pr int d_k N_a d_i N_b + tau alpha c_i int d_k N_a N_b
                + dtau_k alpha c_i int c.grad N_a              (tau variation, every b)
      u_i-p   : -int d_i N_a N_b + tau int (c.grad N_a) d_i N_b
      u_i-T   : B eg_i (M + tau int (c.grad N_a) N_b)
      p-u_k   : int N_a d_k N_b + tau int d_k N_a c.grad N_b + tau alpha int d_k N_a N_b
                + dtau_k alpha int c.grad N_a
      p-p     : tau L
      p-T     : tau B sum_i eg_i int d_i N_a N_b
      T-u_k   : 0   (grad T = 0 and r_T = 0)
      T-p     : 0
      T-T     : int N_a c.grad N_b + K L + tauT int (c.grad N_a) c.grad N_b
    with dtau_k = d tau / d u_{b,k} = -tau^3 c_k / (16 h^2) for every node b.
    """
    I = textbook.Integrals(h)
    M, L = I.M, I.lap()
    U2 = 8.0 * float(c @ c)
    tau, tauT = taus_by_definition(h, Pr, U2, alpha, K)
    Cv = sum(c[j] * I.nd(j) for j in range(3))                          # int N_a c.grad N_b
    SS = sum(c[i] * c[j] * I.dd(i, j) for i in range(3) for j in range(3))
    SN = sum(c[i] * I.dn(i) for i in range(3))                          # int (c.grad N_a) N_b
    SD = [sum(c[i] * I.dd(i, k) for i in range(3)) for k in range(3)]   # int (c.grad N_a) d_k N_b
    DS = [sum(c[j] * I.dd(k, j) for j in range(3)) for k in range(3)]   # int d_k N_a c.grad N_b
    gsum = SN.sum(axis=1)                                               # int c.grad N_a
    dtau = -tau ** 3 * c / (16.0 * h * h)
    ones = np.ones((8, 8))
    Ke = np.zeros((40, 40))
    supg = np.zeros((40, 40))  # the streamline-upwind parts alone

    def put(rf, cf, blk, tgt=Ke):
        tgt[rf::5, cf::5] += blk

    for i in range(3):
        for k in range(3):
            # tau (du . grad N_a) r_M,i with r_M = alpha c:  d_k N_a times N_b
            blk = Pr * I.dd(k, i) + tau * alpha * c[i] * I.dn(k)
            blk = blk + dtau[k] * alpha * c[i] * gsum[:, None] * ones
            if i == k:
                blk = blk + Cv + Pr * L + alpha * M + tau * SS + tau * alpha * SN
                put(i, k, tau * SS + tau * alpha * SN, supg)
            put(i, k, blk)
        put(i, 3, -I.dn(i) + tau * SD[i])
        put(i, 3, tau * SD[i], supg)
        put(i, 4, B * eg[i] * (M + tau * SN))
        put(i, 4, B * eg[i] * tau * SN, supg)
    for k in range(3):
        put(3, k, I.nd(k) + tau * DS[k] + tau * alpha * I.dn(k)
            + dtau[k] * alpha * gsum[:, None] * ones)
    put(3, 3, tau * L)
    put(3, 4, tau * B * sum(eg[i] * I.dn(i) for i in range(3)))
    put(4, 4, Cv + K * L + tauT * SS)
    put(4, 4, tauT * SS, supg)
    return Ke, supg


CASES = [
    # h, Pr, Gr, gamma, c, eg
    (1 / 8, 0.7, 1e3, 1.0, (3.0, -2.0, 5.0), (0.0, 0.0, -1.0)),        # fluid: alpha = 0
    (0.37, 0.71, 2.5e4, 1.0, (40.0, 25.0, -60.0), (0.3, -0.4, -0.866)),  # convection-dominated
    (1 / 16, 1.3, 1e4, 0.6, (-80.0, 30.0, 45.0), (0.0, 0.6, -0.8)),     # porous: alpha > 0
    (1 / 4, 0.9, 2e3, 0.93, (6.0, 9.0, -4.0), (1.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("h,Pr,Gr,gam,c,eg", CASES)
def test_element_jacobian_in_uniform_flow_equals_textbook(h, Pr, Gr, gam, c, eg):
    c = np.asarray(c, dtype=np.float64)
    eg = np.asarray(eg, dtype=np.float64)
    eg = eg / np.linalg.norm(eg)
    p = inputs.tiny_problem(1, 1, 1, Gr=Gr, h=h)
    p.Pr, p.eg = Pr, tuple(eg)
    p.gamma[:] = gam
    p.s[:] = 0.0
    x = np.zeros((8, 5))
    x[:, :3] = c
    Ke = oracle.element_jacobians(p, x.reshape(-1))[0]
    a, K, _, _ = oracle.material(p.phys(), np.array([gam]))
    ref, supg = textbook_jacobian_uniform_flow(h, Pr, Gr * Pr ** 2, eg, a[0], K[0], c)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(Ke, ref, rtol=1e-11, atol=1e-12 * scale)
    # the SUPG parts are far above the tolerance: a flipped sign would fail
    assert np.abs(supg).max() > 1e-4 * scale


def test_residual_in_uniform_flow_is_brinkman_and_supg_only():
    """R at the uniform-flow state itself (p = T = s = 0): the Galerkin convection
    and viscous terms vanish (grad u = 0), leaving the Brinkman force alpha M c,
    its SUPG weight tau alpha int (c.grad N_a) c_i, the PSPG row tau alpha c.int grad N_a
    and nothing in the T rows."""
    h, Pr, gam = 1 / 10, 0.8, 0.55
    c = np.array([7.0, -3.0, 2.0])
    ph = _phys(Pr, 3e3, (0.0, 0.0, -1.0))
    xe = np.zeros((8, 5))
    xe[:, :3] = c
    Re = oracle.element_residual(h, ph, xe, gam).reshape(8, 5)
    a, K, _, _ = oracle.material(ph, np.array([gam]))
    I = textbook.Integrals(h)
    tau, _ = taus_by_definition(h, Pr, 8 * c @ c, a[0], K[0])
    SN = sum(c[i] * I.dn(i) for i in range(3))
    g = SN.sum(axis=1)                            # int c.grad N_a
    gi = [I.dn(i).sum(axis=1) for i in range(3)]  # int d_i N_a
    Msum = I.M.sum(axis=1)                        # int N_a
    for i in range(3):
        np.testing.assert_allclose(Re[:, i], a[0] * c[i] * (Msum + tau * g), rtol=1e-12)
    np.testing.assert_allclose(Re[:, 3], tau * a[0] * sum(c[i] * gi[i] for i in range(3)),
                               rtol=1e-11, atol=1e-13 * np.abs(Re).max())
    np.testing.assert_allclose(Re[:, 4], 0.0, atol=1e-14 * np.abs(Re).max())


# -------------------------------------------------------------- mutation check --

def _mutant_library(tmp_path, edits):
    """Compile a copy of the oracle with textual edits; returns the ctypes library."""
    tmp_path.mkdir(parents=True, exist_ok=True)
    src = open(ORACLE_SRC).read()
    for old, new in edits:
        n = src.count(old)
        assert n >= 1, f"mutation pattern not found in the oracle: {old!r}"
        src = src.replace(old, new)
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(src)
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-std=c11", "-o", str(so_path), str(c_path),
                    "-lm"], check=True)
    return ctypes.CDLL(str(so_path))


def _mutant_element_jacobian(lib, p, x):
    d = ctypes.POINTER(ctypes.c_double)
    out = np.empty((p.n_el, 40, 40))
    ph = p.phys()
    x = np.ascontiguousarray(x, dtype=np.float64)
    lib.or_element_jacobians(ctypes.c_int(p.nx), ctypes.c_int(p.ny), ctypes.c_int(p.nz),
                             ctypes.c_double(p.h), ph.ctypes.data_as(d), x.ctypes.data_as(d),
                             p.gamma.ctypes.data_as(d), p.s.ctypes.data_as(d), None,
                             out.ctypes.data_as(d))
    return out[0]


# Consistent sign flips of the momentum and thermal SUPG terms in the residual,
# J v and lambda^T dR/dgamma: every other pin (rest-state closed forms, finite
# differences, brute-force Jacobians, invariants, the manufactured solution at
# Gr = 100) is blind to them.
SUPG_FLIP = [
    ("tau * udN * rM[i]);", "- tau * udN * rM[i]);"),
    ("+ tauT * udN * rT);", "- tauT * udN * rT);"),
    ("+ dtau * udN * rM[i] + tau * dudN * rM[i] + tau * udN * drM[i]);",
     "- dtau * udN * rM[i] - tau * dudN * rM[i] - tau * udN * drM[i]);"),
    ("+ dtauT * udN * rT + tauT * dudN * rT", "- dtauT * udN * rT - tauT * dudN * rT"),
    ("                                 + tauT * udN * drT);", "                                 - tauT * udN * drT);"),
    ("+ dtau_da * udN * rM[i] + tau * udN * F.u[i];", "- dtau_da * udN * rM[i] - tau * udN * F.u[i];"),
    ("(diff + dtauT_dK * udN * rT)", "(diff - dtauT_dK * udN * rT)"),
]


def test_uniform_flow_pin_rejects_a_sign_flipped_supg(tmp_path):
    h, Pr, Gr, gam, c, eg = CASES[2]
    c = np.asarray(c, dtype=np.float64)
    eg = np.asarray(eg) / np.linalg.norm(eg)
    p = inputs.tiny_problem(1, 1, 1, Gr=Gr, h=h)
    p.Pr, p.eg = Pr, tuple(eg)
    p.gamma[:] = gam
    p.s[:] = 0.0
    x = np.zeros((8, 5))
    x[:, :3] = c
    a, K, _, _ = oracle.material(p.phys(), np.array([gam]))
    ref, _ = textbook_jacobian_uniform_flow(h, Pr, Gr * Pr ** 2, eg, a[0], K[0], c)
    lib = _mutant_library(tmp_path, SUPG_FLIP)
    Km = _mutant_element_jacobian(lib, p, x.reshape(-1))
    err = np.abs(Km - ref).max() / np.abs(ref).max()
    assert err > 1e-4, f"the sign-flipped oracle passes the uniform-flow pin (err {err:.1e})"
    # and the unmodified source compiled the same way passes it
    lib0 = _mutant_library(tmp_path / "plain", [])
    K0 = _mutant_element_jacobian(lib0, p, x.reshape(-1))
    np.testing.assert_allclose(K0, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


# ------------------------------------------------------------------ E11 --

def test_frozen_tau_degrades_adjoint_sensitivities():
    """Appendix "Stabilisation parameters", closing remark: including the
    variations of the stabilisation parameters with the velocity and with the
    design improves the finite-difference agreement of the sensitivities by one
    to two orders of magnitude.  Here: the thermal-compliance gradient from the
    consistent adjoint agrees with central differences of re-solved compliances
    to about 1e-7; with tau and tauT frozen in the Jacobian and in dR/dgamma
    the error is at least ten times larger."""
    n = 6
    p = inputs.tiny_problem(n, n, n, Gr=4e4, seed=37)
    p.gamma = 0.15 + 0.7 * p.gamma          # intermediate design: tau feels alpha
    p.gamma[inputs.source_region(n, n, n)] = 0.0
    p.s = p.s * 40.0                         # strong source: |u| large enough for tau to feel it
    x, _, rr = osolve.newton(p, rtol=1e-14)
    assert rr <= 1e-13
    _, grad = osolve.adjoint_gradient(p, x)
    oracle.set_frozen_tau(True)
    try:
        _, grad_frozen = osolve.adjoint_gradient(p, x)
    finally:
        oracle.set_frozen_tau(False)
    err, err_frozen = [], []
    eps = 1e-6
    for seed in (3101, 3102, 3103, 3104):
        d = inputs.random_gamma_direction(p, seed)
        fp = osolve.compliance(p, osolve.newton(p, x0=x, gamma=p.gamma + eps * d, rtol=1e-14)[0])
        fm = osolve.compliance(p, osolve.newton(p, x0=x, gamma=p.gamma - eps * d, rtol=1e-14)[0])
        fd = (fp - fm) / (2 * eps)
        err.append(abs(grad @ d - fd) / abs(fd))
        err_frozen.append(abs(grad_frozen @ d - fd) / abs(fd))
    print("consistent", ["%.1e" % e for e in err], "frozen tau", ["%.1e" % e for e in err_frozen])
    assert max(err) <= 1e-6
    assert min(err_frozen) >= 10.0 * max(err)
    # the switch changes derivatives only
    oracle.set_frozen_tau(True)
    try:
        r_frozen = oracle.residual(p, x)
    finally:
        oracle.set_frozen_tau(False)
    np.testing.assert_array_equal(r_frozen, oracle.residual(p, x))
