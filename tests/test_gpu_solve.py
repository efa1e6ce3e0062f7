"""GPU Newton / adjoint solves against the oracle (backward error and forward difference)."""
import numpy as np
import pytest

import oracle
from oracle import solve as osolve
from paper_1508_04596_amd import inputs
from tests.helpers import rel_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_04596_amd import fe as fe_mod
    fe_mod.lib()
    return fe_mod


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("pc", ["bjacobi", "multigrid"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_c1_backward_error(fe, prec, pc):
    p = inputs.config(1)
    print(f"[solve] C1 {prec} {pc}", flush=True)
    prob = fe.Problem.from_inputs(p, mask="solve")
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    rep = fe.newton_solve(prob, dev(p.gamma), dev(p.s), x,
                          fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, precond=pc))
    assert rep["precond"] == pc
    xs = host(x)
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    r = np.linalg.norm(oracle.residual(p, xs, mask="solve"))
    print(f"[solve] {prec} {pc}: newton {rep['newton_its']} lin {rep['lin_its']} rel {r / r0:.3e} "
          f"levels {rep['mg_levels']}")
    assert r <= 1e-8 * r0 * 1.0001
    if pc == "multigrid":  # two levels with an exact coarse solve: few iterations
        assert max(rep["lin_its"]) <= 15
    x_or, _, _ = osolve.newton(p, rtol=1e-13)
    print(f"[solve] forward rel diff {rel_norm(xs, x_or):.3e}")
    assert rel_norm(xs, x_or) <= 1e-5
    prob.close()


def test_newton_c1_tight_matches_oracle_solution(fe):
    p = inputs.config(1)
    prob = fe.Problem.from_inputs(p, mask="solve")
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    fe.newton_solve(prob, dev(p.gamma), dev(p.s), x,
                    fe.solve_opts(rtol_newton=1e-13, rtol_lin=1e-12, max_lin=5000))
    x_or, _, _ = osolve.newton(p, rtol=1e-13)
    err = rel_norm(host(x), x_or)
    print(f"[solve] tight forward rel diff {err:.3e}")
    assert err <= 1e-10
    prob.close()


def test_adjoint_gradient_against_oracle(fe):
    p = inputs.scaled_config(10, 10, 10, 2e3, seed=44, extra_passes=1)
    prob = fe.Problem.from_inputs(p, mask="solve")
    g, s = dev(p.gamma), dev(p.s)
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-12, rtol_lin=1e-10))
    xs = host(x)
    lam_or, grad_or = osolve.adjoint_gradient(p, xs)
    c = torch.empty_like(x)
    fe.fe_compliance(prob, x, s, c)
    lam, rep = fe.fe_adjoint_solve(prob, x, g, s, c, opts=fe.solve_opts(rtol_lin=1e-12, max_lin=5000))
    dg = fe.fe_dR_dgamma(prob, x, g, s, lam)
    grad = -host(dg)
    print(f"[adjoint] its {rep['lin_its_total']} lam err {rel_norm(host(lam), lam_or):.3e} "
          f"grad err {rel_norm(grad, grad_or):.3e}")
    # lambda's pressure part is weakly determined (closed cavity, one pinned
    # pressure): compare it through the oracle's backward error, and the
    # gradient, which does not see that part, directly
    lam_h = host(lam)
    cc = osolve.compliance_gradient_x(p, mask="solve")
    bwd = np.linalg.norm(oracle.jtvp(p, xs, lam_h, mask="solve") - cc) / np.linalg.norm(cc)
    print(f"[adjoint] oracle backward error of lambda {bwd:.3e}")
    assert bwd <= 1e-10
    assert rel_norm(grad, grad_or) <= 1e-9
    prob.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multigrid_newton_on_32_cubed(fe, prec):
    """Multigrid-preconditioned solve on a 32^3 C2-style problem (3 levels)."""
    p = inputs.scaled_config(32, 32, 32, 1e4, seed=1032)
    prob = fe.Problem.from_inputs(p, mask="solve")
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    rep = fe.newton_solve(prob, dev(p.gamma), dev(p.s), x,
                          fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, precond="multigrid"))
    xs = host(x)
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    r = np.linalg.norm(oracle.residual(p, xs, mask="solve"))
    print(f"[mg32] {prec}: newton {rep['newton_its']} lin {rep['lin_its']} levels {rep['mg_levels']} "
          f"t {rep['t_total_s']:.3f}s rel {r / r0:.3e}")
    assert rep["mg_levels"] >= 3
    assert r <= 1e-8 * r0 * 1.0001
    prob.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multigrid_on_odd_grids(fe, prec):
    """Odd element counts: the coarse grid of ceil(n/2) elements sticks out of
    the fine one by half a coarse element where n is odd.  The multigrid solve
    must reach the oracle's backward error, and the adjoint solve through the
    transposed V-cycle too."""
    for dims in ((17, 13, 9), (21, 21, 21)):
        p = inputs.scaled_config(*dims, 1e4, seed=1700 + dims[0])
        print(f"[mg-odd] {dims} {prec}", flush=True)
        prob = fe.Problem.from_inputs(p, mask="solve")
        g, s = dev(p.gamma), dev(p.s)
        x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
        rep = fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec,
                                                           precond="multigrid"))
        xs = host(x)
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        r = np.linalg.norm(oracle.residual(p, xs, mask="solve"))
        print(f"[mg-odd] newton {rep['newton_its']} lin {rep['lin_its']} levels {rep['mg_levels']} "
              f"rel {r / r0:.3e}")
        assert rep["mg_levels"] >= 2
        assert r <= 1e-8 * r0 * 1.0001
        assert sum(rep["lin_its"]) <= 40 * rep["newton_its"]
        c = torch.empty_like(x)
        fe.fe_compliance(prob, x, s, c)
        lam, arep = fe.fe_adjoint_solve(prob, x, g, s, c,
                                        opts=fe.solve_opts(rtol_lin=1e-10, precond="multigrid"))
        cc = osolve.compliance_gradient_x(p, mask="solve")
        bwd = np.linalg.norm(oracle.jtvp(p, xs, host(lam), mask="solve") - cc) / np.linalg.norm(cc)
        print(f"[mg-odd] adjoint its {arep['lin_its_total']} backward error {bwd:.3e}")
        assert bwd <= 1e-9
        prob.close()


@pytest.mark.parametrize("case", ["C1 8^3", "32^3"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_assembled_levels_match_matrix_free(fe, case, prec):
    """Multigrid levels applied as assembled 27-point block stencils are the same
    operators as the matrix-free element pass: the preconditioned solves agree
    step by step, and so do the adjoint (transposed V-cycle) solves."""
    p = inputs.config(1) if case == "C1 8^3" else inputs.scaled_config(32, 32, 32, 1e4, seed=1032)
    print(f"[asm] {case} {prec}", flush=True)
    g, s = dev(p.gamma), dev(p.s)
    out = {}
    for asm in (0, -1):
        prob = fe.Problem.from_inputs(p, mask="solve")
        x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
        o = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, precond="multigrid",
                          mg_assembled_nodes=asm)
        rep = fe.newton_solve(prob, g, s, x, o)
        c = torch.empty_like(x)
        fe.fe_compliance(prob, x, s, c)
        lam, arep = fe.fe_adjoint_solve(prob, x, g, s, c, opts=fe.solve_opts(
            rtol_lin=1e-8, precond="multigrid", mg_assembled_nodes=asm))
        out[asm] = (host(x), rep, host(lam), arep)
        print(f"[asm] mg_assembled_nodes={asm}: newton {rep['newton_its']} lin {rep['lin_its']} "
              f"adjoint its {arep['lin_its_total']}")
        prob.close()
    (x0, r0, l0, a0), (x1, r1, l1, a1) = out[0], out[-1]
    assert r0["newton_its"] == r1["newton_its"]
    assert all(abs(a - b) <= 1 for a, b in zip(r0["lin_its"], r1["lin_its"]))
    assert abs(a0["lin_its_total"] - a1["lin_its_total"]) <= 1
    print(f"[asm] x rel diff {rel_norm(x1, x0):.3e} lambda rel diff {rel_norm(l1, l0):.3e}")
    assert rel_norm(x1, x0) <= 1e-6
    assert rel_norm(l1, l0) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multigrid_wide_band_coarsest_level(fe, prec):
    """16x16x4 slab: two levels, the coarsest (8x8x2, 1215 DOF, 438 of them free)
    has a condensed half bandwidth of 287, beyond the register-set size of the
    device inverse (its column-streaming path); the fine level itself is assembled.  The solve must reach the oracle's
    backward-error bar and match the oracle's Newton solution, in few iterations
    (an exact coarse solve on a two-level hierarchy)."""
    p = inputs.scaled_config(16, 16, 4, 2e3, seed=404)
    print(f"[mg-slab] {prec}", flush=True)
    prob = fe.Problem.from_inputs(p, mask="solve")
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    rep = fe.newton_solve(prob, dev(p.gamma), dev(p.s), x,
                          fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, precond="multigrid"))
    xs = host(x)
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    r = np.linalg.norm(oracle.residual(p, xs, mask="solve"))
    x_or, _, _ = osolve.newton(p, rtol=1e-13)
    print(f"[mg-slab] {prec}: levels {rep['mg_levels']} newton {rep['newton_its']} lin {rep['lin_its']} "
          f"rel {r / r0:.3e} forward {rel_norm(xs, x_or):.3e}")
    assert rep["mg_levels"] == 2
    assert r <= 1e-8 * r0 * 1.0001
    assert rel_norm(xs, x_or) <= 1e-5
    assert max(rep["lin_its"]) <= 20
    # the transposed V-cycle on the same hierarchy (adjoint solve, FP64)
    s = dev(p.s)
    c = torch.empty_like(x)
    fe.fe_compliance(prob, x, s, c)
    lam, arep = fe.fe_adjoint_solve(prob, x, dev(p.gamma), s, c,
                                    opts=fe.solve_opts(rtol_lin=1e-10, precond="multigrid"))
    cc = osolve.compliance_gradient_x(p, mask="solve")
    bwd = np.linalg.norm(oracle.jtvp(p, xs, host(lam), mask="solve") - cc) / np.linalg.norm(cc)
    print(f"[mg-slab] adjoint its {arep['lin_its_total']} oracle backward error {bwd:.3e}")
    assert bwd <= 1e-8
    assert arep["lin_its_total"] <= 25
    prob.close()


@pytest.mark.parametrize("design", ["all fluid", "all solid"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_degenerate_designs(fe, design, prec):
    """A design with no Brinkman term anywhere (free natural convection in the
    box) and one with the largest everywhere (conduction through solid, the
    velocity held near zero) both reach the oracle's bar."""
    import dataclasses
    base = inputs.scaled_config(16, 16, 12, 1e4, seed=81)
    g = np.ones(base.n_el) if design == "all fluid" else np.zeros(base.n_el)
    p = dataclasses.replace(base, gamma=g)
    print(f"[solve] {design} {prec}", flush=True)
    prob = fe.Problem.from_inputs(p, mask="solve")
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    rep = fe.newton_solve(prob, dev(p.gamma), dev(p.s), x,
                          fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec))
    xs = host(x)
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    r = np.linalg.norm(oracle.residual(p, xs, mask="solve"))
    vel = np.abs(xs.reshape(-1, 5)[:, :3]).max()
    print(f"[solve] {design} {prec}: newton {rep['newton_its']} lin {rep['lin_its'][:rep['newton_its']]} "
          f"rel {r / r0:.3e} max |u| {vel:.3e} levels {rep['mg_levels']}")
    assert r <= 1e-8 * r0 * 1.0001
    prob.close()


@pytest.mark.parametrize("case", ["16^3", "cavity 32"])
def test_coarse_factorisation_reuse(fe, case):
    """Once a Newton step has cut |R| 100-fold, mg_coarse_reuse keeps the
    coarsest factorisation (1) or the whole preconditioner set-up (2, the
    default) for the next step.  The preconditioner then differs from the one
    of the current state, which flexible GMRES admits: every setting reaches the
    oracle's bar with the same Newton steps, and the kept set-up costs at most
    a few FGMRES iterations (none on the smooth problem)."""
    p = (inputs.scaled_config(16, 16, 16, 1e4, seed=5016) if case == "16^3" else
         inputs.cavity_problem(32, 1e5))
    print(f"[coarse-reuse] {case}", flush=True)
    prob = fe.Problem.from_inputs(p, mask="solve")
    g, s = dev(p.gamma), dev(p.s)
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    out = {}
    for reuse in (0, 1, 2):
        x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
        rep = fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-8, mg_coarse_reuse=reuse))
        r = np.linalg.norm(oracle.residual(p, host(x), mask="solve"))
        its = rep["lin_its"][:rep["newton_its"]]
        print(f"[coarse-reuse] {case} reuse {reuse}: newton {rep['newton_its']} lin {its} "
              f"set-up {rep['t_setup_s'] * 1e3:.2f} ms, oracle |R|/|R0| = {r / r0:.3e}")
        assert r <= 1e-8 * r0 * 1.0001
        out[reuse] = (rep["newton_its"], its)
    for reuse in (1, 2):
        assert out[0][0] == out[reuse][0]
        assert sum(out[reuse][1]) <= 1.3 * sum(out[0][1]) + 2
        if case == "16^3":
            assert out[0][1] == out[reuse][1]
    prob.close()
