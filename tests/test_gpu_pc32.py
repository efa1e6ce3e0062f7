"""FP32 preconditioner with the FP64 operator (fe_solve_opts.pc_prec = FP32).

Flexible GMRES admits a preconditioner that differs from step to step, so an
FP32 block-Jacobi or V-cycle leaves the FP64 Krylov process, its operator and
its residuals as they are: the Newton and adjoint solves must reach the same
oracle bars as the all-FP64 solves, with about as many iterations.  The
adjoint solve runs the transposed FP32 V-cycle, which no other mode uses.
"""
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


CASES = {
    "C1 bjacobi": (lambda: inputs.config(1), "bjacobi"),
    "C1 multigrid": (lambda: inputs.config(1), "multigrid"),
    "32^3 multigrid": (lambda: inputs.scaled_config(32, 32, 32, 1e4, seed=1032), "multigrid"),
    "17x13x9 multigrid": (lambda: inputs.scaled_config(17, 13, 9, 1e4, seed=1717), "multigrid"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_newton_with_fp32_preconditioner(fe, case):
    mk, pc = CASES[case]
    p = mk()
    print(f"[pc32] {case}", flush=True)
    g, s = dev(p.gamma), dev(p.s)
    out = {}
    for pp in ("fp64", "fp32"):
        prob = fe.Problem.from_inputs(p, mask="solve")
        x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
        rep = fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-8, precond=pc, pc_prec=pp))
        out[pp] = (host(x), rep)
        prob.close()
    r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
    (x64, rep64), (x32, rep32) = out["fp64"], out["fp32"]
    r = np.linalg.norm(oracle.residual(p, x32, mask="solve"))
    its64 = rep64["lin_its"][:rep64["newton_its"]]
    its32 = rep32["lin_its"][:rep32["newton_its"]]
    print(f"[pc32] {case}: newton {rep32['newton_its']} lin {its32} (FP64 preconditioner {its64}), "
          f"oracle |R|/|R0| = {r / r0:.3e}, |x - x_fp64| / |x_fp64| = {rel_norm(x32, x64):.1e}")
    assert rep32["precond"] == pc
    assert r <= 1e-8 * r0 * 1.0001
    # the FP32 preconditioner's rounding (1e-7) is far below what it leaves of
    # the error (1e-1 per V-cycle): the iteration counts stay close
    assert rep32["newton_its"] == rep64["newton_its"]
    assert all(b <= a + max(2, a // 5) for a, b in zip(its64, its32)), (its64, its32)
    assert rel_norm(x32, x64) <= 1e-6


@pytest.mark.parametrize("pc", ["bjacobi", "multigrid"])
def test_adjoint_with_fp32_preconditioner(fe, pc):
    """The adjoint solve J^T lambda = df/dx with the transposed FP32
    preconditioner, on an odd grid (overhanging coarse elements) for the
    multigrid case: lambda meets the oracle's backward error bar."""
    p = inputs.scaled_config(17, 13, 9, 1e4, seed=1717)
    print(f"[pc32-adjoint] {pc}", flush=True)
    prob = fe.Problem.from_inputs(p, mask="solve")
    g, s = dev(p.gamma), dev(p.s)
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-10, precond=pc))
    xs = host(x)
    c = torch.empty_like(x)
    fe.fe_compliance(prob, x, s, c)
    cc = osolve.compliance_gradient_x(p, mask="solve")
    its = {}
    for pp in ("fp64", "fp32"):
        lam, arep = fe.fe_adjoint_solve(prob, x, g, s, c, opts=fe.solve_opts(
            rtol_lin=1e-10, precond=pc, pc_prec=pp, max_lin=3000))
        bwd = np.linalg.norm(oracle.jtvp(p, xs, host(lam), mask="solve") - cc) / np.linalg.norm(cc)
        its[pp] = arep["lin_its_total"]
        print(f"[pc32-adjoint] {pc} pc_prec {pp}: its {its[pp]} oracle backward error {bwd:.3e}")
        assert arep["status"] == fe.FE_OK
        assert bwd <= 1e-9
    assert its["fp32"] <= its["fp64"] + max(2, its["fp64"] // 5), its
    prob.close()


def test_fp32_preconditioner_requests_on_the_batched_server(fe):
    """Requests with the FP32 preconditioner share the lockstep engine's steps
    with all-FP64 and mixed requests (their FP64 J z in the same batched
    launches as the FP64 requests', their V-cycles in those of the mixed ones)
    and reach the oracle bar."""
    reqs = inputs.serving_trace(n_requests=4, seed=4300, sizes=(16, 24))
    probs = [inputs.request_problem(r) for r in reqs]
    kinds = ["fp32", "fp64", "fp32", "mixed"]
    with fe.Server(4 << 30, max_active=4, batched=True) as srv:
        tickets = []
        for p, k in zip(probs, kinds):
            o = (fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed") if k == "mixed" else
                 fe.solve_opts(rtol_newton=1e-8, pc_prec=k))
            ph = fe.make_phys(p.Pr, p.Gr, p.Ck, p.qf, p.alpha_max, p.q_alpha, p.eg)
            tickets.append(srv.submit(p.nx, p.ny, p.nz, p.h, ph, p.gamma, p.s, o))
        res = [srv.wait(t) for t in tickets]
    for (rc, x, rep), p, k in zip(res, probs, kinds):
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        r = np.linalg.norm(oracle.residual(p, x, mask="solve"))
        print(f"[pc32-serve] {p.nx}^3 {k}: lin {rep['lin_its'][:rep['newton_its']]} "
              f"oracle |R|/|R0| = {r / r0:.3e}")
        assert rc == fe.FE_OK, rep
        assert r <= 1e-8 * r0 * 1.0001
