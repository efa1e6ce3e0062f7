"""Adjoint sensitivities through the ``torch.autograd.Function`` wrappers,
against central finite differences of re-solved compliances (the paper's
consistency claim for the tau derivatives) and against the oracle gradient."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1508_04596_amd import inputs
from tests.helpers import rel_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_04596_amd import autograd, fe
    fe.lib()
    return fe, autograd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)


def _fd_check(fe, autograd, p, n_dirs, seeds0=3001, eps=1e-6, tol=2e-5):
    prob = fe.Problem.from_inputs(p, mask="solve")
    s = dev(p.s)
    adj = fe.solve_opts(rtol_lin=1e-12, max_lin=5000)
    # converge as far as FP64 rounding allows, then hold every re-solve to
    # the same absolute residual level
    x0 = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    rep = fe.newton_solve(prob, dev(p.gamma), s, x0,
                          fe.solve_opts(rtol_newton=1e-12, rtol_lin=1e-10, max_newton=12),
                          allow_not_converged=True)
    atol = max(1e-12 * rep["res0"], 2.0 * rep["res_final"])
    print(f"[adjoint-fd] {p.name}: cold solve rel residual {rep['res_final'] / rep['res0']:.2e}, "
          f"Newton {rep['newton_its']}")
    warm = fe.solve_opts(rtol_newton=0.0, atol_newton=atol, rtol_lin=1e-10, max_newton=30)
    g = dev(p.gamma).requires_grad_(True)
    f = autograd.compliance(g, prob, s, warm, adj, x0)
    f.backward()
    grad = g.grad.detach().cpu().numpy()
    worst = 0.0
    for k in range(n_dirs):
        d = inputs.random_gamma_direction(p, seeds0 + k)
        vals = []
        for sgn in (+1, -1):
            gp = dev(p.gamma + sgn * eps * d)
            vals.append(float(autograd.compliance(gp, prob, s, warm, adj, x0)))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = float(grad @ d)
        err = abs(an - fd) / max(abs(fd), 1e-300)
        worst = max(worst, err)
    print(f"[adjoint-fd] {p.name}: {n_dirs} directions, worst rel err {worst:.3e}")
    prob.close()
    assert worst <= tol
    return grad


def test_compliance_gradient_against_fd_24_cubed(mods):
    fe, autograd = mods
    p = inputs.scaled_config(24, 24, 24, 1e5, seed=1004, extra_passes=1)
    _fd_check(fe, autograd, p, n_dirs=32)


def test_compliance_gradient_against_fd_c4(mods):
    """96^3, Gr = 1e5 (the adjoint workload), 32 random directions (seeds 3001..3032)."""
    fe, autograd = mods
    p = inputs.config(4)
    print("[adjoint-fd] C4 96^3", flush=True)
    _fd_check(fe, autograd, p, n_dirs=32)


def test_state_solve_vjp_matches_oracle(mods):
    fe, autograd = mods
    p = inputs.scaled_config(8, 8, 8, 3e3, seed=88, extra_passes=1)
    prob = fe.Problem.from_inputs(p, mask="solve")
    s = dev(p.s)
    g = dev(p.gamma).requires_grad_(True)
    x = autograd.state_solve(g, prob, s, fe.solve_opts(rtol_newton=1e-13, rtol_lin=1e-11),
                             fe.solve_opts(rtol_lin=1e-13, max_lin=5000))
    c = torch.from_numpy(osolve.compliance_gradient_x(p, mask="solve")).cuda()
    (x * c).sum().backward()
    _, ref = osolve.adjoint_gradient(p, x.detach().cpu().numpy())
    err = rel_norm(g.grad.cpu().numpy(), ref)
    print(f"[vjp] rel err {err:.3e}")
    assert err <= 1e-9
    prob.close()
