"""Batched launches over tables of problems.

* ``fe_jvp_batch_run``: one element-pass launch and one shared-node launch over
  problems of different grids give, per problem, bitwise the result of
  ``fe_jvp`` on that problem alone, in any order and grouping.
* The lockstep server (``FE_SERVE_BATCHED``): every request of a mix reaches the
  oracle's residual bar, and its result is bitwise the same when it is served
  alone (a batch of one) and inside the mix.
"""
import numpy as np
import pytest

import oracle
from paper_1508_04596_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_04596_amd import fe as fe_mod
    fe_mod.lib()
    return fe_mod


# grids of different tile counts, ragged tiles and a single element
GRIDS = [(16, 16, 16), (24, 24, 24), (17, 13, 9), (8, 8, 8), (1, 1, 1), (33, 9, 20)]


def _problems(fe, dtype):
    dev = torch.device("cuda:0")
    out = []
    for k, (nx, ny, nz) in enumerate(GRIDS):
        p = inputs.scaled_config(nx, ny, nz, 1e4, seed=700 + k)
        prob = fe.Problem.from_inputs(p, mask="solve")
        rng = np.random.default_rng(900 + k)
        x = torch.from_numpy(rng.standard_normal(prob.n_dof) * 0.1).to(dev, dtype)
        v = torch.from_numpy(rng.standard_normal(prob.n_dof)).to(dev, dtype)
        g = torch.from_numpy(p.gamma).to(dev)
        s = torch.from_numpy(p.s).to(dev)
        out.append((prob, x, g, s, v))
    return out


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_jvp_batch_equals_fe_jvp_bitwise(fe, dtype):
    dt = getattr(torch, dtype)
    items = _problems(fe, dt)
    refs = [fe.fe_jvp(pr, x, g, s, v) for pr, x, g, s, v in items]
    torch.cuda.synchronize()
    orders = [list(range(len(items))), list(reversed(range(len(items)))), [3], [5, 0, 2]]
    for order in orders:
        outs = [torch.full_like(items[i][4], float("nan")) for i in order]
        b = fe.JvpBatch([items[i][0] for i in order], [items[i][1] for i in order],
                        [items[i][2] for i in order], [items[i][3] for i in order],
                        [items[i][4] for i in order], outs)
        b.run()
        torch.cuda.synchronize()
        for j, i in enumerate(order):
            assert torch.equal(outs[j], refs[i]), f"problem {i} (grid {GRIDS[i]}) in order {order}"
        b.close()
    for it in items:
        it[0].close()


def test_jvp_batch_rejects_a_repeated_problem(fe):
    items = _problems(fe, torch.float64)[:2]
    pr, x, g, s, v = items[0]
    with pytest.raises(fe.FeError):
        fe.JvpBatch([pr, pr], [x, x], [g, g], [s, s], [v, v], [torch.empty_like(v)] * 2)
    for it in items:
        it[0].close()


def _submit(fe, srv, p, opts):
    ph = fe.make_phys(p.Pr, p.Gr, p.Ck, p.qf, p.alpha_max, p.q_alpha, p.eg)
    return srv.submit(p.nx, p.ny, p.nz, p.h, ph, p.gamma, p.s, opts)


def _opts(fe, prec, **kw):
    """fp64, mixed, or pc32 (FP32 preconditioner under the FP64 operator)."""
    if prec == "pc32":
        return fe.solve_opts(rtol_newton=1e-8, pc_prec="fp32", **kw)
    return fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, **kw)


@pytest.mark.parametrize("prec,n_req", [("mixed", 12), ("fp64", 6), ("pc32", 6)])
def test_batched_server_alone_and_in_the_mix(fe, prec, n_req):
    reqs = inputs.serving_trace(n_requests=n_req, seed=4100)
    probs = [inputs.request_problem(r) for r in reqs]
    opts = _opts(fe, prec)
    alone = {}
    steps_alone = 0
    with fe.Server(4 << 30, max_active=1, batched=True) as srv:
        for i, p in enumerate(probs):
            rc, x, rep = srv.wait(_submit(fe, srv, p, opts))
            assert rc == fe.FE_OK, (i, rep)
            alone[i] = x
        steps_alone, _ = srv.engine_stats()
    with fe.Server(8 << 30, max_active=n_req, batched=True) as srv:
        tickets = [_submit(fe, srv, p, opts) for p in probs]
        res = [srv.wait(t) for t in tickets]
        steps_mix, launches_mix = srv.engine_stats()
    print(f"[batched] {prec}: engine steps alone {steps_alone}, in the mix {steps_mix} "
          f"({launches_mix / max(steps_mix, 1):.1f} launches per step)")
    for i, (rc, x, rep) in enumerate(res):
        p = probs[i]
        assert rc == fe.FE_OK, (i, rep)
        assert rep["mg_levels"] >= 2
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        r = np.linalg.norm(oracle.residual(p, x, mask="solve"))
        print(f"[batched] request {i} grid {p.nx}x{p.ny}x{p.nz} Gr {p.Gr:.3g}: "
              f"oracle |R|/|R0| = {r / r0:.3e}, newton {rep['newton_its']}")
        assert r <= 1e-8 * r0 * 1.0001, (i, r / r0)
        assert np.array_equal(x, alone[i]), f"request {i} differs alone vs in the mix"
    # the requests' linear solves shared engine steps
    assert steps_mix < 0.8 * steps_alone


def test_batched_server_with_requests_that_have_no_multigrid(fe):
    """Grids without a multigrid hierarchy (a three-element-thick slab, a 3^3
    cube) run their block-Jacobi FGMRES on their worker while the others share
    engine steps."""
    probs = [inputs.scaled_config(16, 16, 16, 1e4, seed=61),
             inputs.scaled_config(20, 20, 3, 1e3, seed=62),
             inputs.scaled_config(3, 3, 3, 1e3, seed=63),
             inputs.scaled_config(24, 24, 24, 3e3, seed=64)]
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed")
    alone = []
    with fe.Server(2 << 30, max_active=1, batched=True) as srv:
        for p in probs:
            rc, x, rep = srv.wait(_submit(fe, srv, p, opts))
            assert rc == fe.FE_OK, rep
            alone.append((x, rep))
    with fe.Server(4 << 30, max_active=4, batched=True) as srv:
        res = [srv.wait(t) for t in [_submit(fe, srv, p, opts) for p in probs]]
    for i, ((rc, x, rep), p) in enumerate(zip(res, probs)):
        assert rc == fe.FE_OK, (i, rep)
        assert (rep["mg_levels"] >= 2) == (i in (0, 3)), (i, rep["mg_levels"])
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        assert r0 > 0.0
        r = np.linalg.norm(oracle.residual(p, x, mask="solve"))
        print(f"[batched] {p.nx}x{p.ny}x{p.nz}: levels {rep['mg_levels']}, oracle |R|/|R0| = {r / r0:.3e}")
        assert r <= 1e-8 * r0 * 1.0001, (i, r / r0)
        assert np.array_equal(x, alone[i][0]), f"request {i} differs alone vs in the mix"


@pytest.mark.parametrize("prec,restart", [("mixed", 5), ("fp64", 8), ("pc32", 8)])
def test_batched_server_short_restarts(fe, prec, restart):
    """Cycles that end at the restart length: the engine finishes a cycle's last
    Hessenberg column from the candidate's dot products alone (the delayed
    Gram-Schmidt), then restarts from the true residual.  (At restart 3 two of
    these four systems stagnate, in the one-problem solver as well: restarted
    GMRES with so short a cycle does not converge on them.)"""
    reqs = inputs.serving_trace(n_requests=4, seed=4200, sizes=(16, 24))
    probs = [inputs.request_problem(r) for r in reqs]
    opts = _opts(fe, prec, restart=restart)
    alone = []
    with fe.Server(2 << 30, max_active=1, batched=True) as srv:
        for p in probs:
            rc, x, rep = srv.wait(_submit(fe, srv, p, opts))
            assert rc == fe.FE_OK, rep
            alone.append(x)
    with fe.Server(4 << 30, max_active=4, batched=True) as srv:
        res = [srv.wait(t) for t in [_submit(fe, srv, p, opts) for p in probs]]
    # the default server runs the one-problem FGMRES: the same method, its
    # reductions chunked differently, so the same iterations up to rounding
    with fe.Server(4 << 30, max_active=2) as srv:
        ref = [srv.wait(t) for t in [_submit(fe, srv, p, opts) for p in probs]]
    for i, ((rc, x, rep), p) in enumerate(zip(res, probs)):
        assert rc == fe.FE_OK, (i, rep)
        its = rep["lin_its"][:rep["newton_its"]]
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        r = np.linalg.norm(oracle.residual(p, x, mask="solve"))
        rc_d, x_d, rep_d = ref[i]
        its_d = rep_d["lin_its"][:rep_d["newton_its"]]
        dx = np.linalg.norm(x - x_d) / np.linalg.norm(x_d)
        print(f"[batched] restart {restart} {prec} {p.nx}^3: lin {its} (default server {its_d}), "
              f"oracle |R|/|R0| = {r / r0:.3e}, |x - x_default| / |x_default| = {dx:.1e}")
        assert max(its) > restart, "no cycle reached the restart length"
        assert r <= 1e-8 * r0 * 1.0001, (i, r / r0)
        assert np.array_equal(x, alone[i]), f"request {i} differs alone vs in the mix"
        assert rc_d == fe.FE_OK and len(its_d) == len(its), (its, its_d)
        assert all(abs(a - b) <= 1 for a, b in zip(its, its_d)), (its, its_d)
        assert dx <= 1e-6, dx
