"""Continuous-batching server: results alone vs in a mix, memory admission,
failure isolation, correctness against the oracle's residual."""
import time

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


def submit(fe, srv, p, opts):
    ph = fe.make_phys(p.Pr, p.Gr, p.Ck, p.qf, p.alpha_max, p.q_alpha, p.eg)
    return srv.submit(p.nx, p.ny, p.nz, p.h, ph, p.gamma, p.s, opts)


def test_same_result_alone_and_in_the_mix(fe):
    reqs = inputs.serving_trace(n_requests=12, seed=4000)
    probs = [inputs.request_problem(r) for r in reqs]
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed")
    alone = {}
    with fe.Server(4 << 30, max_active=1) as srv:
        for i in range(len(probs)):
            t = submit(fe, srv, probs[i], opts)
            rc, x, rep = srv.wait(t)
            assert rc == fe.FE_OK, rep
            alone[i] = x
    with fe.Server(4 << 30, max_active=6) as srv:
        tickets = [submit(fe, srv, p, opts) for p in probs]
        res = [srv.wait(t) for t in tickets]
        times = [srv.times(t) for t in tickets]
    for i, (rc, x, rep) in enumerate(res):
        p = probs[i]
        assert rc == fe.FE_OK, (i, rep)
        r0 = np.linalg.norm(oracle.residual(p, np.zeros(p.n_dof), mask="solve"))
        r = np.linalg.norm(oracle.residual(p, x, mask="solve"))
        assert r <= 1e-8 * r0 * 1.0001, (i, r / r0)
    # every request of the mix is bitwise the same as when served alone
    for i, x in alone.items():
        assert np.array_equal(res[i][1], x), f"request {i} differs alone vs in the mix"
    assert len(alone) == len(probs)
    # several requests were on the GPU at the same time
    overlaps = sum(1 for a in range(len(times)) for b in range(a + 1, len(times))
                   if times[a][1] < times[b][2] and times[b][1] < times[a][2])
    print(f"[serve] overlapping request pairs: {overlaps}")
    assert overlaps > 0


def test_admission_by_memory_budget(fe):
    p = inputs.scaled_config(32, 32, 32, 1e4, seed=5)
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed")
    fp = fe.fe_solve_footprint_bytes(32, 32, 32, p.h, opts)
    # room for one 32^3 request at a time, even with 4 worker slots
    with fe.Server(int(fp * 1.6), max_active=4) as srv:
        tickets = [submit(fe, srv, p, opts) for _ in range(3)]
        res = [srv.wait(t) for t in tickets]
        times = [srv.times(t) for t in tickets]
    assert all(r[0] == fe.FE_OK for r in res)
    for k in range(1, 3):
        assert times[k][1] >= times[k - 1][2] - 1e-6, "admitted before memory was released"
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[1][1], res[2][1])


def test_failing_request_is_isolated(fe):
    good = inputs.scaled_config(16, 16, 16, 1e4, seed=9)
    bad = inputs.scaled_config(16, 16, 16, 1e4, seed=10)
    bad.gamma[123] = np.nan
    opts = fe.solve_opts(rtol_newton=1e-8)
    with fe.Server(2 << 30, max_active=3) as srv:
        t1 = submit(fe, srv, good, opts)
        t2 = submit(fe, srv, bad, opts)
        t3 = submit(fe, srv, good, opts)
        r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
        errs = [srv.error(t) for t in (t1, t2, t3)]
    print(f"[serve] statuses {r1[0]} {r2[0]} {r3[0]} errors {errs}")
    assert r1[0] == fe.FE_OK and r3[0] == fe.FE_OK
    assert r2[0] == fe.FE_ENAN
    assert np.array_equal(r1[1], r3[1])


def test_oversized_request_is_refused(fe):
    p = inputs.scaled_config(48, 48, 48, 1e4, seed=11)
    with fe.Server(64 << 20, max_active=2) as srv:
        t = submit_enomem = srv.submit(p.nx, p.ny, p.nz, p.h, fe.make_phys(Gr=p.Gr), p.gamma, p.s,
                                       fe.solve_opts(), allow_enomem=True)
        rc, _, _ = srv.poll(t)
        assert rc == fe.FE_ENOMEM and submit_enomem == t


@pytest.mark.parametrize("prec,pc", [("fp64", "multigrid"), ("mixed", "multigrid"),
                                     ("fp64", "bjacobi")])
def test_no_read_before_write_with_poisoned_memory(fe, monkeypatch, prec, pc):
    """Every buffer a solve uses is filled with NaN bytes when allocated; the
    solve must still succeed and give the result of a clean run."""
    p = inputs.scaled_config(16, 16, 16, 1e4, seed=12)
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec, precond=pc, max_lin=400)
    with fe.Server(1 << 30, max_active=1) as srv:
        clean = srv.wait(submit(fe, srv, p, opts))
    monkeypatch.setenv("FE_ARENA_POISON", "1")
    with fe.Server(1 << 30, max_active=1) as srv:
        t = submit(fe, srv, p, opts)
        poisoned = srv.wait(t)
        err = srv.error(t)
    assert clean[0] == fe.FE_OK and poisoned[0] == fe.FE_OK, err
    assert np.array_equal(clean[1], poisoned[1])


def test_warm_start_from_previous_design(fe):
    """A request started from the converged state of the same design needs no
    Newton step and returns that state; a request for a slightly changed design
    (as between optimisation iterations) started from the previous state begins
    closer than from zero and converges to the same absolute tolerance."""
    p1 = inputs.scaled_config(24, 24, 24, 1e4, seed=31, extra_passes=1)
    rng = np.random.default_rng(3)
    p2 = inputs.scaled_config(24, 24, 24, 1e4, seed=31, extra_passes=1)
    p2.gamma = np.clip(p1.gamma + 1e-3 * rng.standard_normal(p1.n_el), 0.0, 1.0)
    p2.gamma[p1.s > 0] = 0.0
    opts = fe.solve_opts(rtol_newton=1e-8)
    ph1 = fe.make_phys(p1.Pr, p1.Gr, p1.Ck, p1.qf, p1.alpha_max, p1.q_alpha, p1.eg)
    ph2 = fe.make_phys(p2.Pr, p2.Gr, p2.Ck, p2.qf, p2.alpha_max, p2.q_alpha, p2.eg)
    with fe.Server(2 << 30, max_active=2) as srv:
        rc1, x1, r1 = srv.wait(submit(fe, srv, p1, opts))
        assert rc1 == fe.FE_OK
        same_opts = fe.solve_opts(rtol_newton=1e-8, atol_newton=1e-8 * r1["res0"])
        same = srv.wait(srv.submit(p1.nx, p1.ny, p1.nz, p1.h, ph1, p1.gamma, p1.s, same_opts, x0=x1))
        cold = srv.wait(submit(fe, srv, p2, opts))
        warm_opts = fe.solve_opts(rtol_newton=1e-8, atol_newton=1e-8 * cold[2]["res0"])
        warm = srv.wait(srv.submit(p2.nx, p2.ny, p2.nz, p2.h, ph2, p2.gamma, p2.s, warm_opts, x0=x1))
    assert same[0] == fe.FE_OK and same[2]["newton_its"] == 0 and np.array_equal(same[1], x1)
    assert cold[0] == fe.FE_OK and warm[0] == fe.FE_OK
    print(f"[serve] warm start: cold newton {cold[2]['newton_its']} lin {cold[2]['lin_its_total']}, "
          f"warm newton {warm[2]['newton_its']} lin {warm[2]['lin_its_total']}; initial residual "
          f"{cold[2]['res0']:.3e} -> {warm[2]['res0']:.3e}")
    assert warm[2]["res0"] < cold[2]["res0"]
    assert warm[2]["newton_its"] <= cold[2]["newton_its"]
    r0 = np.linalg.norm(oracle.residual(p2, np.zeros(p2.n_dof), mask="solve"))
    for x in (cold[1], warm[1]):
        assert np.linalg.norm(oracle.residual(p2, x, mask="solve")) <= 1e-8 * r0 * 1.0001


def test_burst_into_a_tight_budget_all_succeed(fe):
    """A burst of mixed-size requests into an arena that holds only a few of
    them at a time: requests of different sizes finish in a different order
    than they started, so the arena's free space breaks up; every request must
    still get its memory (it waits for a free block instead of failing)."""
    reqs = inputs.serving_trace(n_requests=40, rate_per_s=1000.0, seed=4100,
                                sizes=(16, 24, 32))
    probs = [inputs.request_problem(r) for r in reqs]
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed")
    big = fe.fe_solve_footprint_bytes(32, 32, 32, 1.0 / 32, opts)
    with fe.Server(int(2.5 * big), max_active=8) as srv:
        tickets = [submit(fe, srv, p, opts) for p in probs]
        res = [srv.wait(t) for t in tickets]
        errs = [srv.error(t) for t in tickets]
    failed = [(i, rc, e) for i, ((rc, _, _), e) in enumerate(zip(res, errs)) if rc != fe.FE_OK]
    print(f"[serve] burst of {len(probs)}: {len(failed)} failed {failed[:3]}")
    assert not failed


def test_request_with_ramping_fits_its_block(fe):
    """With heat-source ramping enabled the solve keeps two more buffers; the
    request's block (sized by the footprint) must hold them."""
    p = inputs.scaled_config(16, 16, 16, 1e4, seed=13)
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed", ramp_steps=2)
    fp = fe.fe_solve_footprint_bytes(16, 16, 16, p.h, opts)
    assert fp > fe.fe_solve_footprint_bytes(16, 16, 16, p.h,
                                            fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed"))
    with fe.Server(1 << 30, max_active=2) as srv:
        t = submit(fe, srv, p, opts)
        rc, x, rep = srv.wait(t)
        err = srv.error(t)
    assert rc == fe.FE_OK, err


def test_smaller_requests_pass_a_blocked_head_a_bounded_number_of_times(fe):
    """A 32^3 request at the head of the queue that does not fit next to the
    16^3 request already running: later 16^3 requests that fit are admitted
    past it, at most max_active of them, then the head is admitted; every
    result is the same as when solved alone."""
    small = inputs.scaled_config(16, 16, 16, 1e4, seed=21)
    big = inputs.scaled_config(32, 32, 32, 1e4, seed=22)
    opts = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed")
    fs = fe.fe_solve_footprint_bytes(16, 16, 16, small.h, opts)
    fb = fe.fe_solve_footprint_bytes(32, 32, 32, big.h, opts)
    # the big one fits only with no small one running (blocks carry about 1 %
    # plus 1 MiB of margin over the footprint), two small ones fit together
    budget = int(fb + 0.5 * fs) + (8 << 20)
    assert budget < fb + fs and budget > 2 * fs
    max_active = 3
    with fe.Server(4 << 30, max_active=1) as srv:
        alone_small = srv.wait(submit(fe, srv, small, opts))[1]
        alone_big = srv.wait(submit(fe, srv, big, opts))[1]
    with fe.Server(budget, max_active=max_active) as srv:
        t0 = submit(fe, srv, small, opts)
        tb = submit(fe, srv, big, opts)
        later = [submit(fe, srv, small, opts) for _ in range(8)]
        res = {t: srv.wait(t) for t in [t0, tb] + later}
        times = {t: srv.times(t) for t in res}
    assert all(r[0] == fe.FE_OK for r in res.values())
    passed = [t for t in later if times[t][1] < times[tb][1]]
    print(f"[serve] later requests admitted before the blocked head: {len(passed)}")
    assert 1 <= len(passed) <= max_active
    assert np.array_equal(res[tb][1], alone_big)
    for t in [t0] + later:
        assert np.array_equal(res[t][1], alone_small)
