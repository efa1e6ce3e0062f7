"""Benchmark of the matrix-free Newton-Krylov state solve on one MI355X.

Workload: 64x64x64 trilinear hex elements (1,373,125 DOF), Gr = 1e4, Pr = 1,
k_s/k_f = 10, alpha_max = 1e4, q = 1, design from a seeded smoothed Gaussian
random field thresholded to 40 % solid, heat source in the central quarter,
walls no-slip and T = 0, pressure pinned at node 0.

One step = the whole hot path on that input:
  residual, Newton solve to 1e-8 in FP64 (FP64 Krylov operator), J v products
  at the converged state in FP64 and in FP32, Newton solve to 1e-8 in mixed
  precision (FP32 Krylov operator and preconditioner, FP64 refinement).

Prints one JSON line.  ``value`` is the FP64 J v throughput in GDOF/s; the solve
times, the FP32 rate and the mixed-vs-FP64 error ride along.  ``roofline``
describes the FP64 element-pass kernel of J v, timed with HIP events that the
library records around each of its launches on the stream it runs on.
``cpu_baseline`` times the CPU oracle on the host cores: J v and residual on
the same workload, and a full Newton solve of the 8x8x8 workload next to the
GPU solve of the same input.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Floating-point work of one FP64 element J v evaluation: the modal 2x2x2
# Gauss pass (points in pairs that share their y/z sums, both for the values and
# gradients and for the test-side sums), counted from the
# FP64 instructions of that element body built with compile-time Gauss-point
# signs (FMA = 2 flops, add/mul = 1).  The kernel runs the same arithmetic with
# run-time signs: multiplications by +-1 are not counted.
FLOPS_PER_ELEM_JV = 3371.0
# the FP32 J v element body counted the same way (FP32 arithmetic instructions)
FLOPS_PER_ELEM_JV32 = 3306.0
# MI355X FP32 vector peak (packed two-wide); the library is built without
# packed FP32 instructions, which caps its FP32 arithmetic at the unpacked rate
PEAK_FP32_VALU, PEAK_FP32_UNPACKED = 157.3e12, 78.6e12
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12
# HBM traffic per launch of the FP64 J v element-pass kernel, per workload
# (64^3: 1024 tiles; 160x160x320: 32,000 tiles), from two rocprofv3 --pmc runs
# of this script each (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the same counter reads for torch's double->float copy of a
# 1,373,125-entry vector (10,985,000 B read, 5,492,500 B written): reads
# x 1.951, writes x 1.000.  Workloads without counters report null.
ELEM_COUNTERS_KIB = {2: (14235.56, 17217.22), 3: (474297.2, 537499.9)}
FETCH_SCALE, WRITE_SCALE = 1.951, 1.000


def elem_traffic_bytes(config):
    kib = ELEM_COUNTERS_KIB.get(config)
    return None if kib is None else 1024 * (kib[0] * FETCH_SCALE + kib[1] * WRITE_SCALE)


# SHA-256 of csrc/fe_elem.hip when those counters were taken: any other source
# of the element kernel reports traffic as null instead of a stale figure.
ELEM_TRAFFIC_SRC_SHA256 = "8a83cf2f44759beb6b4460b9132ff4ec9a6524d8e8fe4e43b018195342b39045"
SOLVES = "Newton to 1e-8 FP64, mixed and FP64 with an FP32 preconditioner"
WORKLOADS = {
    2: "C2: 64x64x64 elements (1,373,125 DOF), Gr=1e4, 40% solid smoothed random design; "
       "{reps} Jv FP64 + {reps} Jv FP32 at x*, " + SOLVES,
    3: "C3: 160x160x320 elements (41,603,205 DOF), Gr=1e6, 30% solid smoothed random design; "
       "{reps} Jv FP64 + {reps} Jv FP32 at x*, " + SOLVES,
    4: "C4: 96x96x96 elements (4,563,365 DOF), Gr=1e5, 40% solid smoothed random design with "
       "intermediate values; {reps} Jv FP64 + {reps} Jv FP32 at x*, " + SOLVES,
}


# Algorithmic HBM bytes of one FP64 J v: x, v read and J v written (5 values per
# node each), gamma and s read (one value per element each).
def jv_bytes(n_nodes, n_el, word=8):
    return 15 * word * n_nodes + 16 * n_el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jv-reps", type=int, default=1000)
    ap.add_argument("--kernel-reps", type=int, default=200,
                    help="J v launches timed per precision with per-launch events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--max-newton", type=int, default=50)
    ap.add_argument("--max-lin", type=int, default=3000)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving trace (Poisson arrivals, 20/s); 0 = skip")
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="mean arrival rate of the serving trace (requests/s)")
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-max-active", type=int, default=8)
    ap.add_argument("--serve-batched-max-active", type=int, default=256,
                    help="worker slots of the batched (lockstep) server")
    ap.add_argument("--serve-burst-rate", type=float, default=1000.0,
                    help="arrival rate of the burst comparison (default vs batched server); 0 = skip")
    ap.add_argument("--serve-burst-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-sizes", type=str, default="16,24,32,48",
                    help="grid sizes n (n^3 elements) the serving trace draws from, comma-separated")
    ap.add_argument("--serve-prec", default="pc32", choices=("pc32", "mixed", "fp64"),
                    help="precision of the served solves: pc32 (FP64 operator, FP32 V-cycle; "
                         "the fastest), mixed (FP32 operator and V-cycle, FP64 true residuals) "
                         "or fp64")
    ap.add_argument("--serve-only", action="store_true",
                    help="diagnostic: run only the serving legs and print their JSON")
    ap.add_argument("--config", type=int, default=2, choices=(2, 3, 4),
                    help="workload: 2 = 64^3 (the reported line), 3 = 160x160x320 (the "
                         "paper's 41.6 M DOF mesh), 4 = 96^3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is a design, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1508_04596_amd import fe, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serve_only:
        print(json.dumps({"serving": serving_legs(fe, inputs, args)}), flush=True)
        return
    p = inputs.config(args.config)
    prob = fe.Problem.from_inputs(p, mask="solve")
    g = torch.from_numpy(p.gamma).to(dev)
    s = torch.from_numpy(p.s).to(dev)
    n_dof, n_el, n_nodes = p.n_dof, p.n_el, p.n_nodes
    vdir = torch.from_numpy(inputs.random_direction(p, 1, mask=p.mask_solve)).to(dev)
    out64 = torch.empty(n_dof, dtype=torch.float64, device=dev)
    out32 = torch.empty(n_dof, dtype=torch.float32, device=dev)
    r = torch.empty(n_dof, dtype=torch.float64, device=dev)
    vb = 1 if args.verbose else 0
    opts64 = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="fp64", verbose=vb,
                           max_newton=args.max_newton, max_lin=args.max_lin)
    optsmx = fe.solve_opts(rtol_newton=1e-8, krylov_op_prec="mixed", verbose=vb,
                           max_newton=args.max_newton, max_lin=args.max_lin)
    # FP64 operator, basis and residuals with the FP32 preconditioner
    optspc = fe.solve_opts(rtol_newton=1e-8, pc_prec="fp32", verbose=vb,
                           max_newton=args.max_newton, max_lin=args.max_lin)
    stream = torch.cuda.current_stream()

    def step(rec):
        x64 = torch.zeros(n_dof, dtype=torch.float64, device=dev)
        fe.fe_residual(prob, x64, g, s, r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep64 = fe.newton_solve(prob, g, s, x64, opts64, allow_not_converged=True)
        t_solve64 = time.perf_counter() - t0
        # J v at the converged state, FP64 then FP32
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        x32 = x64.float()
        v32 = vdir.float()
        e0.record(stream)
        for _ in range(args.jv_reps):
            fe.fe_jvp(prob, x64, g, s, vdir, out64)
        e1.record(stream)
        for _ in range(args.jv_reps):
            fe.fe_jvp(prob, x32, g, s, v32, out32)
        e2.record(stream)
        # element-pass kernel alone: HIP events recorded by the library around
        # each launch, on the stream the kernel runs on
        fe.fe_kernel_timer(prob, True)
        for _ in range(args.kernel_reps):
            fe.fe_jvp(prob, x64, g, s, vdir, out64)
        ms64, n64 = fe.fe_kernel_timer_read(prob)
        for _ in range(args.kernel_reps):
            fe.fe_jvp(prob, x32, g, s, v32, out32)
        ms32, n32 = fe.fe_kernel_timer_read(prob)
        fe.fe_kernel_timer(prob, False)
        xm = torch.zeros(n_dof, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()  # the J v loops above were queued asynchronously
        t0 = time.perf_counter()
        repmx = fe.newton_solve(prob, g, s, xm, optsmx, allow_not_converged=True)
        t_solvemx = time.perf_counter() - t0
        xp = torch.zeros(n_dof, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reppc = fe.newton_solve(prob, g, s, xp, optspc, allow_not_converged=True)
        t_solvepc = time.perf_counter() - t0
        torch.cuda.synchronize()
        rec.update(t_elem64=ms64 * 1e-3 / max(n64, 1), t_elem32=ms32 * 1e-3 / max(n32, 1),
                   t_jv64=e0.elapsed_time(e1) * 1e-3 / args.jv_reps,
                   t_jv32=e1.elapsed_time(e2) * 1e-3 / args.jv_reps,
                   t_solve64=t_solve64, t_solvemx=t_solvemx, rep64=rep64, repmx=repmx,
                   t_solvepc=t_solvepc, reppc=reppc,
                   mixed_vs_fp64=float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)),
                   pc32_vs_fp64=float(torch.linalg.norm(xp - x64) / torch.linalg.norm(x64)),
                   jv32_vs_jv64=float(torch.linalg.norm(out32.double() - out64) /
                                      torch.linalg.norm(out64)))
        # backward error of the mixed solution measured with the FP64 residual
        fe.fe_residual(prob, xm, g, s, r)
        rec["mixed_res_rel"] = float(torch.linalg.norm(r)) / rep64["res0"]

    rec = {}
    for _ in range(args.warmup):
        step(rec)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rr = {}
        step(rr)
        recs.append(rr)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    t_jv64 = float(np.median([q["t_jv64"] for q in recs]))
    t_jv32 = float(np.median([q["t_jv32"] for q in recs]))
    last = recs[-1]
    value = n_dof / t_jv64 / 1e9

    t_elem64 = float(np.median([q["t_elem64"] for q in recs]))
    t_elem32 = float(np.median([q["t_elem32"] for q in recs]))
    bytes_alg = jv_bytes(n_nodes, n_el)
    achieved = FLOPS_PER_ELEM_JV * n_el / t_elem64
    # the traffic counters were taken per workload, for one source of the kernel
    traffic = elem_traffic_bytes(args.config) if elem_source_sha256() == \
        ELEM_TRAFFIC_SRC_SHA256 else None
    n_tiles = -(-p.nx // 8) * -(-p.ny // 8) * -(-p.nz // 4)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
            "traffic": traffic,
            "kernel": f"k_elem<double,double,JV> (FP64 J v element pass, {n_tiles} tiles of 8x8x4)",
            "kernel_avg_us": t_elem64 * 1e6, "flops_per_elem": FLOPS_PER_ELEM_JV,
            "traffic_GBps": traffic / t_elem64 / 1e9 if traffic else None,
            "jv_alg_bytes": bytes_alg,
            "jv_op_alg_GBps": bytes_alg / t_jv64 / 1e9}
    achieved32 = FLOPS_PER_ELEM_JV32 * n_el / t_elem32
    roof32 = {"bound": "alu", "achieved": achieved32 / 1e12, "peak": PEAK_FP32_VALU / 1e12,
              "unit": "TFLOP/s", "frac": achieved32 / PEAK_FP32_VALU,
              "frac_of_unpacked": achieved32 / PEAK_FP32_UNPACKED,
              "kernel": f"k_elem<float,float,JV> (FP32 J v element pass, {n_tiles} tiles of 8x8x4)",
              "kernel_avg_us": t_elem32 * 1e6, "flops_per_elem": FLOPS_PER_ELEM_JV32}

    serve = serving_legs(fe, inputs, args) if args.serve_requests > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, args.cpu_seconds)
        cpu.update(c1_solves(fe, inputs, dev))

    line = {
        "metric": "Jv GDOF/s + Newton solve time to 1e-8 (FP64 vs mixed); p50/p99 serve latency",
        "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config].format(reps=args.jv_reps),
                   "jv_reps": args.jv_reps},
        "jv_fp64_ms": t_jv64 * 1e3, "jv_fp32_ms": t_jv32 * 1e3,
        "elem_fp64_us": t_elem64 * 1e6, "elem_fp32_us": t_elem32 * 1e6,
        "jv_fp32_gdofs": n_dof / t_jv32 / 1e9, "roofline_fp32": roof32,
        "solve_fp64_s": last["t_solve64"], "solve_mixed_s": last["t_solvemx"],
        "solve_fp64_converged": last["rep64"]["status"] == 0,
        "solve_mixed_converged": last["repmx"]["status"] == 0,
        "solve_fp64_rel_res": last["rep64"]["res_final"] / last["rep64"]["res0"],
        "solve_mixed_rel_res": last["repmx"]["res_final"] / last["repmx"]["res0"],
        "newton_its_fp64": last["rep64"]["newton_its"], "krylov_its_fp64": last["rep64"]["lin_its"],
        "newton_its_mixed": last["repmx"]["newton_its"], "krylov_its_mixed": last["repmx"]["lin_its"],
        "solve_fp64_phase_s": {k: last["rep64"][k] for k in ("t_jv_s", "t_prec_s", "t_orth_s", "t_res_s", "t_setup_s")},
        "solve_mixed_phase_s": {k: last["repmx"][k] for k in ("t_jv_s", "t_prec_s", "t_orth_s", "t_res_s", "t_setup_s")},
        "mixed_vs_fp64_rel": last["mixed_vs_fp64"], "mixed_res_rel": last["mixed_res_rel"],
        "solve_fp64_pc32_s": last["t_solvepc"],
        "solve_fp64_pc32_converged": last["reppc"]["status"] == 0,
        "solve_fp64_pc32_rel_res": last["reppc"]["res_final"] / last["reppc"]["res0"],
        "newton_its_fp64_pc32": last["reppc"]["newton_its"],
        "krylov_its_fp64_pc32": last["reppc"]["lin_its"],
        "solve_fp64_pc32_phase_s": {k: last["reppc"][k] for k in ("t_jv_s", "t_prec_s", "t_orth_s", "t_res_s", "t_setup_s")},
        "pc32_vs_fp64_rel": last["pc32_vs_fp64"],
        "jv32_vs_jv64_rel": last["jv32_vs_jv64"],
        "roofline": roof, "cpu_baseline": cpu, "serving": serve,
    }
    prob.close()
    print(json.dumps(line), flush=True)


_SERVE_PROBS = {}


def serving_legs(fe, inputs, args):
    """The configured trace on the default server (each request's solve on its
    worker's stream) and on the batched one (lockstep FGMRES, one launch per
    kernel over all running requests); then a burst that keeps many requests
    in flight, on both."""
    sizes = tuple(int(v) for v in args.serve_sizes.split(","))
    pr = args.serve_prec
    serve = serve_trace(fe, inputs, args.serve_requests, args.serve_budget_gb,
                        args.serve_max_active, args.serve_rate, sizes=sizes, prec=pr)
    serve["batched"] = serve_trace(fe, inputs, args.serve_requests, args.serve_budget_gb,
                                   args.serve_batched_max_active, args.serve_rate, batched=True,
                                   sizes=sizes, prec=pr)
    if args.serve_burst_rate > 0:
        serve["burst"] = {
            "default": serve_trace(fe, inputs, args.serve_requests, args.serve_burst_budget_gb,
                                   args.serve_max_active, args.serve_burst_rate, sizes=sizes,
                                   prec=pr),
            "batched": serve_trace(fe, inputs, args.serve_requests, args.serve_burst_budget_gb,
                                   args.serve_batched_max_active, args.serve_burst_rate,
                                   batched=True, sizes=sizes, prec=pr)}
    return serve


def serve_trace(fe, inputs, n, budget_gb, max_active, rate=20.0, batched=False,
                sizes=(16, 24, 32, 48), prec="pc32"):
    """Serving workload: n requests with Poisson arrivals (20/s by default), grids uniform
    over sizes^3 ({16,24,32,48}^3 by default), log10 Gr uniform in [3,5], 40 %-solid
    smoothed random designs, solved to 1e-8 (``prec``: mixed, pc32 = FP64 operator with the
    FP32 V-cycle, or fp64); latency = completion - arrival.
    ``batched``: the lockstep server (one launch per kernel over all running requests)."""
    import time as _t
    reqs = inputs.serving_trace(n_requests=n, rate_per_s=rate, seed=4000, sizes=sizes)
    # the requests' grids, designs and Grashof numbers do not depend on the
    # arrival rate (the arrival gaps are drawn first): build them once
    if (n, sizes) not in _SERVE_PROBS:
        _SERVE_PROBS[(n, sizes)] = [inputs.request_problem(r) for r in reqs]
    probs = _SERVE_PROBS[(n, sizes)]
    opts = (fe.solve_opts(rtol_newton=1e-8, pc_prec="fp32") if prec == "pc32" else
            fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec))
    lat, tickets, statuses = [], [], []
    with fe.Server(int(budget_gb * (1 << 30)), max_active=max_active, batched=batched) as srv:
        # warm-up, not timed: one request of each grid size (first use of the
        # kernels and of the server's worker threads and streams)
        seen = {}
        for pr in probs:
            seen.setdefault(pr.nx, pr)
        for pr in seen.values():
            ph = fe.make_phys(pr.Pr, pr.Gr, pr.Ck, pr.qf, pr.alpha_max, pr.q_alpha, pr.eg)
            srv.wait(srv.submit(pr.nx, pr.ny, pr.nz, pr.h, ph, pr.gamma, pr.s, opts))
        steps0, launches0 = srv.engine_stats()
        t0 = _t.perf_counter()
        for r, pr in zip(reqs, probs):
            wait = t0 + r.arrival_s - _t.perf_counter()
            if wait > 0:
                _t.sleep(wait)
            ph = fe.make_phys(pr.Pr, pr.Gr, pr.Ck, pr.qf, pr.alpha_max, pr.q_alpha, pr.eg)
            tickets.append(srv.submit(pr.nx, pr.ny, pr.nz, pr.h, ph, pr.gamma, pr.s, opts))
        for t in tickets:
            rc, _, _ = srv.wait(t)
            statuses.append(rc)
        times = [srv.times(t) for t in tickets]
        steps, launches = srv.engine_stats()
        steps, launches = steps - steps0, launches - launches0
    lat = np.array([d - a for a, _, d in times])
    makespan = max(d for _, _, d in times) - min(a for a, _, _ in times)
    return {"requests": n, "sizes": list(sizes), "prec": prec, "rate_per_s": rate, "budget_gb": budget_gb,
            "max_active": max_active, "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "solves_per_s": n / makespan, "all_converged": all(s == 0 for s in statuses),
            "mode": "batched" if batched else "default",
            "engine_steps": steps, "engine_launches": launches,
            "queue_wait_p50_s": float(np.percentile([b - a for a, b, _ in times], 50))}


def elem_source_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_1508_04596_amd", "csrc", "fe_elem.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def host_cpu():
    """lscpu model name, sockets and physical cores, and the CPUs this process may use."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = dict(line.split(":", 1) for line in out.splitlines() if ":" in line)
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "0") or 0)
        cps = int(kv.get("Core(s) per socket", "0") or 0)
        info["sockets"] = sockets
        info["physical_cores"] = sockets * cps
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    info["cpus_available"] = len(os.sched_getaffinity(0))
    return info


def _timed(fn, seconds):
    fn()  # warm
    n, t0 = 0, time.perf_counter()
    while True:
        fn()
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return n, el


def cpu_baseline(p, seconds):
    """The oracle's FP64 J v and residual on this host's cores (about ``seconds``
    of J v, a third of that for the residual and for J v on one thread)."""
    import oracle
    from paper_1508_04596_amd import inputs
    x = inputs.random_state(p, 2001, mask=p.mask_solve)
    v = inputs.random_direction(p, 1, mask=p.mask_solve)
    n, el = _timed(lambda: oracle.jvp(p, x, v, mask="solve"), seconds)
    nr, elr = _timed(lambda: oracle.residual(p, x, mask="solve"), seconds / 3)
    cores = oracle.num_threads()
    # the same on one thread, a shorter sample
    oracle.set_num_threads(1)
    n1, el1 = _timed(lambda: oracle.jvp(p, x, v, mask="solve"), seconds / 3)
    oracle.set_num_threads(cores)
    return {"value": p.n_dof * n / el / 1e9, "unit": "GDOF/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} FP64 J v products of the CPU oracle on the same {p.nx}x{p.ny}x{p.nz} problem "
                      f"({el:.1f} s)",
            "residual_ms": elr / nr * 1e3,
            "sample_residual": f"{nr} residual evaluations ({elr:.1f} s)",
            "value_1_thread": p.n_dof * n1 / el1 / 1e9,
            "sample_1_thread": f"{n1} products on one thread ({el1:.1f} s)",
            "host": host_cpu()}


def c1_solves(fe, inputs, dev):
    """Newton solve to 1e-8 of the 8x8x8 workload (3,645 DOF, Gr = 1e3): the oracle
    (exact sparse linear solves, all cores) against the GPU (FP64 and mixed, the
    library's default preconditioner), same inputs, medians of several runs."""
    import torch
    from oracle import solve as osolve
    p1 = inputs.config(1)
    t_or = []
    for _ in range(3):
        t0 = time.perf_counter()
        _, it_or, rel_or = osolve.newton(p1, rtol=1e-8)
        t_or.append(time.perf_counter() - t0)
    prob = fe.Problem.from_inputs(p1, mask="solve")
    g = torch.from_numpy(p1.gamma).to(dev)
    s = torch.from_numpy(p1.s).to(dev)
    out = {"c1_oracle_solve_s": float(np.median(t_or)), "c1_oracle_newton_its": it_or,
           "c1_oracle_rel_res": rel_or}
    for prec in ("fp64", "mixed"):
        ts = []
        for _ in range(5):
            x = torch.zeros(p1.n_dof, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = fe.newton_solve(prob, g, s, x, fe.solve_opts(rtol_newton=1e-8, krylov_op_prec=prec))
            ts.append(time.perf_counter() - t0)
        out[f"c1_gpu_{prec}_solve_s"] = float(np.median(ts))
        out[f"c1_gpu_{prec}_newton_its"] = rep["newton_its"]
    prob.close()
    return out


if __name__ == "__main__":
    main()
