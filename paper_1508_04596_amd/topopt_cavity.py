"""Topology optimisation of the paper's heat-sink cavity on one GPU.

Quarter domain of the closed cubic cavity (Sec. "Numerical examples"), N
elements per unit length (N/2 x N/2 x N elements), design box 0.75^3 on the
heat-source block, volume fraction 5 %, filter radius 2.5 h, the five-step
continuation of Sec. "Continuation scheme".  Prints one line per design
iteration and a JSON summary line.

    python -m paper_1508_04596_amd.topopt_cavity --N 64 --Gr 1e4 --iters 20,20,20,20,20
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--Gr", type=float, default=1e4)
    ap.add_argument("--iters", default="20,20,20,20,20", help="iterations per continuation step")
    ap.add_argument("--vf", type=float, default=0.05)
    ap.add_argument("--rtol", type=float, default=1e-4, help="Newton tolerance (relative)")
    ap.add_argument("--mixed", action="store_true", help="FP32 Krylov operator in the state solves")
    ap.add_argument("--pc32", action="store_true",
                    help="FP32 preconditioner under the FP64 operator in the state and adjoint solves")
    ap.add_argument("--save", default="", help="write the final design (npy)")
    args = ap.parse_args()

    import torch
    from paper_1508_04596_amd import fe, inputs

    p = inputs.cavity_problem(args.N, args.Gr, vf=args.vf)
    iters = [int(v) for v in args.iters.split(",")]
    prob = fe.Problem.from_inputs(p, mask="solve")
    dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    design = dev(p.design.astype(np.uint8), torch.uint8)
    gfix, s = dev(p.gamma), dev(p.s)
    pc = "fp32" if args.pc32 else "fp64"
    opts = fe.topopt_opts(vf=args.vf, n_steps=len(iters), iters_per_step=iters,
                          state=dict(rtol_newton=args.rtol, pc_prec=pc,
                                     krylov_op_prec="mixed" if args.mixed else "fp64"),
                          adjoint=dict(pc_prec=pc))
    T = fe.TopOpt(prob, design, gfix, s, opts)
    rho = dev(np.where(p.design, 1.0 - args.vf, 0.0))
    x = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    hist = []
    for k, n in enumerate(iters):
        ph = fe.make_phys(p.Pr, p.Gr, p.Ck, opts.q_f[k], opts.alpha_max[k], opts.q_alpha[k], p.eg)
        prob.set_phys(ph)
        for _ in range(n):
            r = T.step(rho, x)
            r["step"] = k
            hist.append(r)
            print(f"step {k} it {r['iter']:4d} f {r['f']:.6e} g {r['g']:+.2e} change {r['change']:.3f} "
                  f"newton {r['newton_its']} lin {r['lin_its']} adj {r['adj_its']} "
                  f"ramp {r['ramp_stages']} {r['t_total_s'] * 1e3:.0f} ms", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.save:
        np.save(args.save, rho.cpu().numpy())
    n = len(hist)
    summary = {"N": args.N, "elements": p.n_el, "dof": p.n_dof, "design_elements": int(p.design.sum()),
               "Gr": args.Gr, "iterations": n, "wall_s": wall, "s_per_iteration": wall / max(n, 1),
               "f_first": hist[0]["f"] if hist else None, "f_last": hist[-1]["f"] if hist else None,
               "g_last": hist[-1]["g"] if hist else None,
               "mean_newton": float(np.mean([h["newton_its"] for h in hist])) if hist else None,
               "mean_lin": float(np.mean([h["lin_its"] for h in hist])) if hist else None,
               "mean_state_s": float(np.mean([h["t_state_s"] for h in hist])) if hist else None,
               "mean_adjoint_s": float(np.mean([h["t_adjoint_s"] for h in hist])) if hist else None}
    print(json.dumps(summary), flush=True)
    T.close()
    prob.close()


if __name__ == "__main__":
    main()
