#!/usr/bin/env python
"""Run the lid-driven cavity on one GPU and report every pressure solve.

Each step is the library's fractional step (cfd_step): forces, semi-
Lagrangian advection, explicit viscosity, then the pressure-Poisson solve
(the hot path) and the gradient correction.  With --compare the same steps
also run with plain FP64 CG on the pinned matrix from a zero guess, and with
--previous with the solver options under test but started from the previous
step's pressure instead of the network (the non-learned warm start), each
from the same initial state; the report gives iterations, solve times and
the velocity difference to the plain FP64 run after each step.

Example (384^3, Re = 1000, mixed + learned + projected vs plain FP64):
    python run_cavity.py --n 384 --re 1000 --dt 0.001 --steps 20 \\
        --precision mixed --formulation projected --net weights/warmstart.npy --compare --previous
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def log(msg):
    print(f"[cavity] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--re", type=float, default=1000.0)
    ap.add_argument("--dt", type=float, default=None, help="default: min(0.005, 0.9 h^2 / (6 nu))")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--formulation", default="pinned", choices=["pinned", "projected"])
    ap.add_argument("--net", default=None, help="warm-start weights (.npy)")
    ap.add_argument("--precond", default="none", choices=["none", "dic"],
                    help="dic: the DIC preconditioner in red-black order")
    ap.add_argument("--compare", action="store_true", help="also run plain FP64 pinned CG from the same state")
    ap.add_argument("--previous", action="store_true",
                    help="also run the same solver started from the previous step's pressure (no network)")
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2504_03697_amd as m

    torch.cuda.set_device(0)
    n = args.n
    nu = 1.0 / args.re
    h = 1.0 / n
    dt = args.dt if args.dt else min(0.005, 0.9 * h * h / (6 * nu))
    net = m.Net(np.load(args.net)) if args.net else None
    S = m.State(n, nu=nu, lid_u=1.0)
    R = m.State(n, nu=nu, lid_u=1.0) if args.compare else None
    P = m.State(n, nu=nu, lid_u=1.0) if args.previous else None
    log(f"{n}^3, Re={args.re:g}, dt={dt:g}, {args.steps} steps, {args.precision}/{args.formulation}/{args.precond}"
        f"{' + learned warm start' if net else ''}")
    rows = []
    for s in range(args.steps):
        info = m.step(S, dt, tol=args.tol, precision=args.precision, net=net, formulation=args.formulation,
                      precond=args.precond)
        row = {"step": s + 1, "iters": info["iters"], "seconds": round(info["seconds"], 4),
               "rel_residual": info["rel_residual"], "init_residual": info["init_residual"]}
        if P is not None:
            ip = m.step(P, dt, tol=args.tol, precision=args.precision, formulation=args.formulation, guess="previous",
                        precond=args.precond)
            row.update({"prev_iters": ip["iters"], "prev_seconds": round(ip["seconds"], 4),
                        "prev_init_residual": ip["init_residual"]})
        if R is not None:
            ir = m.step(R, dt, tol=args.tol, precision="fp64", formulation="pinned")
            row.update({"fp64_iters": ir["iters"], "fp64_seconds": round(ir["seconds"], 4)})
            scale = max(float(R.u.abs().max()), float(R.v.abs().max()), float(R.w.abs().max()))
            du = max(float((S.u - R.u).abs().max()), float((S.v - R.v).abs().max()), float((S.w - R.w).abs().max()))
            row["max_dvel_rel"] = du / max(scale, 1e-300)
        rows.append(row)
        log(json.dumps(row))
    summ = {"grid": n, "re": args.re, "dt": dt, "steps": args.steps, "precision": args.precision,
            "formulation": args.formulation, "precond": args.precond, "learned": net is not None,
            "solve_seconds": round(sum(r["seconds"] for r in rows), 3),
            "iters_total": int(sum(r["iters"] for r in rows)),
            "max_rel_residual": max(r["rel_residual"] for r in rows)}
    if P is not None:
        summ["prev_solve_seconds"] = round(sum(r["prev_seconds"] for r in rows), 3)
        summ["prev_iters_total"] = int(sum(r["prev_iters"] for r in rows))
    if R is not None:
        summ["fp64_solve_seconds"] = round(sum(r["fp64_seconds"] for r in rows), 3)
        summ["fp64_iters_total"] = int(sum(r["fp64_iters"] for r in rows))
        summ["speedup"] = round(summ["fp64_solve_seconds"] / summ["solve_seconds"], 3)
        summ["max_dvel_rel_final"] = rows[-1]["max_dvel_rel"]
        if P is not None:
            summ["prev_speedup"] = round(summ["fp64_solve_seconds"] / summ["prev_solve_seconds"], 3)
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    main()
