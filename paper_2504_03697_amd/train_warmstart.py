#!/usr/bin/env python
"""Train the warm-start network on (rhs, pressure) pairs produced by the
plain solver, then measure what it saves on held-out right-hand sides.

Workload (defaults): 128^3 grid; training pairs from seeded Gaussian-smoothed
random right-hand sides (sigma = 3 cells) and from lid-driven-cavity time
steps at Re = 100, 400, 1000, 2000; held-out set of smoothed right-hand sides
(other seeds) and cavity steps 51..100 at Re = 1000.  Every pair is solved on
the GPU by FP64 CG to a relative residual of 1e-10.  The library forms each
pair (cfd_net_training_pair): input = b / rms(b), target = (p - mean p) /
rms(p - mean p).  The network is bias-free, hence positively homogeneous, so
the input scale loses nothing; the solver rescales the prediction by the
A-optimal factor, so only the target's shape matters, and unit RMS keeps
every pair's loss at the same scale (a target scaled by rms(b) alone grows
like the square of the grid size for smooth right-hand sides).  Training:
Adam on the mean squared error, in the library's own bfloat16 matrix-core
kernels.

Evaluation on every held-out right-hand side: the energy-norm ratio
||x* - gamma y||_A / ||x*||_A of the learned start (gamma the A-optimal
scale; 1 = no better than the zero guess), and FP64 CG from the learned
start against the zero guess (iterations and time).  Prints progress lines
and one JSON summary (also written to --summary); writes the weights
(float32 .npy) to --out.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def log(msg):
    print(f"[train] {msg}", flush=True)


def cavity_dt(n, nu, cap=0.005):
    h = 1.0 / n
    return min(cap, 0.9 * h * h / (6.0 * nu)) if nu > 0 else cap


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--smoothed", type=int, default=1800, help="training pairs from smoothed random rhs")
    ap.add_argument("--cavity-steps", type=int, default=50, help="cavity steps per Reynolds number")
    ap.add_argument("--heldout-smoothed", type=int, default=150)
    ap.add_argument("--heldout-cavity", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-train-seconds", type=float, default=1e9)
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "warmstart.npy"))
    ap.add_argument("--summary", default=os.path.join(HERE, "weights", "warmstart_eval.json"))
    args = ap.parse_args()

    import torch

    import paper_2504_03697_amd as m
    import synth

    torch.cuda.set_device(0)
    n = args.n
    nv = n ** 3
    A = m.assemble(n, 0)
    t_all = time.perf_counter()

    def solve_pair(b):
        m.rhs_prepare(A, b)
        x, info = m.solve(A, b, tol=1e-10, precision="fp64", formulation="projected")
        assert info["status"] == 0
        return x

    init = np.load(args.init) if args.init else synth.net_init(args.seed)
    net = m.Net(init)

    def normalise(b, p):
        return net.training_pair(n, b, p)

    # ---------------------------------------------------------- training pairs
    X, Y = [], []
    t0 = time.perf_counter()
    if args.epochs == 0:  # evaluate the initial weights only
        args.smoothed, args.cavity_steps = 0, 0
    for i in range(args.smoothed):
        b = synth.smoothed_rhs_torch(n, 10000 + i)
        p = solve_pair(b)
        xi, yi = normalise(b, p)
        X.append(xi)
        Y.append(yi)
        if (i + 1) % 200 == 0:
            log(f"smoothed pairs {i + 1}/{args.smoothed} ({time.perf_counter() - t0:.0f} s)")
    for re_ in ((100, 400, 1000, 2000) if args.cavity_steps > 0 else ()):
        nu = 1.0 / re_
        S = m.State(n, nu=nu, lid_u=1.0, keep_rhs=True)
        dt = cavity_dt(n, nu)
        for s in range(args.cavity_steps):
            m.step(S, dt, tol=1e-10, formulation="projected")
            xi, yi = normalise(S.rhs, S.p)
            X.append(xi)
            Y.append(yi)
        log(f"cavity Re={re_}: {args.cavity_steps} pairs (dt={dt:.2e}, {time.perf_counter() - t0:.0f} s)")
    npairs = len(X)
    log(f"{npairs} training pairs in {time.perf_counter() - t0:.0f} s")

    # ---------------------------------------------------------- held-out set
    HB = []
    for i in range(args.heldout_smoothed):
        b = synth.smoothed_rhs_torch(n, 20000 + i)
        m.rhs_prepare(A, b)
        HB.append(b)
    S = m.State(n, nu=1e-3, lid_u=1.0, keep_rhs=True)
    dt = cavity_dt(n, 1e-3)
    for s in range(50 + args.heldout_cavity):
        m.step(S, dt, tol=1e-10, formulation="projected")
        if s >= 50:
            HB.append(S.rhs.clone())
    log(f"{len(HB)} held-out right-hand sides")

    # ---------------------------------------------------------- training
    rng = np.random.default_rng(args.seed)
    xb = torch.empty(args.batch * nv, dtype=torch.float32, device="cuda")
    yb = torch.empty_like(xb)
    t1 = time.perf_counter()
    losses = []
    steps = 0
    stop = False
    for ep in range(args.epochs):
        order = rng.permutation(npairs)
        tot = 0.0
        nb = 0
        for k in range(0, npairs - args.batch + 1, args.batch):
            for j in range(args.batch):
                xb[j * nv:(j + 1) * nv] = X[order[k + j]]
                yb[j * nv:(j + 1) * nv] = Y[order[k + j]]
            tot += net.train_step(n, xb, yb, args.lr, batch=args.batch)
            nb += 1
            steps += 1
            if time.perf_counter() - t1 > args.max_train_seconds:
                stop = True
                break
        losses.append(tot / max(nb, 1))
        log(f"epoch {ep + 1}: mean loss {losses[-1]:.5f} ({steps} steps, {time.perf_counter() - t1:.0f} s)")
        if stop:
            log("training time budget reached")
            break
    train_s = time.perf_counter() - t1
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, net.params())
    log(f"weights written to {args.out}")

    # ---------------------------------------------------------- evaluation
    # energy-norm ratio of the learned start on the pinned system A x* = b:
    # ||x* - gamma y||_A^2 = b^T x* - (b^T y)^2 / (y^T A y), y[pin] = 0
    ratios = []
    for b in HB:
        xs, info = m.solve(A, b, tol=1e-12, precision="fp64")
        y = net.forward(n, b)
        y[0] = 0.0
        ay = m.spmv(A, y)
        bx, by, yay = float(torch.dot(b, xs)), float(torch.dot(b, y)), float(torch.dot(y, ay))
        ratios.append(float(np.sqrt(max(0.0, 1.0 - by * by / (yay * bx)))) if yay > 0 and bx > 0 else 1.0)
    ratios = np.array(ratios)
    log(f"energy-norm ratio ||x* - gamma y||_A / ||x*||_A: mean {ratios.mean():.4f}, "
        f"median {np.median(ratios):.4f}, min {ratios.min():.4f}, max {ratios.max():.4f}")
    res = {"a_norm_ratio": {"mean": float(ratios.mean()), "median": float(np.median(ratios)),
                            "min": float(ratios.min()), "max": float(ratios.max()),
                            "smoothed_mean": float(ratios[:args.heldout_smoothed].mean()),
                            "cavity_mean": float(ratios[args.heldout_smoothed:].mean())
                            if len(ratios) > args.heldout_smoothed else None}}
    for form in ("pinned", "projected"):
        it0, it1, t0s, t1s, fb = [], [], [], [], 0
        for b in HB:
            torch.cuda.synchronize()
            _, i0 = m.solve(A, b, tol=1e-10, precision="fp64", formulation=form)
            _, i1 = m.solve(A, b, tol=1e-10, precision="fp64", formulation=form, net=net)
            assert i0["status"] == 0 and i1["status"] == 0 and i1["rel_residual"] <= 1e-10
            it0.append(i0["iters"])
            it1.append(i1["iters"])
            t0s.append(i0["seconds"])
            t1s.append(i1["seconds"])
            fb += i1["used_fallback"]
        it0, it1 = np.array(it0), np.array(it1)
        res[form] = {"iters_zero_guess_mean": float(it0.mean()), "iters_learned_mean": float(it1.mean()),
                     "iters_saved_mean": float((it0 - it1).mean()),
                     "iters_saved_frac": float((it0 - it1).sum() / it0.sum()),
                     "seconds_zero_guess_mean": float(np.mean(t0s)), "seconds_learned_mean": float(np.mean(t1s)),
                     "time_ratio": float(np.sum(t1s) / np.sum(t0s)), "fallbacks": int(fb)}
        log(f"{form}: zero guess {it0.mean():.1f} it, learned {it1.mean():.1f} it, "
            f"saved {res[form]['iters_saved_frac'] * 100:.2f} %, time ratio {res[form]['time_ratio']:.3f}")
    summary = {"grid": n, "pairs": npairs, "epochs_run": len(losses), "steps": steps, "batch": args.batch,
               "lr": args.lr, "train_seconds": round(train_s, 1), "loss_first_epoch": losses[0] if losses else None,
               "loss_last_epoch": losses[-1] if losses else None, "heldout": len(HB), "eval": res,
               "total_seconds": round(time.perf_counter() - t_all, 1),
               "target": "(p - mean p) / rms(p - mean p)", "input": "b / rms(b)"}
    with open(args.summary, "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
