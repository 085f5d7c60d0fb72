#!/usr/bin/env python
"""Benchmark of the pressure-Poisson hot path on one MI355X.

A step is one pass of the whole hot path over one synthetic right-hand side
at 256^3 (16.8M unknowns, 117M nonzeros): right-hand-side preparation,
learned warm start (when trained weights are present), and the mixed
FP32/FP64 reliable-update CG solve (projected formulation) to a relative
residual of 1e-10.  (The library's default stopping margin, which the 1e-9
pressure-error bar needs on rough right-hand sides, takes the mixed solve on
to 0.05 * 1e-10 only when b^T A b / b^T b > 0.5; these smoothed right-hand
sides are at ~0.16 and stop at 1e-10.  The same solves with the margin
forced are reported beside them.)  The value is the mean time-to-tolerance
per solve.  The
same right-hand sides are then solved by plain FP64 CG on the pinned matrix
(the plain method), by FP64 CG in the projected formulation, by the mixed
solver without the network, and with the paper's DIC preconditioner in
red-black order (mixed, mixed + network, FP64), for the comparison factors;
the CG SpMV kernel's launches inside the timed solves are timed with HIP
events for the roofline.

Prints ONE JSON line.  --gpus N > 1 is rejected: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def a_kernel_bytes(n, nnz, mixed):
    """Algorithmic bytes of one launch of the CG SpMV kernel (normal mode).

    CSR: row pointers 4(n+1), columns 4 nnz, values 4 nnz (both kernels read
    the float32 copy of the values, which are small integers and exact).
    Vectors per row: read r and p_old, write p_new and q (float32 in the
    mixed kernel, float64 otherwise); the float64 kernel also reads and
    writes x (the mixed path applies its queued x updates in the vector
    kernel that follows).
    """
    w = 4 if mixed else 8
    return 4 * (n + 1) + nnz * 8 + 4 * w * n + (0 if mixed else 16 * n)


def s_product_bytes(n3, w=4):
    """Algorithmic bytes of one product with the Schur complement on an N^3
    grid in red-black order (projected formulation, float32 values, vectors
    of w bytes): the red sweep reads its rows' CSR (row pointers, columns,
    values = diagonal + in-domain neighbours), z and p_old of the black cells
    and writes y and the new direction; the black sweep reads its rows' CSR,
    the direction and the gathered y, and writes q."""
    n = n3 ** 3
    nr = (n + 1) // 2
    nb = n - nr
    edges = 3 * n3 * n3 * (n3 - 1)
    red = 4 * (nr + 1) + 8 * (nr + edges) + 2 * w * nb + w * nr + w * nb
    black = 4 * (nb + 1) + 8 * (nb + edges) + w * nb + w * nr + w * nb
    return red + black


def kernel_source_sha():
    """Hash of the sources the CG kernels are built from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_03697_amd", "csrc")
    for f in ("cg.hip", "common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, grid):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (profiles/*.md, line 'traffic-json: {...}'), or None when no summary
    matches the current kernel sources."""
    sha = kernel_source_sha()
    for md in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(md) as fh:
            for line in fh:
                if not line.startswith("traffic-json: "):
                    continue
                d = json.loads(line[len("traffic-json: "):])
                if d.get("kernel") == kernel and d.get("grid") == grid and d.get("source_sha") == sha:
                    return d["bytes_per_launch"]
    return None


def spmv_bytes(n, nnz, w):
    """Plain SpMV y = A x with vectors of w bytes: CSR (float32 values in
    both precisions) + x read once + y written once."""
    return 4 * (n + 1) + nnz * 8 + 2 * w * n


def spmv_sym_bytes(n, nnz, w):
    """y = A x from the symmetric storage: two row-pointer arrays, the
    diagonal and upper entries (column + float32 value), the lower entries'
    columns, x read once and y written once (the looked-up lower values are
    entries already counted in the upper storage)."""
    nnz_l = (nnz - n) // 2
    nnz_u = nnz - nnz_l
    return 8 * (n + 1) + 8 * nnz_u + 4 * nnz_l + 2 * w * n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dic", action="store_true", help="skip the DIC-preconditioned comparison solves")
    ap.add_argument("--net", default=os.path.join(ROOT, "paper_2504_03697_amd", "weights", "warmstart.npy"))
    ap.add_argument("--workload", choices=("solve", "step"), default="solve",
                    help="solve: the headline Poisson solves; step: cavity time steps (for the step kernels)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on a single GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "step":
        return step_workload(args)

    import numpy as np
    import torch

    import paper_2504_03697_amd as m
    import synth

    torch.cuda.set_device(0)
    n = args.n
    nrows = n ** 3
    A = m.assemble(n, 0)
    log(f"assembled {n}^3: n={A.n} nnz={A.nnz}")

    net = None
    if os.path.exists(args.net):
        net = m.Net(np.load(args.net))
        log(f"warm-start network loaded from {args.net}")

    seeds = [1000 + i for i in range(args.warmup + args.steps)]
    rhs = []
    for s in seeds:
        rhs.append(torch.from_numpy(synth.smoothed_rhs(n, s)).cuda())
    torch.cuda.synchronize()
    log(f"{len(rhs)} right-hand sides resident in HBM")

    def run(b, precision, use_net, form="projected", precond="none", margin=0.0):
        m.rhs_prepare(A, b)
        x, info = m.solve(A, b, tol=args.tol, precision=precision, net=net if use_net else None, timing=True,
                          formulation=form, precond=precond, stop_margin=margin)
        return x, info

    for i in range(args.warmup):
        run(rhs[i], "mixed", True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    xs_head = []
    for i in range(args.warmup, len(rhs)):
        x, info = run(rhs[i], "mixed", True)
        infos.append(info)
        if len(xs_head) < 2:
            xs_head.append(x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"mixed{'+learned' if net else ''}: {ms_per_step:.1f} ms/solve, iters "
        f"{[i['iters'] for i in infos]}, relres max {max(i['rel_residual'] for i in infos):.2e}")

    def compare(precision, use_net, form, precond="none", margin=0.0):
        out = []
        if precond != "none":  # the first preconditioned solve builds the red-black matrix: keep it untimed
            run(rhs[0], precision, use_net, form, precond, margin)
            torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(args.warmup, len(rhs)):
            _, info = run(rhs[i], precision, use_net, form, precond, margin)
            out.append(info)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        d = {"ms_per_solve": round((t3 - t2) * 1e3 / args.steps, 3), "iters": [i["iters"] for i in out],
             "rel_residual_max": max(i["rel_residual"] for i in out)}
        key = "a_kernel_ms" if precond == "none" else "s_product_ms"  # S product: the red + the black sweep
        d[key] = round(float(np.mean([i["spmv_ms"] for i in out if i["spmv_samples"]])), 5)
        if precond != "none" and form == "projected" and d[key] > 0:
            sb = s_product_bytes(n, 4 if precision == "mixed" else 8)
            d["s_product_bytes"] = sb
            d["s_product_gbs"] = round(sb / (d[key] * 1e-3) / 1e9, 1)
        elif precond == "none" and precision == "fp64" and d[key] > 0:
            ab = a_kernel_bytes(A.n, A.nnz, False)
            d["a_kernel_bytes"] = ab
            d["a_kernel_gbs"] = round(ab / (d[key] * 1e-3) / 1e9, 1)
        log(f"{precision} {form}{' +net' if use_net else ''}{' +' + precond if precond != 'none' else ''}: "
            f"{d['ms_per_solve']:.1f} ms/solve iters {d['iters']}")
        return d

    # the headline solves with the stopping margin forced (0.05): what the
    # margin would cost if it were always on
    forced = compare("mixed", True, "projected", margin=0.05)

    # energy-norm ratio of the learned start, ||x* - gamma y||_A / ||x*||_A on
    # the pinned system (x* from the headline solves): 1 = no better than zero
    a_ratio = []
    if net is not None:
        for k, xh in enumerate(xs_head):
            b = rhs[args.warmup + k]  # prepared in place by the headline solve
            y = net.forward(n, b)
            y[0] = 0.0
            ay = m.spmv(A, y)
            bx, by, yay = float(torch.dot(b, xh)), float(torch.dot(b, y)), float(torch.dot(y, ay))
            a_ratio.append(round(float(np.sqrt(max(0.0, 1.0 - by * by / (yay * bx)))), 4))

    fp64 = fp64p = mixed_nonet = dic_mixed = dic_mixed_net = dic_fp64 = None
    if not args.no_fp64:
        fp64 = compare("fp64", False, "pinned")
        fp64p = compare("fp64", False, "projected")
        if net is not None:
            mixed_nonet = compare("mixed", False, "projected")
    if not args.no_dic:
        # the paper's DIC preconditioner in red-black order (same tolerance, same right-hand sides)
        dic_mixed = compare("mixed", False, "projected", "dic")
        if net is not None:
            dic_mixed_net = compare("mixed", True, "projected", "dic")
        if not args.no_fp64:
            dic_fp64 = compare("fp64", False, "projected", "dic")

    # dominant kernel: the mixed-precision CG SpMV kernel, sampled live with
    # HIP events on the solve stream inside the timed region
    samples = [(i["spmv_ms"], i["spmv_samples"]) for i in infos if i["spmv_samples"]]
    a_ms = sum(ms * k for ms, k in samples) / max(1, sum(k for _, k in samples))
    a_bytes = a_kernel_bytes(A.n, A.nnz, True)
    achieved = a_bytes / (a_ms * 1e-3) / 1e9 if a_ms > 0 else 0.0
    traffic = measured_traffic("cg_a32", n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "cg_a32", "bytes_per_launch": a_bytes, "avg_launch_ms": round(a_ms, 5)}

    # isolated plain SpMV: 100 launches, each bracketed by HIP events on the
    # stream it runs on (median and mean; the bracket leaves the GPU idle
    # between launches), then 100 back-to-back launches under one pair of
    # events (the sustained time per product, launch gaps included)
    def time_spmv(dtype, f=m.spmv):
        xs = torch.randn(A.n, dtype=dtype, device="cuda")
        ys = torch.empty_like(xs)
        for _ in range(3):
            f(A, xs, ys)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
        for e0, e1 in ev:
            e0.record()
            f(A, xs, ys)
            e1.record()
        torch.cuda.synchronize()
        t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(100):
            f(A, xs, ys)
        e1.record()
        torch.cuda.synchronize()
        return 0.5 * (t[49] + t[50]), sum(t) / len(t), e0.elapsed_time(e1) / 100

    spmv_ms, spmv_mean, spmv_b2b = time_spmv(torch.float32)
    spmv_gbs = spmv_bytes(A.n, A.nnz, 4) / (spmv_ms * 1e-3) / 1e9
    spmv64_ms, spmv64_mean, spmv64_b2b = time_spmv(torch.float64)
    spmv64_gbs = spmv_bytes(A.n, A.nnz, 8) / (spmv64_ms * 1e-3) / 1e9
    # the same product from the symmetric storage (diagonal + upper triangle)
    sym_ms, sym_mean, _ = time_spmv(torch.float32, m.spmv_sym)
    sym_gbs = spmv_sym_bytes(A.n, A.nnz, 4) / (sym_ms * 1e-3) / 1e9

    # plain copy of known size (256 MiB read, 256 MiB written): the reference
    # that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes
    ca = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    torch.cuda.synchronize()
    del ca, cb

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, seeds[args.warmup], args.tol, fp64["iters"][0] if fp64 else None)

    value = ms_per_step / 1e3
    line = {
        "metric": "Poisson CG time-to-1e-10 & SpMV GB/s, 256^3, plain FP64 vs mixed+learned",
        "value": round(value, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"pressure-Poisson CG, {n}^3 pinned Neumann 7-point CSR, Gaussian-smoothed "
                               f"(sigma=3) random rhs seeds {seeds[args.warmup]}..{seeds[-1]}, tol {args.tol:g}, "
                               f"mixed FP32/FP64 reliable-update CG, projected formulation"
                               + (" + learned warm start" if net else ""),
                   "grid": n, "unknowns": A.n, "nnz": A.nnz, "learned_warm_start": net is not None},
        "iters": [i["iters"] for i in infos],
        "refreshes": [i["updates"] for i in infos],
        "rel_residual_max": max(i["rel_residual"] for i in infos),
        "stop_margin": sorted({i["stop_margin"] for i in infos}),
        "forced_margin_0.05": {**forced, "extra_iters": int(np.sum(forced["iters"])
                                                            - np.sum([i["iters"] for i in infos])),
                               "extra_time_frac": round(forced["ms_per_solve"] / ms_per_step - 1.0, 4)},
        "warm_start": {"init_residual_mean": float(np.mean([i["init_residual"] for i in infos])),
                       "gamma": [round(i["gamma"], 6) for i in infos],
                       "a_norm_ratio": a_ratio,
                       "fallbacks": int(sum(i["used_fallback"] for i in infos))} if net else None,
        "fp64_plain_pinned": fp64,
        "fp64_projected": fp64p,
        "mixed_projected_no_net": mixed_nonet,
        "dic_mixed_projected": dic_mixed,
        "dic_mixed_projected_learned": dic_mixed_net,
        "dic_fp64_projected": dic_fp64,
        "speedup_dic_mixed_vs_fp64_plain": (round(fp64["ms_per_solve"] / dic_mixed["ms_per_solve"], 3)
                                            if fp64 and dic_mixed else None),
        "speedup_vs_fp64_plain": round(fp64["ms_per_solve"] / ms_per_step, 3) if fp64 else None,
        "speedup_vs_fp64_projected": round(fp64p["ms_per_solve"] / ms_per_step, 3) if fp64p else None,
        "spmv_fp32_isolated": {"ms": round(spmv_ms, 5), "ms_mean": round(spmv_mean, 5), "launches": 100,
                               "gbs": round(spmv_gbs, 1), "frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
                               "back_to_back_ms": round(spmv_b2b, 5),
                               "back_to_back_frac": round(spmv_bytes(A.n, A.nnz, 4) / (spmv_b2b * 1e-3) / 1e9
                                                          / HBM_PEAK_GBS, 4)},
        "spmv_fp64_isolated": {"ms": round(spmv64_ms, 5), "ms_mean": round(spmv64_mean, 5), "launches": 100,
                               "gbs": round(spmv64_gbs, 1), "frac": round(spmv64_gbs / HBM_PEAK_GBS, 4),
                               "back_to_back_ms": round(spmv64_b2b, 5),
                               "back_to_back_frac": round(spmv_bytes(A.n, A.nnz, 8) / (spmv64_b2b * 1e-3) / 1e9
                                                          / HBM_PEAK_GBS, 4)},
        "spmv_sym_fp32_isolated": {"ms": round(sym_ms, 5), "ms_mean": round(sym_mean, 5), "launches": 100,
                                   "bytes": spmv_sym_bytes(A.n, A.nnz, 4), "gbs": round(sym_gbs, 1),
                                   "time_vs_full_csr": round(sym_ms / spmv_ms, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


_CPU_CHILD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle, synth
n, seed, tol = int(sys.argv[2]), int(sys.argv[3]), float(sys.argv[4])
t = time.perf_counter()
A = oracle.assemble(n, 0)
b = oracle.rhs_prepare(synth.smoothed_rhs(n, seed), 0)
setup = time.perf_counter() - t
t = time.perf_counter()
x, it, rr, st = oracle.cg(A, b, tol=tol)
dt = time.perf_counter() - t
threads = oracle.threads()
oracle.set_threads(1)
t = time.perf_counter()
_, it1, _, _ = oracle.cg(A, b, tol=0.0, max_iters=20)
dt1 = time.perf_counter() - t
print(json.dumps({"seconds": dt, "iters": it, "relres": rr, "status": st, "threads": threads,
                  "setup_seconds": setup, "one_thread_iters": it1, "one_thread_seconds": dt1}))
"""


def step_workload(args):
    """Time steps of the cavity (Sec. 3.1 fractional step) at n^3 from a
    random flow (synth.random_flow, |u| <= 1, seed 7), nu = 1e-3, lid 1,
    dt = 0.4 h; each pressure solve mixed + projected to tol.  One JSON line
    (ms per step and the solves' iterations); the step kernels' own times
    come from a kernel trace of this run."""
    import torch

    import paper_2504_03697_amd as m
    import synth

    torch.cuda.set_device(0)
    n = args.n
    h = 1.0 / n
    dt = 0.4 * h
    S = m.State(n, nu=1e-3, lid_u=1.0)
    for t, a in zip((S.u, S.v, S.w), synth.random_flow(n, 7)):
        t.copy_(torch.from_numpy(a))
    # 256 MiB device copy: the calibration kernel of the PMC byte counters
    cal = torch.empty(32 << 20, dtype=torch.float64, device="cuda")
    cal.copy_(torch.zeros_like(cal))
    kw = dict(tol=args.tol, precision="mixed", formulation="projected")
    for _ in range(args.warmup):
        m.step(S, dt, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = [m.step(S, dt, **kw)["iters"] for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    faces = 3 * n * n * (n + 1)
    print(json.dumps({"metric": f"cavity time step, {n}^3", "value": round(ms, 3), "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "dtype": "f64",
                      "data": "synthetic", "config": {"workload": f"cavity step {n}^3 from a random flow, nu 1e-3, "
                                                                  f"dt 0.4 h, mixed + projected solve to {args.tol:g}",
                                                      "faces": faces, "iters": iters}}))


def host_cpu_info():
    """nproc, the CPUs this process may run on, and lscpu's model, sockets and
    cores (what the oracle's threads ran on)."""
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
                "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus"}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                v = v.strip()
                info[keys[k.strip()]] = int(v) if v.isdigit() else v
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(n, seed, tol, iters_gpu):
    """The oracle's plain FP64 CG (pinned matrix, zero guess, the plain method)
    on one of the timed right-hand sides, solved in full on the host cores in
    a child process started with OMP_PROC_BIND=close, OMP_PLACES=cores (so
    the binding applies: this process's OpenMP runtime is already running)."""
    import subprocess
    env = dict(os.environ, OMP_PROC_BIND="close", OMP_PLACES="cores")
    r = subprocess.run([sys.executable, "-c", _CPU_CHILD, ROOT, str(n), str(seed), repr(tol)], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        log(f"oracle baseline failed: {r.stderr[-400:]}")
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    hw = host_cpu_info()
    log(f"oracle: full {n}^3 FP64 CG solve, {d['iters']} iterations in {d['seconds']:.1f} s on {d['threads']} "
        f"threads ({hw.get('model', '?')}); 1 thread: {d['one_thread_iters']} iterations in "
        f"{d['one_thread_seconds']:.1f} s")
    per1 = d["one_thread_seconds"] / d["one_thread_iters"]
    return {"value": round(d["seconds"], 3), "unit": "s", "cores": d["threads"], "kind": "oracle",
            "sample": f"one full plain FP64 CG solve (pinned matrix, zero guess) of the {n}^3 smoothed right-hand "
                      f"side seed {seed} to {tol:g}: {d['iters']} iterations, relative residual "
                      f"{d['relres']:.2e} (the GPU's plain FP64 CG took {iters_gpu} on it)",
            "full_solve": True, "iters": d["iters"], "seconds_per_iter": round(d["seconds"] / d["iters"], 5),
            "omp": {"OMP_PROC_BIND": "close", "OMP_PLACES": "cores", "threads": d["threads"]},
            "host": hw,
            "one_thread": {"value": round(per1 * d["iters"], 3), "seconds_per_iter": round(per1, 5),
                           "sample": f"first {d['one_thread_iters']} iterations on 1 thread "
                                     f"({d['one_thread_seconds']:.1f} s), scaled to the full solve's iterations"}}


if __name__ == "__main__":
    main()
