"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): every C entry point runs on small ragged grids in a child
process that loads a sanitized build; any out-of-bounds access, use of freed
memory or undefined behaviour aborts it.  A bad access in the oracle would
corrupt the expected values the GPU tests compare against."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

WORKLOAD = r"""
import numpy as np
import oracle, synth
dims = (5, 4, 3)
for pin in (0, 7, -1):
    A = oracle.assemble(dims, pin)
    x = np.random.default_rng(1).standard_normal(A.n)
    oracle.spmv(A, x); oracle.dot(x, x)
    b = oracle.rhs_prepare(x, pin if pin >= 0 else 0)
    if pin >= 0:
        oracle.cg(A, b, tol=1e-12)
        for pc, rb in (("none", True), ("jacobi", True), ("dic", False), ("dic", True)):
            oracle.pcg(A, b, tol=1e-12, precond=pc, redblack=rb)
    for rb in (False, True):
        oracle.order(dims, rb)
        d = oracle.dic_factor(A, rb)
        oracle.dic_apply(A, d, x, rb)
S = oracle.State((6, 5, 4), nu=0.01, lid=1.0, g=(0.0, -0.3, 0.1))
for _ in range(3):
    oracle.step(S, 0.01)
shapes = synth.net_layer_shapes()
theta = synth.net_init(2)
g = (4, 3, 5)
n = 60
for cin, cout in ((1, 16), (16, 16), (16, 1)):
    X = synth.bf16_values(n * cin, 1); W = synth.bf16_values(27 * cin * cout, 2)
    Y = oracle.conv3d_fwd(g, X, W, cin, cout)
    oracle.conv3d_bwd_data(g, Y, W, cin, cout)
    oracle.conv3d_bwd_weight(g, X, Y, cin, cout)
loss, grad = oracle.net_loss_grad(g, synth.uniform_rhs(g, 3), synth.uniform_rhs(g, 4), theta, shapes)
m = np.zeros_like(theta); v = np.zeros_like(theta)
oracle.adam(theta, m, v, grad, 1e-3, 1)
print("sanitized oracle ok")
"""


def _libasan():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_ubsan(tmp_path):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc's libasan is not available")
    lib = str(tmp_path / "libcfd_oracle_san.so")
    src = os.path.join(ROOT, "oracle", "cfd_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
                           "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", lib, src, "-lm"])
    env = dict(os.environ)
    env.update({"CFD_ORACLE_LIB": lib, "LD_PRELOAD": asan, "OMP_NUM_THREADS": "2",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1",
                "PYTHONPATH": ROOT + os.pathsep + env.get("PYTHONPATH", "")})
    r = subprocess.run([sys.executable, "-c", WORKLOAD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
