"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_rejected():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    n, nnz = 256**3, 7 * 256**3 - 6 * 256**2 - 6
    assert bench.a_kernel_bytes(n, nnz, True) == 4 * (n + 1) + 8 * nnz + 16 * n == 1271922644
    # the float64 kernel reads the float32 copy of the (integer) matrix values too
    assert bench.a_kernel_bytes(n, nnz, False) == 4 * (n + 1) + 8 * nnz + 48 * n == 1808793556
    assert bench.spmv_bytes(n, nnz, 4) == 4 * (n + 1) + 8 * nnz + 8 * n
    assert bench.spmv_bytes(n, nnz, 8) == 4 * (n + 1) + 8 * nnz + 16 * n
    # symmetric storage: every row holds its diagonal, so the off-diagonal
    # entries split evenly between the triangles
    nl = (nnz - n) // 2
    assert bench.spmv_sym_bytes(n, nnz, 4) == 8 * (n + 1) + 8 * (n + nl) + 4 * nl + 8 * n
    assert len(bench.kernel_source_sha()) == 16


def test_s_product_bytes_match_the_matrix():
    """The byte model of the red-black S product counts the entries of the
    Neumann matrix's red and black rows; check those counts on small grids
    against the oracle's matrix split by colour."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle
    for N in (4, 6, 8):
        A = oracle.assemble((N, N, N), -1)
        n = N ** 3
        idx = np.arange(n)
        red = ((idx % N) + (idx // N) % N + idx // (N * N)) % 2 == 0
        lens = np.diff(A.row_ptr)
        nnz_r, nnz_b = int(lens[red].sum()), int(lens[~red].sum())
        nr, nb = int(red.sum()), int((~red).sum())
        want = (4 * (nr + 1) + 8 * nnz_r + 8 * nb + 4 * nr + 4 * nb) + (4 * (nb + 1) + 8 * nnz_b + 4 * nb + 4 * nr + 4 * nb)
        assert bench.s_product_bytes(N) == want
        want64 = (4 * (nr + 1) + 8 * nnz_r + 16 * nb + 8 * nr + 8 * nb) + (4 * (nb + 1) + 8 * nnz_b + 8 * nb + 8 * nr + 8 * nb)
        assert bench.s_product_bytes(N, 8) == want64


def test_committed_profile_matches_the_kernel_sources():
    """The HBM traffic the bench reports comes from a committed PMC summary
    keyed by a hash of the CG kernel sources: one must exist for the sources
    as they are, within a few percent of the kernel's algorithmic bytes."""
    sys.path.insert(0, ROOT)
    import bench
    n = 256
    t = bench.measured_traffic("cg_a32", n)
    assert t is not None, "re-profile cg_a32 (profiles/cg_a32_poisson_256.md) for the current sources"
    alg = bench.a_kernel_bytes(n**3, 7 * n**3 - 6 * n**2 - 6, True)
    assert alg <= t <= 1.2 * alg


def test_step_workload_options():
    """--workload takes solve (the headline) or step (cavity steps for the
    time-step kernels); the step workload is one GPU too."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "other"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "step", "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "single GPU" in r.stderr


def test_step_profile_face_count():
    """The step-kernel profile's faces: 3 n^2 (n+1) at 256^3, the count its
    algorithmic bytes are built from (16 B per face for advection +
    viscosity, 8 B per face + 8 B per cell for the divergence)."""
    text = open(os.path.join(ROOT, "profiles", "step_kernels_256.md")).read()
    n = 256
    faces = 3 * n * n * (n + 1)
    assert f"{faces:,}" in text
    assert f"| {8 * faces / 1e6:.1f} + {8 * faces / 1e6:.1f} |" in text
    assert f"| {8 * faces / 1e6:.1f} + {8 * n**3 / 1e6:.1f} |" in text
