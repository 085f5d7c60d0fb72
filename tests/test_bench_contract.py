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
    assert bench.a_kernel_bytes(n, nnz, False) == 4 * (n + 1) + 12 * nnz + 48 * n
    assert bench.spmv_bytes(n, nnz, 4) == 4 * (n + 1) + 8 * nnz + 8 * n
    assert len(bench.kernel_source_sha()) == 16
