"""FP64 CPU oracle for the pressure-Poisson hot path (arXiv 2504.03697).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.
It shares no code with the HIP path.  The arithmetic lives in
``cfd_oracle.c`` (plain C, FP64, OpenMP loops with fixed-order dots); this
module only builds it, marshals numpy arrays, and composes the network
layers of the warm-start model from the C primitives.

Functions and the passage each follows:

* ``assemble``      - Sec. 3.1 (Poisson system stored as CSR), with the
                      integer-stencil / pinned-cell reading.
* ``spmv``, ``dot`` - Table 1 kernels ``spmv`` and ``dot``.
* ``cg``            - Sec. 3.1 conjugate-gradient solve (no preconditioner).
* ``neumann_solve_spectral``, ``pinned_solve_spectral`` - the exact solution
                      of the Sec. 3.1 pressure system (singular Neumann form,
                      or with the pinned cell), by the discrete cosine
                      eigenbasis of the 7-point Laplacian: a direct reference
                      for large grids, where CG to 1e-12 takes minutes.
* ``order``, ``dic_factor``, ``dic_apply``, ``pcg`` - Sec. 3.1 preconditioned
                      CG with the DIC or Jacobi preconditioner; DIC's
                      recurrences follow an elimination order (natural, or
                      red-black: the order in which they run in parallel,
                      cf. Sec. 3.3 on DIC's loop dependencies).
* ``step``          - Sec. 3.1 fractional step (forces, semi-Lagrangian
                      advection, pressure correction) on the staggered grid,
                      plus explicit viscosity (Sec. 5 future-work item).
* ``conv3d_*``, ``net_*``, ``adam``, ``round_bf16``, ``training_pair`` - the learned warm
                      start's network (not in the paper; definitions written
                      out directly; its activations are stored in bfloat16).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfd_oracle.c")
# CFD_ORACLE_LIB: load a prebuilt copy instead (the sanitizer test builds
# one with -fsanitize=address,undefined)
_LIB_OVERRIDE = os.environ.get("CFD_ORACLE_LIB")
_LIB = _LIB_OVERRIDE or os.path.join(_HERE, "libcfd_oracle.so")

OK, ENOCONV, EBREAKDOWN, ENONFINITE = 0, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile cfd_oracle.c with gcc into libcfd_oracle.so (in-tree)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-fno-fast-math", "-ffp-contract=off", "-o", _LIB, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.ora_nnz.restype = i64
        lib.ora_nnz.argtypes = [i32, i32, i32, i64]
        lib.ora_assemble.restype = None
        lib.ora_assemble.argtypes = [i32, i32, i32, i64, vp, vp, vp]
        lib.ora_spmv.restype = None
        lib.ora_spmv.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.ora_dot.restype = dbl
        lib.ora_dot.argtypes = [i64, vp, vp]
        lib.ora_rhs_prepare.restype = None
        lib.ora_rhs_prepare.argtypes = [i64, vp, i64]
        lib.ora_cg.restype = i32
        lib.ora_cg.argtypes = [i64, vp, vp, vp, vp, vp, dbl, i32, vp, vp, vp]
        lib.ora_order.argtypes = [i32, i32, i32, i32, vp, vp]
        lib.ora_dic_factor.restype = i32
        lib.ora_dic_factor.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        lib.ora_dic_apply.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.ora_pcg.restype = i32
        lib.ora_pcg.argtypes = [i64, vp, vp, vp, vp, vp, dbl, i32, i32, vp, vp, vp, vp, vp]
        lib.ora_advect.restype = None
        lib.ora_advect.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp]
        lib.ora_diffuse.restype = None
        lib.ora_diffuse.argtypes = [i32, i32, i32, dbl, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp]
        lib.ora_divergence.restype = None
        lib.ora_divergence.argtypes = [i32, i32, i32, vp, vp, vp, vp]
        lib.ora_correct.restype = None
        lib.ora_correct.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, vp, vp, vp]
        lib.ora_step.restype = i32
        lib.ora_step.argtypes = [i32, i32, i32, dbl, dbl, dbl, dbl, dbl, dbl, dbl, dbl,
                                 vp, vp, vp, i64, dbl, i32, vp, vp, vp, vp, vp, vp]
        for name in ("ora_conv3d_fwd", "ora_conv3d_bwd_data", "ora_conv3d_bwd_weight"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
        lib.ora_threads.restype = i32
        lib.ora_threads.argtypes = []
        lib.ora_set_threads.restype = None
        lib.ora_set_threads.argtypes = [i32]
        lib.ora_adam.restype = None
        lib.ora_adam.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, i32]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(grid):
    if isinstance(grid, int):
        return grid, grid, grid
    nx, ny, nz = grid
    return int(nx), int(ny), int(nz)


# ---------------------------------------------------------------- matrix

class Csr:
    """Host CSR matrix (int32 row pointers and columns, float64 values)."""

    def __init__(self, row_ptr, col, val, dims, pin):
        self.row_ptr, self.col, self.val = row_ptr, col, val
        self.dims, self.pin = dims, pin
        self.n = len(row_ptr) - 1
        self.nnz = len(col)

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            for e in range(self.row_ptr[i], self.row_ptr[i + 1]):
                a[i, self.col[e]] += self.val[e]
        return a


def nnz(grid, pin: int = 0) -> int:
    nx, ny, nz = _dims(grid)
    return int(_load().ora_nnz(nx, ny, nz, pin))


def assemble(grid, pin: int = 0) -> Csr:
    """CSR of the 7-point integer Neumann stencil, pinned at ``pin`` (pin < 0: singular)."""
    nx, ny, nz = _dims(grid)
    n = nx * ny * nz
    m = nnz((nx, ny, nz), pin)
    rp = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(m, dtype=np.int32)
    val = np.zeros(m, dtype=np.float64)
    _load().ora_assemble(nx, ny, nz, pin, _p(rp), _p(col), _p(val))
    return Csr(rp, col, val, (nx, ny, nz), pin)


def spmv(A: Csr, x) -> np.ndarray:
    x = _f64(x)
    y = np.zeros(A.n)
    _load().ora_spmv(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(x), _p(y))
    return y


def dot(x, y) -> float:
    x, y = _f64(x), _f64(y)
    return float(_load().ora_dot(len(x), _p(x), _p(y)))


def rhs_prepare(b, pin: int = 0) -> np.ndarray:
    """Return a consistent copy of b: mean removed, then b[pin] = 0."""
    b = _f64(b).copy()
    _load().ora_rhs_prepare(len(b), _p(b), pin)
    return b


def cg(A: Csr, b, x0=None, tol: float = 1e-10, max_iters: int = 100000):
    """Textbook CG.  Returns (x, iters, relres, status)."""
    b = _f64(b)
    x = np.zeros(A.n)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    x0p = None
    if x0 is not None:
        x0 = _f64(x0)
        x0p = _p(x0)
    st = _load().ora_cg(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), x0p, tol,
                        max_iters, _p(x), ctypes.byref(it), ctypes.byref(rr))
    return x, it.value, rr.value, st


def _neumann_eigenvalues(m: int) -> np.ndarray:
    """Eigenvalues 4 sin^2(pi k / (2 m)), k = 0..m-1, of the 1-D cell-centred
    Neumann second difference (degree on the diagonal, -1 off it); the k-th
    eigenvector is cos(pi k (i + 1/2) / m), the k-th orthonormal DCT-II row."""
    return 4.0 * np.sin(np.pi * np.arange(m) / (2.0 * m)) ** 2


def neumann_solve_spectral(grid, c) -> np.ndarray:
    """Minimum-norm (mean-zero) solution of L x = c - mean(c), L the singular
    Neumann matrix ``assemble(grid, -1)`` (Sec. 3.1's pressure system).

    L is the Kronecker sum of the 1-D Neumann second differences, so the 3-D
    orthonormal DCT-II diagonalises it with eigenvalue lx_i + ly_j + lz_k on
    mode (i, j, k): transform, divide, drop the constant mode (the null
    space), transform back.  Rounding error is about eps * cond(L) relative.
    """
    from scipy import fft
    nx, ny, nz = _dims(grid)
    c = _f64(c).reshape(nz, ny, nx)  # x is the fastest index
    C = fft.dctn(c, type=2, norm="ortho")
    lam = (_neumann_eigenvalues(nz)[:, None, None] + _neumann_eigenvalues(ny)[None, :, None]
           + _neumann_eigenvalues(nx)[None, None, :])
    lam[0, 0, 0] = 1.0
    C /= lam
    C[0, 0, 0] = 0.0
    return np.ascontiguousarray(fft.idctn(C, type=2, norm="ortho").reshape(-1))


def pinned_solve_spectral(grid, pin: int, b) -> np.ndarray:
    """Exact solution of ``assemble(grid, pin)`` x = b (pin >= 0).

    Row pin gives x[pin] = b[pin]; every other row is the Neumann row with
    the pin's column dropped, i.e. (L x)_j = b_j + L[j, pin] x[pin].  With
    c_j = b_j + L[j, pin] b[pin] (j != pin) and c[pin] = -sum_{j != pin} c_j
    (the columns of L sum to zero), L x = c is consistent and x is the
    mean-zero solution shifted so that x[pin] = b[pin].
    """
    nx, ny, nz = _dims(grid)
    b = _f64(b)
    c = b.copy()
    i, j, k = pin % nx, (pin // nx) % ny, pin // (nx * ny)
    for di, dj, dk in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        a, bb, cc = i + di, j + dj, k + dk
        if 0 <= a < nx and 0 <= bb < ny and 0 <= cc < nz:
            c[a + nx * (bb + ny * cc)] -= b[pin]  # L[j, pin] = -1
    c[pin] = 0.0
    c[pin] = -c.sum()
    x = neumann_solve_spectral((nx, ny, nz), c)
    return x + (b[pin] - x[pin])


PRECOND = {"none": 0, "jacobi": 1, "dic": 2}


def order(grid, redblack: bool):
    """Elimination order: (ord, pos) with ord[t] = cell at position t."""
    nx, ny, nz = _dims(grid)
    n = nx * ny * nz
    ordv = np.zeros(n, dtype=np.int64)
    pos = np.zeros(n, dtype=np.int64)
    _load().ora_order(nx, ny, nz, int(bool(redblack)), _p(ordv), _p(pos))
    return ordv, pos


def dic_factor(A: Csr, redblack: bool = True):
    """DIC pivots d (diag(M) = diag(A)); raises if a pivot is not positive."""
    ordv, pos = order(A.dims, redblack)
    d = np.zeros(A.n)
    if _load().ora_dic_factor(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(ordv), _p(pos), _p(d)) != 0:
        raise ValueError("DIC: non-positive pivot")
    return d


def dic_apply(A: Csr, d, r, redblack: bool = True):
    """z = M^{-1} r for the DIC preconditioner M = (D+L) D^{-1} (D+U)."""
    ordv, pos = order(A.dims, redblack)
    r = _f64(r)
    d = _f64(d)
    z = np.zeros(A.n)
    work = np.zeros(A.n)
    _load().ora_dic_apply(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(ordv), _p(pos), _p(d), _p(r), _p(z),
                          _p(work))
    return z


def pcg(A: Csr, b, x0=None, tol: float = 1e-10, max_iters: int = 100000, precond: str = "dic",
        redblack: bool = True):
    """Preconditioned CG.  Returns (x, iters, relres, status)."""
    b = _f64(b)
    x = np.zeros(A.n)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    ordv, pos = order(A.dims, redblack)
    x0p = None
    if x0 is not None:
        x0 = _f64(x0)
        x0p = _p(x0)
    st = _load().ora_pcg(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), x0p, tol, max_iters,
                         PRECOND[precond], _p(ordv), _p(pos), _p(x), ctypes.byref(it), ctypes.byref(rr))
    return x, it.value, rr.value, st


# ---------------------------------------------------------------- time step

def face_shapes(grid):
    nx, ny, nz = _dims(grid)
    return (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1), nx * ny * nz


def advect(grid, h, lid, dt, u, v, w):
    nx, ny, nz = _dims(grid)
    u, v, w = _f64(u), _f64(v), _f64(w)
    un, vn, wn = np.empty_like(u), np.empty_like(v), np.empty_like(w)
    _load().ora_advect(nx, ny, nz, h, lid, dt, _p(u), _p(v), _p(w), _p(un), _p(vn), _p(wn))
    return un, vn, wn


def diffuse(grid, h, lid, dt, nu, u, v, w):
    nx, ny, nz = _dims(grid)
    u, v, w = _f64(u), _f64(v), _f64(w)
    un, vn, wn = np.empty_like(u), np.empty_like(v), np.empty_like(w)
    _load().ora_diffuse(nx, ny, nz, h, lid, dt, nu, _p(u), _p(v), _p(w), _p(un), _p(vn), _p(wn))
    return un, vn, wn


def divergence(grid, u, v, w):
    nx, ny, nz = _dims(grid)
    u, v, w = _f64(u), _f64(v), _f64(w)
    D = np.empty(nx * ny * nz)
    _load().ora_divergence(nx, ny, nz, _p(u), _p(v), _p(w), _p(D))
    return D


def correct(grid, h, rho, dt, p, u, v, w):
    nx, ny, nz = _dims(grid)
    u, v, w = _f64(u).copy(), _f64(v).copy(), _f64(w).copy()
    p = _f64(p)
    _load().ora_correct(nx, ny, nz, h, rho, dt, _p(p), _p(u), _p(v), _p(w))
    return u, v, w


class State:
    """Cavity state on the MAC grid (float64 numpy arrays)."""

    def __init__(self, grid, h=None, nu=0.0, rho=1.0, lid=1.0, g=(0.0, 0.0, 0.0), pin=0):
        self.dims = _dims(grid)
        nx, ny, nz = self.dims
        self.h = 1.0 / max(self.dims) if h is None else h
        su, sv, sw, sp = face_shapes(self.dims)
        self.u, self.v, self.w = np.zeros(su), np.zeros(sv), np.zeros(sw)
        self.p = np.ones(sp)
        self.nu, self.rho, self.lid, self.g, self.pin = nu, rho, lid, g, pin
        self.A = assemble(self.dims, pin)
        self.t, self.step_count = 0.0, 0


def step(S: State, dt: float, tol: float = 1e-10, max_iters: int = 100000):
    """Advance ``S`` by one fractional step in place.  Returns (iters, relres, status)."""
    nx, ny, nz = S.dims
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    A = S.A
    st = _load().ora_step(nx, ny, nz, S.h, S.lid, S.nu, S.rho, S.g[0], S.g[1], S.g[2], dt,
                          _p(A.row_ptr), _p(A.col), _p(A.val), S.pin, tol, max_iters,
                          _p(S.u), _p(S.v), _p(S.w), _p(S.p), ctypes.byref(it), ctypes.byref(rr))
    S.t += dt
    S.step_count += 1
    return it.value, rr.value, st


# ---------------------------------------------------------------- network

def conv3d_fwd(grid, X, W, cin, cout):
    """Replicate-padded 3x3x3 convolution: X[v, cin] -> Y[v, cout] (float64)."""
    nx, ny, nz = _dims(grid)
    X, W = _f64(X), _f64(W)
    Y = np.empty(nx * ny * nz * cout)
    _load().ora_conv3d_fwd(nx, ny, nz, cin, cout, _p(X), _p(W), _p(Y))
    return Y


def conv3d_bwd_data(grid, dY, W, cin, cout):
    nx, ny, nz = _dims(grid)
    dY, W = _f64(dY), _f64(W)
    dX = np.empty(nx * ny * nz * cin)
    _load().ora_conv3d_bwd_data(nx, ny, nz, cin, cout, _p(dY), _p(W), _p(dX))
    return dX


def conv3d_bwd_weight(grid, X, dY, cin, cout):
    nx, ny, nz = _dims(grid)
    X, dY = _f64(X), _f64(dY)
    dW = np.empty(27 * cin * cout)
    _load().ora_conv3d_bwd_weight(nx, ny, nz, cin, cout, _p(X), _p(dY), _p(dW))
    return dW


def threads() -> int:
    """OpenMP threads the oracle's parallel loops run on."""
    return int(_load().ora_threads())


def set_threads(t: int) -> None:
    """Run the parallel loops on t threads (timings only: the sums have a
    fixed order, so results do not depend on it)."""
    _load().ora_set_threads(int(t))


def split_params(theta, shapes):
    out, off = [], 0
    for cin, cout in shapes:
        m = 27 * cin * cout
        out.append(np.asarray(theta[off:off + m], dtype=np.float64))
        off += m
    return out


def round_bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits, float32's exponent
    range), ties to even, via float32 (as a float32 accumulator would hold the
    value first).  Written from the format's definition: a value m * 2^e with
    0.5 <= |m| < 1 keeps m rounded to a multiple of 2^-8; below float32's
    normal range the spacing stays 2^-133.  Returns float64."""
    v = np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    m, e = np.frexp(v)
    e = np.maximum(e, -125)  # float32 normals start at 2^-126 = 0.5 * 2^-125
    return np.ldexp(np.rint(np.ldexp(v, 8 - e)), e - 8)


def net_forward(grid, x, theta, shapes, act_bf16=False):
    """Conv-ReLU stack (ReLU after every layer but the last).  Returns (y, acts).

    act_bf16: store the input and every hidden activation in bfloat16, as the
    network's definition has it (the convolutions themselves stay exact in
    float64 here)."""
    Ws = split_params(theta, shapes)
    acts = [round_bf16(x) if act_bf16 else _f64(x)]
    h = acts[0]
    for l, ((cin, cout), W) in enumerate(zip(shapes, Ws)):
        h = conv3d_fwd(grid, h, W, cin, cout)
        if l < len(shapes) - 1:
            h = np.maximum(h, 0.0)
            if act_bf16:
                h = round_bf16(h)
        acts.append(h)
    return acts[-1], acts


def net_loss_grad(grid, x, target, theta, shapes):
    """Mean-squared error over voxels and its gradient w.r.t. every weight.

    loss = mean_v (y_v - target_v)^2; returns (loss, grad) with grad laid out
    like theta.
    """
    y, acts = net_forward(grid, x, theta, shapes)
    Ws = split_params(theta, shapes)
    n = len(y)
    diff = y - _f64(target)
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / n
    grads = [None] * len(shapes)
    for l in range(len(shapes) - 1, -1, -1):
        cin, cout = shapes[l]
        if l < len(shapes) - 1:
            g = g * (acts[l + 1] > 0.0)
        grads[l] = conv3d_bwd_weight(grid, acts[l], g, cin, cout)
        if l > 0:
            g = conv3d_bwd_data(grid, g, Ws[l], cin, cout)
    return loss, np.concatenate(grads)


def training_pair(b, p):
    """Warm-start training pair (written out from its definition, float64,
    returned as float32): input b / rms(b), target (p - mean p) /
    rms(p - mean p); zero where the divisor is zero."""
    b = _f64(b)
    p = _f64(p)
    rb = np.sqrt(np.mean(b * b))
    d = p - np.mean(p)
    rp = np.sqrt(np.mean(d * d))
    x = b / rb if rb > 0 else np.zeros_like(b)
    t = d / rp if rp > 0 else np.zeros_like(d)
    return x.astype(np.float32), t.astype(np.float32)


def adam(theta, m, v, g, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on float64 copies; returns (theta, m, v)."""
    theta, m, v, g = _f64(theta).copy(), _f64(m).copy(), _f64(v).copy(), _f64(g)
    _load().ora_adam(len(theta), _p(theta), _p(m), _p(v), _p(g), lr, beta1, beta2, eps, t)
    return theta, m, v


def warm_start_gamma(A: Csr, b, y):
    """A-norm-optimal scale of a predicted solution y: gamma = b^T y / y^T A y."""
    y = _f64(y)
    return dot(b, y) / dot(y, spmv(A, y))
