"""Pins of the oracle's matrix and CG against facts fixed by the mathematics.

Each check is independent of the oracle's own code: the matrix is rebuilt
from 1-D Neumann matrices with Kronecker products, eigenvalues come from
the closed form of the Neumann Laplacian, solutions from LAPACK dense solves
or from manufactured eigenvector right-hand sides, residuals are recomputed
in extended precision.
"""
import numpy as np
import pytest

import oracle
import synth


def neumann_1d(n):
    """1-D integer Neumann stencil: degree on the diagonal, -1 off it."""
    a = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            a[i, i - 1] = -1
            a[i, i] += 1
        if i < n - 1:
            a[i, i + 1] = -1
            a[i, i] += 1
    return a


def neumann_3d_dense(nx, ny, nz):
    """Kronecker sum; x is the fastest index, so it is the last Kronecker factor."""
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(iz, np.kron(iy, neumann_1d(nx)))
            + np.kron(iz, np.kron(neumann_1d(ny), ix))
            + np.kron(neumann_1d(nz), np.kron(iy, ix)))


def pin_dense(a, pin):
    a = a.copy()
    a[pin, :] = 0.0
    a[:, pin] = 0.0
    a[pin, pin] = 1.0
    return a


def cos_mode(n):
    x = (np.arange(n) + 0.5) / n
    c = np.cos(np.pi * x)
    # x fastest: P[k, j, i] = c_i c_j c_k
    return np.einsum("k,j,i->kji", c, c, c).reshape(-1)


@pytest.mark.parametrize("dims,pin", [((4, 4, 4), 0), ((4, 4, 4), -1), ((3, 5, 2), 7),
                                      ((5, 4, 3), 59), ((1, 1, 1), -1), ((6, 1, 3), 0)])
def test_assembly_matches_kronecker_sum(dims, pin):
    A = oracle.assemble(dims, pin)
    ref = neumann_3d_dense(*dims)
    if pin >= 0:
        ref = pin_dense(ref, pin)
    np.testing.assert_array_equal(A.dense(), ref)
    # one stored entry per structural nonzero (the diagonal is always stored)
    offdiag = np.count_nonzero(ref - np.diag(np.diag(ref)))
    assert A.nnz == offdiag + ref.shape[0]


@pytest.mark.parametrize("n", [2, 4, 16, 33])
def test_nnz_closed_form(n):
    # every cell has 7 entries minus one per missing wall neighbour (6 n^2 over
    # the six faces); a corner pin removes 3 off-diagonals in its own row and
    # one entry in each of its 3 neighbours.
    assert oracle.nnz(n, -1) == 7 * n**3 - 6 * n**2
    assert oracle.nnz(n, 0) == 7 * n**3 - 6 * n**2 - 6


@pytest.mark.parametrize("n", [4, 9])
def test_csr_structure(n):
    A = oracle.assemble(n, 0)
    rp, col = A.row_ptr, A.col
    assert rp[0] == 0 and rp[-1] == A.nnz
    assert np.all(np.diff(rp) >= 1) and np.all(np.diff(rp) <= 7)
    for i in range(A.n):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0), "columns ascending"
    d = A.dense()
    np.testing.assert_array_equal(d, d.T)  # bitwise symmetric


def test_singular_rowsum_zero_exact():
    A = oracle.assemble(12, -1)
    np.testing.assert_array_equal(oracle.spmv(A, np.ones(A.n)), np.zeros(A.n))


def test_eigenvalues_closed_form():
    n = 4
    d = oracle.assemble(n, -1).dense()
    ev = np.sort(np.linalg.eigvalsh(d))
    s = np.sin(np.pi * np.arange(n) / (2 * n)) ** 2
    ref = np.sort((4 * (s[:, None, None] + s[None, :, None] + s[None, None, :])).reshape(-1))
    np.testing.assert_allclose(ev, ref, atol=1e-13)


@pytest.mark.parametrize("n", [4, 16])
def test_cos_mode_is_eigenvector(n):
    P = cos_mode(n)
    A = oracle.assemble(n, -1)
    lam = 3 * (2 - 2 * np.cos(np.pi / n))
    np.testing.assert_allclose(oracle.spmv(A, P), lam * P, atol=1e-14 * n)


def test_cg_matches_dense_solve():
    n = 4
    b = oracle.rhs_prepare(synth.uniform_rhs(n, 0), 0)
    dense = pin_dense(neumann_3d_dense(n, n, n), 0)
    ref = np.linalg.solve(dense, b)
    A = oracle.assemble(n, 0)
    x, it, rr, st = oracle.cg(A, b, tol=1e-12)
    assert st == oracle.OK
    assert rr <= 1e-12
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_pinned_equals_shifted_min_norm():
    n = 4
    b = oracle.rhs_prepare(synth.uniform_rhs(n, 3), -1)  # consistent: zero mean
    dense_neu = neumann_3d_dense(n, n, n)
    p_mn = np.linalg.lstsq(dense_neu, b, rcond=None)[0]
    bp = b.copy()
    bp[0] = 0.0
    x, it, rr, st = oracle.cg(oracle.assemble(n, 0), bp, tol=1e-13)
    assert st == oracle.OK
    np.testing.assert_allclose(x, p_mn - p_mn[0], atol=1e-11)


@pytest.mark.parametrize("n", [4, 16])
def test_manufactured_pressure(n):
    # b = lam * P for the cos eigenvector P: the pinned solution is P - P[0].
    P = cos_mode(n)
    lam = 3 * (2 - 2 * np.cos(np.pi / n))
    b = oracle.rhs_prepare(lam * P, 0)
    A = oracle.assemble(n, 0)
    x, it, rr, st = oracle.cg(A, b, tol=1e-12)
    assert st == oracle.OK
    ref = P - P[0]
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-8


def test_singular_eigenvector_rhs_one_iteration():
    n = 8
    P = cos_mode(n)
    A = oracle.assemble(n, -1)
    x, it, rr, st = oracle.cg(A, P, tol=1e-10)
    assert st == oracle.OK and it == 1
    lam = 3 * (2 - 2 * np.cos(np.pi / n))
    np.testing.assert_allclose(x, P / lam, atol=1e-14)


def test_singular_cg_finite_termination():
    # 4^3 singular matrix: 15 distinct nonzero eigenvalues, so CG on a
    # consistent right-hand side terminates within 15 products.
    n = 4
    b = oracle.rhs_prepare(synth.uniform_rhs(n, 0), -1)
    x, it, rr, st = oracle.cg(oracle.assemble(n, -1), b, tol=1e-10)
    assert st == oracle.OK and it <= 15


def test_relres_self_certified_in_extended_precision():
    n = 12
    A = oracle.assemble(n, 0)
    b = oracle.rhs_prepare(synth.smoothed_rhs(n, 5), 0)
    x, it, rr, st = oracle.cg(A, b, tol=1e-10)
    assert st == oracle.OK
    d = A.dense().astype(np.longdouble)
    r = b.astype(np.longdouble) - d @ x.astype(np.longdouble)
    true_rr = float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b.astype(np.longdouble) ** 2)))
    assert true_rr <= 1e-10
    assert abs(true_rr - rr) <= 1e-3 * rr + 1e-16


def test_cg_zero_rhs_and_warm_start():
    A = oracle.assemble(6, 0)
    x, it, rr, st = oracle.cg(A, np.zeros(A.n), x0=np.ones(A.n))
    assert st == oracle.OK and it == 0 and rr == 0.0 and not x.any()
    b = oracle.rhs_prepare(synth.uniform_rhs(6, 1), 0)
    xs, it0, _, _ = oracle.cg(A, b, tol=1e-12)
    # starting at the solution needs no iteration
    x, it, rr, st = oracle.cg(A, b, x0=xs, tol=1e-10)
    assert st == oracle.OK and it == 0 and rr <= 1e-10


def test_cg_independent_of_thread_count():
    """Every oracle sum runs in a fixed order, so the thread count the
    timings use changes no bit of the result."""
    A = oracle.assemble(14, 0)
    b = oracle.rhs_prepare(synth.uniform_rhs(14, 3), 0)
    t0 = oracle.threads()
    try:
        oracle.set_threads(1)
        assert oracle.threads() == 1
        x1, it1, rr1, _ = oracle.cg(A, b, tol=1e-10)
        oracle.set_threads(3)
        x3, it3, rr3, _ = oracle.cg(A, b, tol=1e-10)
    finally:
        oracle.set_threads(t0)
    assert it1 == it3 and rr1 == rr3 and np.array_equal(x1, x3)


def test_cg_error_codes():
    A = oracle.assemble(8, 0)
    b = oracle.rhs_prepare(synth.uniform_rhs(8, 2), 0)
    x, it, rr, st = oracle.cg(A, b, tol=1e-10, max_iters=3)
    assert st == oracle.ENOCONV and it == 3
    bn = b.copy()
    bn[5] = np.nan
    assert oracle.cg(A, bn)[3] == oracle.ENONFINITE
    An = oracle.Csr(A.row_ptr, A.col, -A.val, A.dims, A.pin)
    assert oracle.cg(An, b)[3] == oracle.EBREAKDOWN


def test_rhs_prepare():
    b = synth.uniform_rhs(5, 9)
    c = oracle.rhs_prepare(b, 0)
    assert c[0] == 0.0
    np.testing.assert_allclose(c[1:], b[1:] - b.mean(), atol=1e-15)
    c = oracle.rhs_prepare(b, -1)
    assert abs(c.sum()) < 1e-12


def test_warm_start_gamma_never_worse():
    # ||x* - gamma y||_A <= ||x*||_A for any y (A-orthogonal projection).
    n = 8
    A = oracle.assemble(n, 0)
    b = oracle.rhs_prepare(synth.smoothed_rhs(n, 4), 0)
    xs = oracle.cg(A, b, tol=1e-13)[0]
    anorm = lambda e: np.sqrt(oracle.dot(e, oracle.spmv(A, e)))
    rng = np.random.default_rng(0)
    for y in (xs * (1 + 0.3 * rng.standard_normal(A.n)), rng.standard_normal(A.n), -xs):
        g = oracle.warm_start_gamma(A, b, y)
        assert anorm(xs - g * y) <= anorm(xs) * (1 + 1e-12)
    # exact prediction is recovered exactly
    assert abs(oracle.warm_start_gamma(A, b, 2.0 * xs) - 0.5) < 1e-9


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (3, 5, 2), (6, 4, 5), (1, 7, 3), (8, 8, 8)])
def test_spectral_solve_matches_dense_solves(dims):
    """The DCT solver against LAPACK on the Kronecker-sum matrix: the
    Neumann form's minimum-norm least-squares solution (null space = the
    constants, so it is the mean-zero one) and the pinned form's unique
    solution, for pins at a corner, on a face and inside, with b[pin] != 0."""
    nx, ny, nz = dims
    n = nx * ny * nz
    rng = np.random.default_rng(n)
    L = neumann_3d_dense(nx, ny, nz)
    c = rng.standard_normal(n)
    want = np.linalg.lstsq(L, c - c.mean(), rcond=None)[0]
    got = oracle.neumann_solve_spectral(dims, c)
    assert np.abs(got - want).max() <= 1e-11 * max(np.abs(want).max(), 1.0)
    assert abs(got.sum()) <= 1e-11 * n * max(np.abs(want).max(), 1.0)
    for pin in sorted({0, nx // 2, n - 1, nx // 2 + nx * (ny // 2 + ny * (nz // 2))}):
        b = rng.standard_normal(n)
        want = np.linalg.solve(pin_dense(L, pin), b)
        got = oracle.pinned_solve_spectral(dims, pin, b)
        assert np.abs(got - want).max() <= 1e-10 * max(np.abs(want).max(), 1.0), pin


@pytest.mark.parametrize("n", [4, 16, 64])
def test_spectral_solve_of_an_eigenvector(n):
    """The lowest non-constant symmetric mode: L v = 3 * 4 sin^2(pi / (2n)) v."""
    v = cos_mode(n)
    lam = 3 * 4 * np.sin(np.pi / (2 * n)) ** 2
    np.testing.assert_allclose(oracle.neumann_solve_spectral(n, v), v / lam, rtol=0, atol=1e-12 / lam)


def test_spectral_solve_agrees_with_cg():
    """32^3 pinned system, smoothed right-hand side: CG at 1e-13 and the DCT
    solve agree to within CG's own error bound (cond ~ 1e3 times 1e-13)."""
    n = 32
    b = oracle.rhs_prepare(synth.smoothed_rhs(n, 4), 0)
    A = oracle.assemble(n, 0)
    x_cg, _, _, st = oracle.cg(A, b, tol=1e-13)
    assert st == oracle.OK
    x = oracle.pinned_solve_spectral(n, 0, b)
    assert x[0] == 0.0
    assert np.linalg.norm(x - x_cg) <= 1e-9 * np.linalg.norm(x)
    r = b - oracle.spmv(A, x)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)
