"""Pins of the oracle's preconditioned CG (Sec. 3.1: PCG with a DIC or Jacobi
preconditioner) against facts fixed by the definitions, not by the oracle:

* the elimination orders are the stated bijections;
* the DIC pivots make diag(M) = diag(A) and leave A's off-diagonal entries
  unchanged, for M = (D + L) D^{-1} (D + U) built densely with numpy;
* in red-black order the pivots have a closed form (red: a_mm; black:
  a_mm - sum over red neighbours of a_mj^2 / a_jj);
* applying M^{-1} equals a dense solve with that M;
* PCG reaches the dense solution; red-black DIC PCG takes the iteration
  count of Jacobi-preconditioned CG on the black Schur complement (the
  red block of A is diagonal, so the two are the same method);
* the orders of iteration counts: natural DIC < red-black DIC < none.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def csr(A):
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def dense_dic(A, d, pos):
    """M = (D + L) D^{-1} (D + U) with L/U the entries of A before/after in the order."""
    a = A.dense()
    before = pos[None, :] < pos[:, None]
    L = np.where(before & (a != 0), a, 0.0)
    np.fill_diagonal(L, 0.0)
    U = np.where((~before) & (a != 0), a, 0.0)
    np.fill_diagonal(U, 0.0)
    D = np.diag(d)
    return (D + L) @ np.diag(1.0 / d) @ (D + U)


@pytest.mark.parametrize("dims", [(4, 3, 5), (2, 2, 2), (1, 3, 2)])
@pytest.mark.parametrize("redblack", [False, True])
def test_order_is_the_stated_bijection(dims, redblack):
    nx, ny, nz = dims
    ordv, pos = oracle.order(dims, redblack)
    n = nx * ny * nz
    assert sorted(ordv.tolist()) == list(range(n))
    assert np.array_equal(pos[ordv], np.arange(n))
    cells = [(m % nx, (m // nx) % ny, m // (nx * ny)) for m in range(n)]
    if redblack:
        want = [m for m in range(n) if sum(cells[m]) % 2 == 0] + [m for m in range(n) if sum(cells[m]) % 2 == 1]
    else:
        want = list(range(n))
    assert ordv.tolist() == want


@pytest.mark.parametrize("dims,pin", [((4, 4, 4), 0), ((3, 4, 5), 7), ((4, 3, 2), -1)])
@pytest.mark.parametrize("redblack", [False, True])
def test_dic_keeps_diagonal_and_entries(dims, pin, redblack):
    A = oracle.assemble(dims, pin)
    d = oracle.dic_factor(A, redblack)
    _, pos = oracle.order(dims, redblack)
    M = dense_dic(A, d, pos)
    a = A.dense()
    assert np.abs(np.diag(M) - np.diag(a)).max() <= 1e-13
    off = (a != 0) & ~np.eye(A.n, dtype=bool)
    assert np.abs(M[off] - a[off]).max() <= 1e-13
    assert np.all(d > 0)


@pytest.mark.parametrize("dims,pin", [((5, 4, 3), 0), ((4, 4, 4), -1), ((3, 5, 4), 9)])
def test_redblack_pivots_closed_form(dims, pin):
    A = oracle.assemble(dims, pin)
    a = A.dense()
    d = oracle.dic_factor(A, True)
    nx, ny, nz = dims
    for m in range(A.n):
        i, j, k = m % nx, (m // nx) % ny, m // (nx * ny)
        if (i + j + k) % 2 == 0:
            assert d[m] == a[m, m]
        else:
            nbrs = [c for c in range(A.n) if c != m and a[m, c] != 0]
            want = a[m, m] - sum(a[m, c] ** 2 / a[c, c] for c in nbrs)
            assert abs(d[m] - want) <= 1e-14 * abs(want)


@pytest.mark.parametrize("redblack", [False, True])
@pytest.mark.parametrize("pin", [0, -1])
def test_dic_apply_is_dense_solve(redblack, pin):
    dims = (4, 3, 4)
    A = oracle.assemble(dims, pin)
    d = oracle.dic_factor(A, redblack)
    _, pos = oracle.order(dims, redblack)
    M = dense_dic(A, d, pos)
    r = np.random.default_rng(3).standard_normal(A.n)
    z = oracle.dic_apply(A, d, r, redblack)
    assert np.abs(z - np.linalg.solve(M, r)).max() <= 1e-12 * np.abs(z).max()


@pytest.mark.parametrize("precond,redblack", [("none", True), ("jacobi", True), ("dic", False), ("dic", True)])
def test_pcg_reaches_dense_solution(precond, redblack):
    A = oracle.assemble((5, 4, 4), 0)
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    b[0] = 0.0
    x, it, rr, st = oracle.pcg(A, b, tol=1e-13, precond=precond, redblack=redblack)
    xd = np.linalg.solve(A.dense(), b)
    assert st == oracle.OK and rr <= 1e-13
    assert np.abs(x - xd).max() <= 1e-11 * np.abs(xd).max()


def schur_jacobi_cg_iters(A, b, dims, tol):
    """Jacobi-preconditioned CG on the black Schur complement (numpy)."""
    nx, ny, nz = dims
    M = csr(A)
    idx = np.arange(A.n)
    red = ((idx % nx) + (idx // nx) % ny + idx // (nx * ny)) % 2 == 0
    R, B = idx[red], idx[~red]
    Arr, Arb, Abb = M[R][:, R], M[R][:, B], M[B][:, B]
    assert abs(Arr - sp.diags(Arr.diagonal())).max() == 0  # red block diagonal
    Dr = Arr.diagonal()
    S = (Abb - Arb.T @ sp.diags(1.0 / Dr) @ Arb).tocsr()
    bS = b[B] - Arb.T @ (b[R] / Dr)
    dS = S.diagonal()
    xb = np.zeros(len(B))
    r = bS.copy()
    z = r / dS
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for k in range(1, 10000):
        q = S @ p
        a = rz / (p @ q)
        xb += a * p
        r -= a * q
        if np.linalg.norm(r) <= tol * bn:  # = ||b - A x|| once x_r is recovered
            return k
        z = r / dS
        rz2 = r @ z
        p = z + (rz2 / rz) * p
        rz = rz2
    return -1


@pytest.mark.parametrize("n,pin", [(8, 0), (12, -1)])
def test_redblack_dic_is_schur_jacobi_cg(n, pin):
    dims = (n, n, n)
    A = oracle.assemble(dims, pin)
    b = synth.smoothed_rhs(n, 1001).reshape(-1).copy()
    if pin >= 0:
        b[pin] = 0.0
    else:
        b -= b.mean()
    _, it, rr, st = oracle.pcg(A, b, tol=1e-10, precond="dic", redblack=True)
    assert st == oracle.OK
    assert abs(it - schur_jacobi_cg_iters(A, b, dims, 1e-10)) <= 1


def test_iteration_order_of_preconditioners():
    A = oracle.assemble((16, 16, 16), 0)
    b = synth.smoothed_rhs(16, 1001).reshape(-1).copy()
    b[0] = 0.0
    its = {}
    for name, pc, rb in (("none", "none", True), ("rb", "dic", True), ("nat", "dic", False)):
        _, its[name], rr, st = oracle.pcg(A, b, tol=1e-10, precond=pc, redblack=rb)
        assert st == oracle.OK and rr <= 1e-10
    assert its["nat"] < its["rb"] < its["none"]
    assert its["rb"] <= 0.6 * its["none"]
