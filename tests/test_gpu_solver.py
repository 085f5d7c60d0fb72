"""GPU parity of the matrix, SpMV, right-hand-side preparation and CG solver
against the FP64 oracle (all calls go through the C ABI).

Tolerances (each derived from the arithmetic it bounds):
* assembly, SpMV on small-integer vectors: bit-exact (all arithmetic exact);
* SpMV on real vectors: |y - y_ref| <= 2*gamma_7*(|A||x|) (two different
  rounding sequences of a 7-term dot product, u = 2^-53 or 2^-24);
* solve: true relative residual <= tol recomputed on the CPU (plus the
  rounding bound of that recomputation); pressure error vs an oracle
  solution at tol 1e-12 <= 1e-9 in relative L2 after removing the mean
  (the pressure-error bar); float64 iteration counts within 2 % + 2 of the
  oracle's (same algorithm, different summation order).
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2504_03697_amd as m
    m.load()
    return m


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def true_relres(A, b, x):
    r = b - oracle.spmv(A, x)
    return np.linalg.norm(r) / np.linalg.norm(b)


def relres_rounding(A, b, x):
    """Bound on the error of recomputing ||b - A x|| / ||b|| in float64."""
    g7 = 8 * 2.0**-53 / (1 - 8 * 2.0**-53)
    absA = oracle.Csr(A.row_ptr, A.col, np.abs(A.val), A.dims, A.pin)
    return g7 * np.linalg.norm(np.abs(b) + oracle.spmv(absA, np.abs(x))) / np.linalg.norm(b)


def mean_removed_err(x, ref):
    a = x - x.mean()
    r = ref - ref.mean()
    return np.linalg.norm(a - r) / np.linalg.norm(r)


# ---------------------------------------------------------------- assembly

@pytest.mark.parametrize("dims,pin", [((1, 1, 1), 0), ((1, 1, 1), -1), ((2, 1, 1), 1), ((5, 7, 3), 0),
                                      ((5, 7, 3), 52), ((16, 16, 16), 0), ((17, 17, 17), 0),
                                      ((17, 17, 17), -1), ((33, 20, 9), 3000), ((64, 64, 64), 0)])
def test_assembly_bitwise(lib, dims, pin):
    A = lib.assemble(dims, pin)
    ref = oracle.assemble(dims, pin)
    assert A.n == ref.n and A.nnz == ref.nnz
    rp, col, val = (host(t) for t in A.export())
    np.testing.assert_array_equal(rp, ref.row_ptr)
    np.testing.assert_array_equal(col, ref.col)
    np.testing.assert_array_equal(val, ref.val)


def test_assembly_rejects_bad_args(lib):
    with pytest.raises(lib.CfdError):
        lib.assemble((0, 4, 4))
    with pytest.raises(lib.CfdError):
        lib.assemble(4, pin=64)


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("dims", [(16, 16, 16), (17, 17, 17), (33, 9, 21), (1, 1, 1), (3, 1, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spmv_integer_vectors_bitwise(lib, dims, prec):
    A = lib.assemble(dims, 0)
    ref = oracle.assemble(dims, 0)
    rng = np.random.default_rng(11)
    x = rng.integers(-8, 9, size=ref.n).astype(np.float64)
    y_ref = oracle.spmv(ref, x)
    dt = torch.float64 if prec == "fp64" else torch.float32
    y = host(lib.spmv(A, dev(x, dt)))
    np.testing.assert_array_equal(y.astype(np.float64), y_ref)


@pytest.mark.parametrize("dims", [(40, 40, 40), (37, 29, 31)])
def test_spmv_real_vectors(lib, dims):
    A = lib.assemble(dims, 0)
    ref = oracle.assemble(dims, 0)
    absA = oracle.Csr(ref.row_ptr, ref.col, np.abs(ref.val), ref.dims, ref.pin)
    x = synth.uniform_rhs(dims, 5)
    y_ref = oracle.spmv(ref, x)
    bound64 = 2 * 7 * 2.0**-53 * oracle.spmv(absA, np.abs(x)) * 1.01
    y = host(lib.spmv(A, dev(x)))
    assert np.all(np.abs(y - y_ref) <= bound64)
    x32 = x.astype(np.float32)
    y_ref32 = oracle.spmv(ref, x32.astype(np.float64))
    bound32 = 2 * 7 * 2.0**-24 * oracle.spmv(absA, np.abs(x32.astype(np.float64))) * 1.01
    y32 = host(lib.spmv(A, dev(x32, torch.float32))).astype(np.float64)
    assert np.all(np.abs(y32 - y_ref32) <= bound32)


def test_spmv_full_size_256(lib):
    """256^3 (117M nonzeros), the launch configuration of the benchmark."""
    n = 256
    A = lib.assemble(n, 0)
    ref = oracle.assemble(n, 0)
    rng = np.random.default_rng(3)
    x = rng.integers(-4, 5, size=ref.n).astype(np.float32)
    y = host(lib.spmv(A, dev(x, torch.float32))).astype(np.float64)
    np.testing.assert_array_equal(y, oracle.spmv(ref, x.astype(np.float64)))


@pytest.mark.parametrize("dims,pin", [((256, 128, 128), 0), ((256, 17, 1000), 4 * 256 * 17 + 9 * 256 + 100),
                                      ((256, 1, 16400), 0), ((256, 16400, 1), 77), ((256, 130, 127), 256 * 130 * 127 - 1)])
def test_spmv_plane_marching_shapes(lib, dims, pin):
    """Grids with 256-cell x-rows and at least 2^22 rows take the
    plane-marching float32 SpMV: ny not a multiple of 8 and nz not a
    multiple of its 8-plane range, ny = 1 (the z offset equals the x-row
    length), nz = 1, and pins inside and at the last cell.  Integer vectors:
    bit-exact against the oracle; real vectors: within 2 gamma_7 |A||x|."""
    A = lib.assemble(dims, pin)
    ref = oracle.assemble(dims, pin)
    rng = np.random.default_rng(13)
    xi = rng.integers(-8, 9, size=ref.n).astype(np.float32)
    y = host(lib.spmv(A, dev(xi, torch.float32))).astype(np.float64)
    np.testing.assert_array_equal(y, oracle.spmv(ref, xi.astype(np.float64)))
    x32 = rng.uniform(-1, 1, size=ref.n).astype(np.float32)
    absA = oracle.Csr(ref.row_ptr, ref.col, np.abs(ref.val), ref.dims, ref.pin)
    y_ref = oracle.spmv(ref, x32.astype(np.float64))
    bound = 2 * 7 * 2.0**-24 * oracle.spmv(absA, np.abs(x32.astype(np.float64))) * 1.01
    y32 = host(lib.spmv(A, dev(x32, torch.float32))).astype(np.float64)
    assert np.all(np.abs(y32 - y_ref) <= bound)


# ---------------------------------------------------------------- symmetric storage

SYM_CASES = [((1, 1, 1), 0), ((1, 1, 1), -1), ((2, 1, 1), 1), ((3, 1, 2), 0), ((5, 7, 3), 52),
             ((16, 16, 16), 0), ((17, 17, 17), -1), ((33, 9, 21), 3000), ((40, 40, 40), 21000)]


@pytest.mark.parametrize("dims,pin", SYM_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spmv_sym_matches_full_csr(lib, dims, pin, prec):
    """The symmetric storage (diagonal + upper triangle with values, lower
    pattern only) gives the full-CSR product's bits: same terms, same
    ascending order.  Integer vectors also match the oracle exactly, real
    vectors within the summation bound."""
    A = lib.assemble(dims, pin)
    ref = oracle.assemble(dims, pin)
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(sum(dims) + pin)
    xi = rng.integers(-8, 9, size=ref.n).astype(np.float64)
    y = host(lib.spmv_sym(A, dev(xi, dt))).astype(np.float64)
    np.testing.assert_array_equal(y, oracle.spmv(ref, xi))
    xr = synth.uniform_rhs(dims, 6)
    xd = dev(xr, dt)
    ys = host(lib.spmv_sym(A, xd))
    yf = host(lib.spmv(A, xd))
    assert np.array_equal(ys, yf)
    absA = oracle.Csr(ref.row_ptr, ref.col, np.abs(ref.val), ref.dims, ref.pin)
    u = 2.0**-53 if prec == "fp64" else 2.0**-24
    xe = xr if prec == "fp64" else xr.astype(np.float32).astype(np.float64)
    bound = 2 * 7 * u * oracle.spmv(absA, np.abs(xe)) * 1.01
    assert np.all(np.abs(ys.astype(np.float64) - oracle.spmv(ref, xe)) <= bound)


def test_spmv_sym_full_size_256(lib):
    """256^3 in the benchmark's launch configuration: integer vectors, the
    oracle's product exactly; a second call reuses the stored layout."""
    n = 256
    A = lib.assemble(n, 0)
    ref = oracle.assemble(n, 0)
    rng = np.random.default_rng(4)
    x = rng.integers(-4, 5, size=ref.n).astype(np.float32)
    xd = dev(x, torch.float32)
    y1 = host(lib.spmv_sym(A, xd)).astype(np.float64)
    np.testing.assert_array_equal(y1, oracle.spmv(ref, x.astype(np.float64)))
    y2 = host(lib.spmv_sym(A, xd)).astype(np.float64)
    assert np.array_equal(y1, y2)


# ---------------------------------------------------------------- RHS preparation

@pytest.mark.parametrize("dims,pin", [((16, 16, 16), 0), ((17, 13, 11), 100), ((9, 9, 9), -1)])
def test_rhs_prepare(lib, dims, pin):
    A = lib.assemble(dims, pin)
    b = synth.uniform_rhs(dims, 2) + 0.3
    ref = oracle.rhs_prepare(b, pin)
    got = host(lib.rhs_prepare(A, dev(b)))
    np.testing.assert_allclose(got, ref, rtol=0, atol=4 * len(b) * 2.0**-53)
    if pin >= 0:
        assert got[pin] == 0.0


# ---------------------------------------------------------------- solver

CASES = [  # dims, rhs kind, seed
    ((16, 16, 16), "uniform", 0),
    ((17, 17, 17), "smoothed", 1),
    ((33, 33, 33), "smoothed", 2),
    ((24, 13, 31), "uniform", 3),
]


def make_rhs(dims, kind, seed):
    if kind == "uniform":
        b = synth.uniform_rhs(dims, seed)
    else:
        b = synth.smoothed_rhs(dims[0], seed)
    return oracle.rhs_prepare(b, 0)


@pytest.mark.parametrize("dims,kind,seed", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_parity(lib, dims, kind, seed, precision):
    tol = 1e-10
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, kind, seed)
    x_ora, it_ora, rr_ora, st = oracle.cg(ref, b, tol=tol)
    assert st == oracle.OK
    truth = oracle.cg(ref, b, tol=1e-12)[0]
    A = lib.assemble(dims, 0)
    x, info = lib.solve(A, dev(b), tol=tol, precision=precision)
    x = host(x)
    assert info["status"] == 0
    assert info["rel_residual"] <= tol
    rr = true_relres(ref, b, x)
    assert rr <= tol + relres_rounding(ref, b, x)
    assert abs(rr - info["rel_residual"]) <= 0.05 * tol + relres_rounding(ref, b, x)
    assert mean_removed_err(x, truth) <= 1e-9
    if precision == "fp64":
        assert abs(info["iters"] - it_ora) <= 2 + 0.02 * it_ora, (info["iters"], it_ora)
        np.testing.assert_allclose(x, x_ora, rtol=0, atol=1e-7 * np.abs(truth).max())
    else:
        assert info["updates"] >= 1
        assert info["iters"] <= 2.0 * it_ora + 10, (info["iters"], it_ora)


@pytest.mark.parametrize("dims,kind,seed", CASES + [((40, 40, 40), "uniform", 9), ((1, 1, 1), "uniform", 0),
                                             ((2, 3, 1), "uniform", 1)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_projected_parity(lib, dims, kind, seed, precision):
    """Projected formulation (CG on the consistent Neumann system, shifted):
    the same pinned solution, checked against the oracle's pinned CG."""
    tol = 1e-10
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, kind, seed)
    truth = oracle.cg(ref, b, tol=1e-13)[0]
    A = lib.assemble(dims, 0)
    x, info = lib.solve(A, dev(b), tol=tol, precision=precision, formulation="projected")
    x = host(x)
    assert info["status"] == 0 and info["rel_residual"] <= tol
    assert x[0] == 0.0  # b[pin] = 0: the shifted solution is exactly 0 there
    if not np.any(b):
        assert not np.any(x) and info["iters"] == 0
        return
    rr = true_relres(ref, b, x)
    assert rr <= tol + relres_rounding(ref, b, x)
    assert abs(rr - info["rel_residual"]) <= 0.05 * tol + relres_rounding(ref, b, x)
    assert mean_removed_err(x, truth) <= 1e-9 if ref.n > 1 else True
    np.testing.assert_allclose(x, truth, rtol=0, atol=1e-8 * max(np.abs(truth).max(), 1e-300))


def test_solve_projected_general_pin_value(lib):
    """b[pin] != 0 (an unprepared right-hand side): x[pin] = b[pin] exactly and
    the other rows solve the pinned system; centre pin."""
    dims = (11, 9, 7)
    pin = 5 + 11 * (4 + 9 * 3)
    ref = oracle.assemble(dims, pin)
    b = synth.uniform_rhs(dims, 4)
    b = b - b.mean()
    b[pin] = 0.37
    truth = oracle.cg(ref, b, tol=1e-13)[0]
    A = lib.assemble(dims, pin)
    for prec in ("fp64", "mixed"):
        x, info = lib.solve(A, dev(b), tol=1e-11, precision=prec, formulation="projected")
        x = host(x)
        assert info["status"] == 0
        assert x[pin] == 0.37
        np.testing.assert_allclose(x, truth, rtol=0, atol=1e-8 * np.abs(truth).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_128_smoothed(lib, precision):
    """128^3, smoothed random right-hand side (2.1M unknowns)."""
    n = 128
    ref = oracle.assemble(n, 0)
    b = make_rhs((n, n, n), "smoothed", 0)
    A = lib.assemble(n, 0)
    truth = _truth_128(ref, b)
    for form in ("pinned", "projected"):
        x, info = lib.solve(A, dev(b), tol=1e-10, precision=precision, formulation=form)
        x = host(x)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-10
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)
        assert mean_removed_err(x, truth) <= 1e-9


def test_config_128_100_standalone_solves(lib):
    """128^3 plain FP64 CG on 100 seeded Gaussian-smoothed right-hand sides
    (zero mean, tol 1e-10): every returned x's true residual, recomputed by the
    oracle's SpMV, meets the tolerance; two of the solves are compared with
    the oracle's own solve (solution and iteration count)."""
    n = 128
    ref = oracle.assemble(n, 0)
    A = lib.assemble(n, 0)
    iters = []
    for k in range(100):
        # drawn by the seeded generator on the device, prepared by the oracle
        raw = host(synth.smoothed_rhs_torch(n, 5000 + k)).reshape(-1)
        b = oracle.rhs_prepare(raw, 0)
        x, info = lib.solve(A, dev(b), tol=1e-10, precision="fp64")
        x = host(x)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-10, k
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x), k
        iters.append(info["iters"])
        if k < 2:
            truth, it, _, st = oracle.cg(ref, b, tol=1e-10)
            assert st == oracle.OK
            assert abs(info["iters"] - it) <= 2 + 0.02 * it
            tight = oracle.cg(ref, b, tol=1e-12)[0]
            assert mean_removed_err(x, tight) <= 1e-9
    print(f"128^3, 100 solves: iterations {min(iters)}..{max(iters)}, mean {np.mean(iters):.1f}")



@pytest.mark.parametrize("precision,precond", [("fp64", "none"), ("mixed", "none"), ("fp64", "dic"),
                                               ("mixed", "dic")])
@pytest.mark.parametrize("k", [37, 38, 39, 40])
def test_breakdown_returns_last_iterate(lib, precision, precond, k):
    """A breakdown at iteration k (p^T A p <= 0, forced through the testing
    option debug_breakdown_at) ends the solve with CFD_EBREAKDOWN and x = the
    iterate of k-1 updates: the same bits as a solve capped at k-1 iterations
    (CFD_ENOCONV).  k = 37..40 puts the breakdown at every position of the
    mixed path's four-deep queue of x updates."""
    from paper_2504_03697_amd._lib import CFD_EBREAKDOWN, CFD_ENOCONV
    dims = (24, 13, 31)
    b = make_rhs(dims, "uniform", 3)
    A = lib.assemble(dims, 0)
    bd = dev(b)
    xb, ib = lib.solve(A, bd, tol=1e-10, precision=precision, precond=precond, debug_breakdown_at=k,
                       raise_on_error=False)
    xc, ic = lib.solve(A, bd, tol=1e-10, precision=precision, precond=precond, max_iters=k - 1,
                       raise_on_error=False)
    assert ib["rc"] == CFD_EBREAKDOWN and ib["status"] == CFD_EBREAKDOWN and ib["iters"] == k
    assert ic["rc"] == CFD_ENOCONV and ic["iters"] == k - 1
    xb, xc = host(xb), host(xc)
    assert np.array_equal(xb, xc)
    # and that iterate is what the reported residual belongs to
    ref = oracle.assemble(dims, 0)
    rr = true_relres(ref, b, xb)
    assert abs(rr - ib["rel_residual"]) <= 1e-6 * rr


def test_solve_rejects_x_overlapping_b(lib):
    """x is written while b is still read: x = b, or any overlap, is CFD_EINVAL
    (and so is an x0 that overlaps x without being x)."""
    dims = (8, 8, 8)
    A = lib.assemble(dims, 0)
    b = dev(make_rhs(dims, "uniform", 0))
    with pytest.raises(lib.CfdError):
        lib.solve(A, b, x=b)
    buf = torch.zeros(2 * A.n, dtype=torch.float64, device="cuda")
    buf[: A.n] = b
    with pytest.raises(lib.CfdError):
        lib.solve(A, buf[: A.n], x=buf[5: 5 + A.n])
    with pytest.raises(lib.CfdError):
        lib.solve(A, b, x0=buf[: A.n], x=buf[3: 3 + A.n])
    x, info = lib.solve(A, b, x0=buf[: A.n], x=buf[: A.n])  # x0 aliasing x is allowed
    assert info["status"] == 0



def _white_truth(n, seed):
    key = ("white", n, seed)
    if key not in _TRUTH:
        ref = oracle.assemble(n, 0)
        b = make_rhs((n, n, n), "uniform", seed)
        _TRUTH[key] = (ref, b, oracle.pinned_solve_spectral(n, 0, b))
    return _TRUTH[key]


@pytest.mark.parametrize("n,seed", [(96, 0), (96, 1), (128, 1), (128, 2)])
@pytest.mark.parametrize("form", ["pinned", "projected"])
@pytest.mark.parametrize("precond", ["none", "dic"])
def test_mixed_white_noise_pressure_error(lib, n, seed, form, precond):
    """Mixed precision on white-noise (uniform[-1,1]) right-hand sides, whose
    lowest modes hold the least of b, so float32 rounding noise there weighs
    most: with the default stopping margin (0.05 tol for a right-hand side
    whose Rayleigh quotient b^T A b / b^T b exceeds 0.5) the pressure is
    within 1e-9 of the oracle's exact solution (its DCT solve; relative L2,
    mean removed) and the residual meets tol.  At a residual of 1e-10 itself these
    right-hand sides measured 1.8e-9..3e-8 (128^3)."""
    ref, b, truth = _white_truth(n, seed)
    A = lib.assemble(n, 0)
    x, info = lib.solve(A, dev(b), tol=1e-10, precision="mixed", formulation=form, precond=precond)
    x = host(x)
    assert info["stop_margin"] == 0.05  # white noise: Rayleigh quotient ~6
    assert info["status"] == 0 and info["rel_residual"] <= 0.05e-10 * 1.0001
    assert true_relres(ref, b, x) <= 0.05e-10 + relres_rounding(ref, b, x)
    e = mean_removed_err(x, truth)
    print(f"white {n}^3 seed {seed} {form} {precond}: {info['iters']} iterations, error {e:.2e}")
    assert e <= 1e-9


def test_stop_margin_option(lib):
    """stop_margin sets the residual the solve runs to (tol * margin); 1
    gives the residual-only stop, more iterations follow a smaller margin.
    Defaults: float64 1; mixed 0.05 for a rough right-hand side (white
    noise, Rayleigh quotient b^T A b / b^T b ~6 > 0.5), 1 for a smooth one
    (Gaussian-smoothed, ~0.16)."""
    n = 32
    A = lib.assemble(n, 0)
    ref = oracle.assemble(n, 0)
    b = make_rhs((n, n, n), "uniform", 5)
    bd = dev(b)
    its = []
    for m in (1.0, 0.1, 0.01):
        x, info = lib.solve(A, bd, tol=1e-10, precision="mixed", stop_margin=m)
        assert info["rel_residual"] <= 1e-10 * m
        assert true_relres(ref, b, host(x)) <= 1e-10 * m + relres_rounding(ref, b, host(x))
        its.append(info["iters"])
    assert its[0] < its[1] < its[2]
    for drv in ("steps", "persistent"):
        x, info = lib.solve(A, bd, tol=1e-10, precision="mixed", driver=drv)
        assert info["stop_margin"] == 0.05
        assert info["iters"] == lib.solve(A, bd, tol=1e-10, precision="mixed", stop_margin=0.05,
                                          driver=drv)[1]["iters"]
        bs = dev(make_rhs((n, n, n), "smoothed", 5))
        _, i_s = lib.solve(A, bs, tol=1e-10, precision="mixed", driver=drv)
        assert i_s["stop_margin"] == 1.0
        assert i_s["iters"] == lib.solve(A, bs, tol=1e-10, precision="mixed", stop_margin=1.0,
                                         driver=drv)[1]["iters"]
        for prec in ("fp64", "mixed"):
            _, i_p = lib.solve(A, bs, tol=1e-10, precision=prec, stop_margin=0.3, driver=drv)
            assert i_p["stop_margin"] == 0.3 and i_p["rel_residual"] <= 0.3e-10
    _, i64 = lib.solve(A, bd, tol=1e-10, precision="fp64")
    assert i64["stop_margin"] == 1.0
    assert i64["iters"] == lib.solve(A, bd, tol=1e-10, precision="fp64", stop_margin=1.0)[1]["iters"]
    _, idic = lib.solve(A, bd, tol=1e-10, precision="mixed", precond="dic")
    assert idic["stop_margin"] == 0.05 and idic["rel_residual"] <= 0.05e-10


def test_mixed_cavity_rhs_pressure_error(lib):
    """A cavity right-hand side (64^3, Re = 1000, after 15 oracle time steps
    from rest), built from the oracle's own step pieces (advection, viscosity,
    divergence, consistency): the mixed solve, both formulations, is within
    1e-9 of an oracle solve at 1e-12."""
    n, dt, nu = 64, 0.005, 1e-3
    S = oracle.State(n, nu=nu, lid=1.0)
    for _ in range(15):
        assert oracle.step(S, dt, tol=1e-10)[2] == oracle.OK
    ua, va, wa = oracle.advect(n, S.h, 1.0, dt, S.u, S.v, S.w)
    u, v, w = oracle.diffuse(n, S.h, 1.0, dt, nu, ua, va, wa)
    b = oracle.rhs_prepare(-(S.rho * S.h / dt) * oracle.divergence(n, u, v, w), 0)
    ref = oracle.assemble(n, 0)
    truth = oracle.cg(ref, b, tol=1e-12)[0]
    A = lib.assemble(n, 0)
    bab = float(b @ oracle.spmv(ref, b)) / float(b @ b)
    assert bab > 0.5  # a rough right-hand side: the stopping margin applies
    for form in ("pinned", "projected"):
        x, info = lib.solve(A, dev(b), tol=1e-10, precision="mixed", formulation=form)
        x = host(x)
        assert info["status"] == 0 and info["stop_margin"] == 0.05
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)
        assert mean_removed_err(x, truth) <= 1e-9, form


_TRUTH = {}


def _truth_128(ref, b):
    if "t" not in _TRUTH:
        _TRUTH["t"] = oracle.cg(ref, b, tol=1e-12)[0]
    return _TRUTH["t"]


def test_solve_256_mixed_full_size(lib):
    """256^3 (16.8M unknowns, 117M nonzeros), the benchmark's workload and
    launch configuration: mixed precision + projected formulation against the
    oracle's exact solution of the pinned system (its DCT solve, a second on
    the host; FP64 CG to 1e-12 takes minutes there); the true residual is
    recomputed by the oracle's SpMV; plain FP64 GPU CG agrees."""
    n = 256
    ref = oracle.assemble(n, 0)
    b = make_rhs((n, n, n), "smoothed", 1000)
    truth = oracle.pinned_solve_spectral(n, 0, b)
    A = lib.assemble(n, 0)
    bd = dev(b)
    x, info = lib.solve(A, bd, tol=1e-10, precision="mixed", formulation="projected")
    x = host(x)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)
    assert mean_removed_err(x, truth) <= 1e-9
    x64, info64 = lib.solve(A, bd, tol=1e-10, precision="fp64")
    x64 = host(x64)
    assert info64["status"] == 0
    assert true_relres(ref, b, x64) <= 1e-10 + relres_rounding(ref, b, x64)
    assert mean_removed_err(x64, truth) <= 1e-9
    # the headline path: mixed + projected from the learned warm start
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_2504_03697_amd", "weights", "warmstart.npy")
    xl, infol = lib.solve(A, bd, tol=1e-10, precision="mixed", formulation="projected",
                          net=lib.Net(np.load(wpath)))
    xl = host(xl)
    assert infol["status"] == 0 and infol["used_fallback"] == 0 and infol["rel_residual"] <= 1e-10
    assert true_relres(ref, b, xl) <= 1e-10 + relres_rounding(ref, b, xl)
    assert mean_removed_err(xl, truth) <= 1e-9
    # the DIC-preconditioned solve (red-black order) at the same size
    for precision in ("mixed", "fp64"):
        xd, infod = lib.solve(A, bd, tol=1e-10, precision=precision, formulation="projected", precond="dic")
        xd = host(xd)
        assert infod["status"] == 0 and infod["iters"] < 0.6 * info["iters"]
        assert true_relres(ref, b, xd) <= 1e-10 + relres_rounding(ref, b, xd)
        assert mean_removed_err(xd, truth) <= 1e-9


def test_config_256_mixed_20_solves(lib):
    """256^3 mixed precision (projected formulation) on 20 seeded smoothed
    right-hand sides: every returned x's true FP64 residual, recomputed by the
    oracle's SpMV, meets 1e-10, and its pressure error against the oracle's
    exact solution of the pinned system (DCT solve), mean removed, is within
    1e-9."""
    n = 256
    ref = oracle.assemble(n, 0)
    A = lib.assemble(n, 0)
    worst, worst_e = 0.0, 0.0
    for k in range(20):
        raw = host(synth.smoothed_rhs_torch(n, 7000 + k)).reshape(-1)
        b = oracle.rhs_prepare(raw, 0)
        print(f"256^3 mixed, right-hand side {k}", flush=True)
        x, info = lib.solve(A, dev(b), tol=1e-10, precision="mixed", formulation="projected")
        x = host(x)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-10, k
        rr = true_relres(ref, b, x)
        assert rr <= 1e-10 + relres_rounding(ref, b, x), k
        e = mean_removed_err(x, oracle.pinned_solve_spectral(n, 0, b))
        assert e <= 1e-9, (k, e)
        worst, worst_e = max(worst, rr), max(worst_e, e)
    print(f"256^3 mixed, 20 solves: worst true relative residual {worst:.3e}, worst pressure error {worst_e:.3e}")


def test_solve_384_combined_size(lib):
    """384^3 (56.6M unknowns, 395M nonzeros): mixed + projected converges and
    its true residual, recomputed by the oracle's SpMV, meets the tolerance."""
    n = 384
    ref = oracle.assemble(n, 0)
    b = make_rhs((n, n, n), "smoothed", 7)
    A = lib.assemble(n, 0)
    for pc in ("none", "dic"):
        x, info = lib.solve(A, dev(b), tol=1e-10, precision="mixed", formulation="projected", precond=pc)
        x = host(x)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-10
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)


def test_solve_512_largest_grid(lib):
    """512^3 (134M unknowns, 938M nonzeros, beyond every configured size; the
    int32 CSR holds up to N = 674): the headline path, mixed + learned +
    projected, and the DIC-preconditioned solve converge; their true
    residuals, recomputed by the oracle's SpMV, meet the tolerance."""
    n = 512
    ref = oracle.assemble(n, 0)
    assert ref.nnz == 7 * n**3 - 6 * n**2 - 6
    A = lib.assemble(n, 0)
    raw = host(synth.smoothed_rhs_torch(n, 2024)).reshape(-1)
    b = oracle.rhs_prepare(raw, 0)
    del raw
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_2504_03697_amd", "weights", "warmstart.npy")
    bd = dev(b)
    for kw in (dict(net=lib.Net(np.load(wpath))), dict(precond="dic")):
        x, info = lib.solve(A, bd, tol=1e-10, precision="mixed", formulation="projected", **kw)
        x = host(x)
        assert info["status"] == 0 and info["rel_residual"] <= 1e-10
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)
        assert x[0] == 0.0
        print(f"512^3 {list(kw)}: {info['iters']} iterations, {info['seconds']:.2f} s")
        del x
    # the products at this size, on integer vectors: the oracle's bits, from
    # the full CSR in both precisions and from the symmetric storage
    xi = np.random.default_rng(7).integers(-4, 5, size=ref.n).astype(np.float32)
    y_ref = oracle.spmv(ref, xi.astype(np.float64))
    x32 = dev(xi, torch.float32)
    assert np.array_equal(host(lib.spmv(A, x32)).astype(np.float64), y_ref)
    assert np.array_equal(host(lib.spmv_sym(A, x32)).astype(np.float64), y_ref)
    assert np.array_equal(host(lib.spmv(A, dev(xi.astype(np.float64)))), y_ref)


def test_solve_edge_cases(lib):
    dims = (12, 12, 12)
    ref = oracle.assemble(dims, 0)
    A = lib.assemble(dims, 0)
    # b = 0 -> x = 0 after 0 iterations, whatever x0 is
    x0 = dev(np.ones(ref.n))
    x, info = lib.solve(A, dev(np.zeros(ref.n)), x0=x0)
    assert info["iters"] == 0 and not host(x).any() and info["rel_residual"] == 0.0
    # starting at the solution: no iteration
    b = make_rhs(dims, "uniform", 4)
    xs = oracle.cg(ref, b, tol=1e-13)[0]
    for prec in ("fp64", "mixed"):
        x, info = lib.solve(A, dev(b), x0=dev(xs), precision=prec)
        assert info["iters"] == 0 and info["rel_residual"] <= 1e-10
    # x0 aliasing x
    xa = dev(np.zeros(ref.n))
    x, info = lib.solve(A, dev(b), x0=xa, x=xa)
    assert x.data_ptr() == xa.data_ptr() and info["rel_residual"] <= 1e-10
    # iteration cap
    x, info = lib.solve(A, dev(b), max_iters=3, raise_on_error=False)
    assert info["rc"] == lib._lib.CFD_ENOCONV and info["iters"] == 3
    xr = oracle.cg(ref, b, max_iters=3)[0]
    np.testing.assert_allclose(host(x), xr, rtol=0, atol=1e-12 * np.abs(xr).max())
    # non-finite input
    bn = b.copy()
    bn[7] = np.nan
    x, info = lib.solve(A, dev(bn), raise_on_error=False)
    assert info["rc"] == lib._lib.CFD_ENONFINITE
    # the singular matrix is rejected
    with pytest.raises(lib.CfdError):
        lib.solve(lib.assemble(dims, -1), dev(b))
    # one cell
    A1 = lib.assemble(1, 0)
    x, info = lib.solve(A1, dev(np.zeros(1)))
    assert info["iters"] == 0


def test_solve_deterministic(lib):
    dims = (29, 31, 27)
    A = lib.assemble(dims, 0)
    b = dev(make_rhs(dims, "uniform", 8))
    for prec in ("fp64", "mixed"):
        x1, i1 = lib.solve(A, b, precision=prec)
        x2, i2 = lib.solve(A, b, precision=prec)
        assert i1["iters"] == i2["iters"]
        assert torch.equal(x1, x2)


def test_solve_timing_samples(lib):
    A = lib.assemble(48, 0)
    b = dev(make_rhs((48, 48, 48), "uniform", 1))
    x, info = lib.solve(A, b, timing=True)
    assert info["spmv_samples"] >= 1 and info["spmv_ms"] > 0
    assert info["seconds"] > 0


# ---------------------------------------------------------------- persistent driver

@pytest.mark.parametrize("dims,kind,seed", CASES + [((40, 40, 40), "uniform", 9), ((1, 1, 1), "uniform", 0),
                                             ((2, 3, 1), "uniform", 1), ((64, 64, 64), "smoothed", 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("formulation", ["pinned", "projected"])
def test_persistent_driver_parity(lib, dims, kind, seed, precision, formulation):
    """The persistent driver (one cooperative launch, grid barriers between
    the steps) against the oracle: the same bars as the launch-per-step
    driver, and the same iteration count up to the rounding of different
    partial-sum groupings (float64: 2 % + 2; mixed: 10 % + 5)."""
    tol = 1e-10
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, kind, seed)
    truth = oracle.cg(ref, b, tol=1e-13)[0]
    A = lib.assemble(dims, 0)
    print(f"persistent {dims} {kind} {seed} {precision} {formulation}", flush=True)
    x, info = lib.solve(A, dev(b), tol=tol, precision=precision, formulation=formulation, driver="persistent")
    x = host(x)
    assert info["status"] == 0
    if not np.any(b):
        assert not np.any(x) and info["iters"] == 0
        return
    assert info["stop_margin"] == (0.05 if precision == "mixed" and kind == "uniform" else 1.0)
    stop = tol * info["stop_margin"]
    assert info["rel_residual"] <= stop
    rr = true_relres(ref, b, x)
    assert rr <= stop + relres_rounding(ref, b, x)
    assert abs(rr - info["rel_residual"]) <= 0.05 * stop + relres_rounding(ref, b, x)
    if ref.n > 1:
        assert mean_removed_err(x, truth) <= 1e-9
    _, it_steps = lib.solve(A, dev(b), tol=tol, precision=precision, formulation=formulation, driver="steps")
    # float64: the same iteration up to rounding; mixed: float32 rounding of
    # different partial-sum groupings moves the count further
    slack = 2 + 0.02 * it_steps["iters"] if precision == "fp64" else 5 + 0.1 * it_steps["iters"]
    assert abs(info["iters"] - it_steps["iters"]) <= slack, (info["iters"], it_steps["iters"])
    if precision == "fp64" and formulation == "pinned":
        _, it_ora, _, st = oracle.cg(ref, b, tol=tol)
        assert abs(info["iters"] - it_ora) <= 2 + 0.02 * it_ora, (info["iters"], it_ora)


def test_persistent_driver_warm_start_and_errors(lib):
    """Persistent driver with a warm-start network and with x0, b = 0, the
    iteration cap and a breakdown: the same outcomes as the launch-per-step
    driver."""
    from paper_2504_03697_amd._lib import CFD_EBREAKDOWN, CFD_ENOCONV
    dims = (20, 18, 22)
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, "uniform", 8)
    A = lib.assemble(dims, 0)
    bd = dev(b)
    net = lib.Net(synth.net_init(3))
    for drv in ("steps", "persistent"):
        x, info = lib.solve(A, bd, tol=1e-10, precision="mixed", formulation="projected", net=net, driver=drv)
        assert info["status"] == 0 and info["gamma"] != 0.0
        assert true_relres(ref, b, host(x)) <= 0.05e-10 + relres_rounding(ref, b, host(x))
    x0 = dev(synth.uniform_rhs(dims, 9))
    xs, i_s = lib.solve(A, bd, x0=x0, tol=1e-10, precision="fp64", driver="steps")
    xp, i_p = lib.solve(A, bd, x0=x0, tol=1e-10, precision="fp64", driver="persistent")
    assert abs(i_s["iters"] - i_p["iters"]) <= 2
    np.testing.assert_allclose(host(xp), host(xs), rtol=0, atol=1e-8 * np.abs(host(xs)).max())
    # deterministic: every decision comes from fixed-order sums
    x1, i1 = lib.solve(A, bd, tol=1e-10, precision="mixed", driver="persistent")
    x2, i2 = lib.solve(A, bd, tol=1e-10, precision="mixed", driver="persistent")
    assert i1["iters"] == i2["iters"] and torch.equal(x1, x2)
    z, iz = lib.solve(A, dev(np.zeros(ref.n)), tol=1e-10, precision="mixed", driver="persistent")
    assert iz["iters"] == 0 and not np.any(host(z))
    xc, ic = lib.solve(A, bd, tol=1e-10, precision="mixed", max_iters=30, driver="persistent", raise_on_error=False)
    assert ic["rc"] == CFD_ENOCONV and ic["iters"] == 30
    x64p, _ = lib.solve(A, bd, tol=1e-10, precision="fp64", max_iters=30, driver="persistent", raise_on_error=False)
    x64s, _ = lib.solve(A, bd, tol=1e-10, precision="fp64", max_iters=30, driver="steps", raise_on_error=False)
    assert np.abs(host(x64p) - host(x64s)).max() <= 1e-10 * np.abs(host(x64s)).max()
    xb, ib = lib.solve(A, bd, tol=1e-10, precision="mixed", debug_breakdown_at=31, driver="persistent",
                       raise_on_error=False)
    assert ib["rc"] == CFD_EBREAKDOWN and ib["iters"] == 31
    assert np.array_equal(host(xb), host(xc))


def test_persistent_driver_barrier_timeout_is_an_error(lib):
    """A grid barrier that waits longer than its poll limit ends the solve
    with CFD_EHIP instead of waiting on (forced here with a one-poll limit:
    every workgroup still leaves the kernel), and the next solve on the same
    handle is unaffected."""
    from paper_2504_03697_amd._lib import CFD_EHIP
    dims = (16, 16, 16)  # 16 workgroups
    b = make_rhs(dims, "uniform", 0)
    A = lib.assemble(dims, 0)
    bd = dev(b)
    x, info = lib.solve(A, bd, tol=1e-10, precision="fp64", driver="persistent", barrier_spins=1,
                        raise_on_error=False)
    assert info["rc"] == CFD_EHIP
    x, info = lib.solve(A, bd, tol=1e-10, precision="fp64", driver="persistent")
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10


RESIDENT_CASES = [  # dims, rhs kind, seed (at most 4096 cells)
    ((16, 16, 16), "uniform", 0),
    ((16, 16, 16), "smoothed", 5),
    ((15, 15, 15), "smoothed", 1),
    ((24, 13, 13), "uniform", 3),
    ((31, 11, 7), "uniform", 4),
    ((64, 64, 1), "uniform", 6),
    ((1, 1, 1), "uniform", 0),
    ((2, 1, 1), "uniform", 2),
    ((3, 5, 2), "uniform", 7),
]


@pytest.mark.parametrize("dims,kind,seed", RESIDENT_CASES)
@pytest.mark.parametrize("formulation", ["pinned", "projected"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_driver_parity(lib, dims, kind, seed, formulation, precision):
    """The resident driver (one workgroup, matrix and vectors in registers
    and LDS) against the oracle: true residual <= tol times the stopping
    margin, pressure error <= 1e-9, and iteration counts within 2 % + 2
    (float64; mixed: 10 % + 5, float32 rounding of other groupings) of the
    launch-per-step driver's and, float64 pinned, the oracle's CG."""
    tol = 1e-10
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, kind, seed)
    A = lib.assemble(dims, 0)
    print(f"resident {dims} {kind} {seed} {formulation} {precision}", flush=True)
    x, info = lib.solve(A, dev(b), tol=tol, precision=precision, formulation=formulation, driver="resident")
    x = host(x)
    assert info["status"] == 0
    if not np.any(b):
        assert not np.any(x) and info["iters"] == 0
        return
    _, it_steps = lib.solve(A, dev(b), tol=tol, precision=precision, formulation=formulation, driver="steps")
    assert info["stop_margin"] == it_steps["stop_margin"]
    stop = tol * info["stop_margin"]
    assert info["rel_residual"] <= stop
    assert x[0] == 0.0
    rr = true_relres(ref, b, x)
    assert rr <= stop + relres_rounding(ref, b, x)
    assert abs(rr - info["rel_residual"]) <= 0.05 * stop + relres_rounding(ref, b, x)
    if ref.n > 1:
        truth = oracle.pinned_solve_spectral(dims, 0, b)
        assert mean_removed_err(x, truth) <= 1e-9
    slack = 2 + 0.02 * it_steps["iters"] if precision == "fp64" else 5 + 0.1 * it_steps["iters"]
    assert abs(info["iters"] - it_steps["iters"]) <= slack, (info["iters"], it_steps["iters"])
    if precision == "fp64" and formulation == "pinned":
        _, it_ora, _, st = oracle.cg(ref, b, tol=tol)
        assert st == oracle.OK
        assert abs(info["iters"] - it_ora) <= 2 + 0.02 * it_ora, (info["iters"], it_ora)


@pytest.mark.parametrize("pin", [1, 8 * 9 * 3 + 9 * 4 + 4, 9 * 8 * 7 - 1])
def test_resident_driver_pin_positions(lib, pin):
    """Pinned cell on a face, inside and at the far corner: the projected
    formulation's correction rows (the pin and its neighbours) are handled
    in the resident kernel as in the other drivers."""
    dims = (9, 8, 7)
    ref = oracle.assemble(dims, pin)
    b = oracle.rhs_prepare(synth.uniform_rhs(dims, 11), pin)
    truth = oracle.pinned_solve_spectral(dims, pin, b)
    A = lib.assemble(dims, pin)
    for form in ("pinned", "projected"):
        x, info = lib.solve(A, dev(b), tol=1e-10, precision="fp64", formulation=form, driver="resident")
        x = host(x)
        assert info["status"] == 0 and x[pin] == 0.0
        assert true_relres(ref, b, x) <= 1e-10 + relres_rounding(ref, b, x)
        assert mean_removed_err(x, truth) <= 1e-9


def test_resident_driver_options_and_errors(lib):
    """Resident driver with x0, a warm-start network, b = 0, a stopping
    margin, the iteration cap and a forced breakdown: the outcomes of the
    launch-per-step driver, in both precisions.  Grids up to 4096 cells take
    it by default; a larger grid asked to take it is an error."""
    from paper_2504_03697_amd._lib import CFD_EBREAKDOWN, CFD_EINVAL, CFD_ENOCONV
    dims = (16, 16, 16)
    ref = oracle.assemble(dims, 0)
    b = make_rhs(dims, "uniform", 8)
    A = lib.assemble(dims, 0)
    bd = dev(b)
    x0 = dev(synth.uniform_rhs(dims, 9))
    xs, i_s = lib.solve(A, bd, x0=x0, tol=1e-10, precision="fp64", driver="steps")
    xr, i_r = lib.solve(A, bd, x0=x0, tol=1e-10, precision="fp64", driver="resident")
    assert i_r["status"] == 0 and abs(i_s["iters"] - i_r["iters"]) <= 2
    assert i_r["init_residual"] == pytest.approx(i_s["init_residual"], rel=1e-12)
    np.testing.assert_allclose(host(xr), host(xs), rtol=0, atol=1e-8 * np.abs(host(xs)).max())
    net = lib.Net(synth.net_init(3))
    for form in ("pinned", "projected"):
        xn, i_n = lib.solve(A, bd, tol=1e-10, precision="fp64", formulation=form, net=net, driver="resident")
        _, i_ns = lib.solve(A, bd, tol=1e-10, precision="fp64", formulation=form, net=net, driver="steps")
        assert i_n["status"] == 0 and i_n["gamma"] == i_ns["gamma"] and i_n["used_fallback"] == i_ns["used_fallback"]
        assert true_relres(ref, b, host(xn)) <= 1e-10 + relres_rounding(ref, b, host(xn))
    z, iz = lib.solve(A, dev(np.zeros(ref.n)), tol=1e-10, precision="fp64", driver="resident")
    assert iz["status"] == 0 and iz["iters"] == 0 and not np.any(host(z))
    xm, im = lib.solve(A, bd, tol=1e-10, precision="fp64", stop_margin=0.1, driver="resident")
    assert im["stop_margin"] == 0.1 and im["rel_residual"] <= 1e-11
    assert true_relres(ref, b, host(xm)) <= 1e-11 + relres_rounding(ref, b, host(xm))
    # the iteration cap and a breakdown leave the same iterate
    xc, ic = lib.solve(A, bd, tol=1e-10, precision="fp64", max_iters=30, driver="resident", raise_on_error=False)
    assert ic["rc"] == CFD_ENOCONV and ic["iters"] == 30
    xcs, _ = lib.solve(A, bd, tol=1e-10, precision="fp64", max_iters=30, driver="steps", raise_on_error=False)
    assert np.abs(host(xc) - host(xcs)).max() <= 1e-10 * np.abs(host(xcs)).max()
    xb, ib = lib.solve(A, bd, tol=1e-10, precision="fp64", debug_breakdown_at=31, driver="resident",
                       raise_on_error=False)
    assert ib["rc"] == CFD_EBREAKDOWN and ib["iters"] == 31
    assert np.array_equal(host(xb), host(xc))
    # deterministic, and the default at this size
    for prec in ("fp64", "mixed"):
        x1, i1 = lib.solve(A, bd, tol=1e-10, precision=prec, driver="resident")
        x2, i2 = lib.solve(A, bd, tol=1e-10, precision=prec)
        assert i1["iters"] == i2["iters"] and torch.equal(x1, x2)
    # mixed: warm start, b = 0, the cap and a breakdown at each position of
    # the update queue the other drivers keep
    for form in ("pinned", "projected"):
        xn, i_n = lib.solve(A, bd, tol=1e-10, precision="mixed", formulation=form, net=net, driver="resident")
        assert i_n["status"] == 0 and i_n["stop_margin"] == 0.05 and i_n["updates"] >= 1
        assert true_relres(ref, b, host(xn)) <= 0.05e-10 + relres_rounding(ref, b, host(xn))
    z, iz = lib.solve(A, dev(np.zeros(ref.n)), tol=1e-10, precision="mixed", driver="resident")
    assert iz["status"] == 0 and iz["iters"] == 0 and not np.any(host(z))
    for k in (37, 38, 39, 40):
        xc, ic = lib.solve(A, bd, tol=1e-10, precision="mixed", max_iters=k - 1, driver="resident",
                           raise_on_error=False)
        assert ic["rc"] == CFD_ENOCONV and ic["iters"] == k - 1
        xb, ib = lib.solve(A, bd, tol=1e-10, precision="mixed", debug_breakdown_at=k, driver="resident",
                           raise_on_error=False)
        assert ib["rc"] == CFD_EBREAKDOWN and ib["iters"] == k
        assert np.array_equal(host(xb), host(xc))
    A17 = lib.assemble(17, 0)
    _, e2 = lib.solve(A17, dev(make_rhs((17, 17, 17), "uniform", 1)), tol=1e-10, precision="fp64", driver="resident",
                      raise_on_error=False)
    assert e2["rc"] == CFD_EINVAL
