"""Pins of the oracle's fractional time step (staggered grid, Sec. 3.1).

Checks use facts that hold for the method whatever its implementation:
the projection leaves a discretely divergence-free field (up to the solve
tolerance), wall-normal faces stay zero, a quiescent cavity stays at rest,
the cavity is mirror-symmetric in z, semi-Lagrangian advection of a shear
flow along its own streamlines is the identity, explicit diffusion of a
quadratic profile adds exactly 2*nu*dt, and the projected divergence obeys
D_new = D + (dt/(rho h)) * A_neu p.
"""
import numpy as np
import pytest

import oracle


def shapes(n):
    return oracle.face_shapes((n, n, n))


def u_index(n, i, j, k):
    return i + (n + 1) * (j + n * k)


def test_quiescent_cavity_stays_at_rest():
    S = oracle.State(8, nu=0.01, lid=0.0)
    S.p[:] = 0.0
    for _ in range(3):
        it, rr, st = oracle.step(S, 0.005)
        assert st == oracle.OK and it == 0
    assert not S.u.any() and not S.v.any() and not S.w.any()


def _run_cavity(n, steps, nu=0.01, dt=0.005, lid=1.0):
    S = oracle.State(n, nu=nu, lid=lid)
    for _ in range(steps):
        it, rr, st = oracle.step(S, dt, tol=1e-12)
        assert st == oracle.OK and rr <= 1e-12
    return S


def test_divergence_free_and_walls():
    n = 10
    S = _run_cavity(n, 3)
    D = oracle.divergence(n, S.u, S.v, S.w)
    # the projection removes the divergence up to the solve tolerance
    scale = np.abs(S.u).max()
    assert np.abs(D).max() <= 1e-9 * scale
    u = S.u.reshape(n, n, n + 1)
    v = S.v.reshape(n, n + 1, n)
    w = S.w.reshape(n + 1, n, n)
    assert not u[:, :, 0].any() and not u[:, :, n].any()
    assert not v[:, 0, :].any() and not v[:, n, :].any()
    assert not w[0].any() and not w[n].any()
    assert np.abs(S.u).max() > 0.01  # the lid did drive a flow


def test_z_mirror_symmetry():
    n = 8
    S = _run_cavity(n, 3)
    u = S.u.reshape(n, n, n + 1)
    v = S.v.reshape(n, n + 1, n)
    w = S.w.reshape(n + 1, n, n)
    np.testing.assert_allclose(u, u[::-1], atol=1e-10)
    np.testing.assert_allclose(v, v[::-1], atol=1e-10)
    np.testing.assert_allclose(w, -w[::-1], atol=1e-10)


def test_advection_of_shear_flow_is_identity():
    # u = f(y), v = w = 0: back-traces move along x only, where u is constant.
    n = 10
    h = 1.0 / n
    su, sv, sw, _ = shapes(n)
    y = (np.arange(n) + 0.5) * h
    u = np.zeros((n, n, n + 1))
    u[:, :, 1:n] = (0.3 + 0.5 * y)[None, :, None]
    u = u.reshape(-1)
    dt = 0.5 * h / 0.8  # departure stays within one cell
    un, vn, wn = oracle.advect(n, h, 0.0, dt, u, np.zeros(sv), np.zeros(sw))
    ref = u.reshape(n, n, n + 1)
    got = un.reshape(n, n, n + 1)
    np.testing.assert_allclose(got[:, :, 2:n], ref[:, :, 2:n], atol=1e-15)
    assert not vn.any() and not wn.any()


def test_advection_zero_velocity_identity():
    n = 6
    h = 1.0 / n
    su, sv, sw, _ = shapes(n)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(su)
    u.reshape(n, n, n + 1)[:, :, [0, n]] = 0.0
    un, _, _ = oracle.advect(n, h, 0.0, 0.0, u, np.zeros(sv), np.zeros(sw))
    # the face position (j + 1/2) h / h - 1/2 is exact only up to rounding
    np.testing.assert_allclose(un, u, rtol=0, atol=1e-14)


def test_diffusion_of_quadratic_profile():
    n = 10
    h = 1.0 / n
    su, sv, sw, _ = shapes(n)
    y = (np.arange(n) + 0.5) * h
    u = np.zeros((n, n, n + 1))
    u[:, :, 1:n] = (y * y)[None, :, None]
    dt, nu = 1e-3, 0.05
    un, _, _ = oracle.diffuse(n, h, 0.0, dt, nu, u.reshape(-1), np.zeros(sv), np.zeros(sw))
    got = un.reshape(n, n, n + 1)
    # away from the x walls (which are 0 faces) and the y/z walls (ghosts)
    np.testing.assert_allclose(got[1:n - 1, 1:n - 1, 2:n - 1], (u + 2 * nu * dt)[1:n - 1, 1:n - 1, 2:n - 1],
                               rtol=0, atol=1e-14)


def test_projection_identity():
    n = 8
    h = 1.0 / n
    rho, dt = 1.3, 0.01
    su, sv, sw, sp = shapes(n)
    rng = np.random.default_rng(1)
    u, v, w = rng.standard_normal(su), rng.standard_normal(sv), rng.standard_normal(sw)
    u.reshape(n, n, n + 1)[:, :, [0, n]] = 0
    v.reshape(n, n + 1, n)[:, [0, n], :] = 0
    w.reshape(n + 1, n, n)[[0, n]] = 0
    p = rng.standard_normal(sp)
    D = oracle.divergence(n, u, v, w)
    u2, v2, w2 = oracle.correct(n, h, rho, dt, p, u, v, w)
    D2 = oracle.divergence(n, u2, v2, w2)
    Aneu = oracle.assemble(n, -1)
    np.testing.assert_allclose(D2, D + dt / (rho * h) * oracle.spmv(Aneu, p), atol=1e-12)


def test_lid_ghost_sets_tangential_shear():
    # one step from rest: only the lid drives the flow, through diffusion of
    # the ghost value 2U - u at the top row; u right below the lid grows by
    # dt*nu*(2U)/h^2 (advection of a zero field does nothing).
    n = 8
    h = 1.0 / n
    su, sv, sw, _ = shapes(n)
    dt, nu, U = 1e-3, 0.01, 1.0
    ua, va, wa = oracle.advect(n, h, U, dt, np.zeros(su), np.zeros(sv), np.zeros(sw))
    un, _, _ = oracle.diffuse(n, h, U, dt, nu, ua, va, wa)
    got = un.reshape(n, n, n + 1)
    np.testing.assert_allclose(got[:, n - 1, 1:n], dt * nu * 2 * U / h**2, rtol=1e-14)
    assert not got[:, : n - 1, :].any()


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_wall_ghosts_by_diffusion(comp):
    # A uniform tangential value c on every interior face of one component:
    # explicit diffusion changes a face only through the ghosts beyond the
    # walls it touches, each contributing (ghost - c) = (2 U_wall - 2c).
    n, c, U = 6, 0.7, 0.4
    h = 1.0 / n
    dt, nu = 1e-3, 0.02
    su, sv, sw, _ = shapes(n)
    f = [np.zeros(su), np.zeros(sv), np.zeros(sw)]
    dims = [(n, n, n + 1), (n, n + 1, n), (n + 1, n, n)]  # (k, j, i) views
    a = f[comp].reshape(dims[comp])
    if comp == 0:
        a[:, :, 1:n] = c
    elif comp == 1:
        a[:, 1:n, :] = c
    else:
        a[1:n] = c
    out = oracle.diffuse(n, h, U, dt, nu, *f)[comp].reshape(dims[comp])
    coef = dt * nu / h**2
    k_, j_, i_ = np.meshgrid(*(np.arange(d) for d in dims[comp]), indexing="ij")
    expect = np.full(dims[comp], c)
    # tangential walls of this component: the two axes other than its own
    axes = {0: [(j_, n), (k_, n)], 1: [(i_, n), (k_, n)], 2: [(i_, n), (j_, n)]}[comp]
    for which, (idx, m) in enumerate(axes):
        lo = idx == 0
        hi = idx == m - 1
        lid = comp == 0 and which == 0  # u at the top wall y = 1 (j = n-1 side)
        expect = expect + coef * np.where(lo, -2 * c, 0.0)
        expect = expect + coef * np.where(hi, (2 * U if lid else 0.0) - 2 * c, 0.0)
    # faces next to the component's own (normal) walls see a zero wall face
    own = {0: i_, 1: j_, 2: k_}[comp]
    expect = expect + coef * np.where(own == 1, -c, 0.0) + coef * np.where(own == n - 1, -c, 0.0)
    interior = (own >= 1) & (own <= n - 1)
    np.testing.assert_allclose(out[interior], expect[interior], rtol=0, atol=1e-15)
    assert not out[~interior].any()


def _face_coords(dims, h, comp):
    """Physical coordinates of every face of one component, in storage order
    (x fastest): u faces sit at (i h, (j+1/2) h, (k+1/2) h), v faces at
    ((i+1/2) h, j h, (k+1/2) h), w faces at ((i+1/2) h, (j+1/2) h, k h)."""
    nx, ny, nz = dims
    fx, fy, fz = nx + (comp == 0), ny + (comp == 1), nz + (comp == 2)
    k, j, i = np.meshgrid(np.arange(fz), np.arange(fy), np.arange(fx), indexing="ij")
    x = (i + (0.0 if comp == 0 else 0.5)) * h
    y = (j + (0.0 if comp == 1 else 0.5)) * h
    z = (k + (0.0 if comp == 2 else 0.5)) * h
    return (i, j, k), (x.reshape(-1), y.reshape(-1), z.reshape(-1))


@pytest.mark.parametrize("dims", [(12, 10, 14), (9, 13, 11)])
def test_advection_of_linear_fields_is_exact(dims):
    """Semi-Lagrangian advection (Sec. 3.1) of a velocity whose three
    components are affine functions of position.  Trilinear interpolation
    reproduces an affine function exactly, so on every face whose sampling
    stencils stay among real faces, the advected value must equal the
    component's affine function at the departure point X - dt V(X), with V(X)
    the affine velocity at the face position X.  Every component depends on
    all three coordinates, so a wrong half-cell offset when one component is
    sampled at another component's faces, or a wrong weight in any
    direction, moves the departure point and fails this check."""
    nx, ny, nz = dims
    h = 1.0 / max(dims)
    # u = a0 + a.(x, y, z), v = b0 + b.(x, y, z), w = c0 + c.(x, y, z)
    coef = np.array([[0.30, 0.20, -0.50, 0.40],
                     [-0.20, 0.60, 0.10, -0.30],
                     [0.25, -0.40, 0.35, 0.15]])

    def field(comp, x, y, z):
        c = coef[comp]
        return c[0] + c[1] * x + c[2] * y + c[3] * z

    # |V| <= 0.3 + 0.2 + 0.5 + 0.4 < 1.5 on the unit box; dt keeps every
    # departure point within 0.4 h of its face
    dt = 0.4 * h / 1.5
    comps = [_face_coords(dims, h, c) for c in range(3)]
    f = [field(c, *comps[c][1]) for c in range(3)]
    out = oracle.advect(dims, h, 0.0, dt, *f)
    checked = 0
    for c in range(3):
        (i, j, k), (x, y, z) = comps[c]
        i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
        V = [field(d, x, y, z) for d in range(3)]
        xd, yd, zd = x - dt * V[0], y - dt * V[1], z - dt * V[2]
        expect = field(c, xd, yd, zd)
        # two faces of margin from every wall: all sampling corners (at X and
        # at the departure point, for all three components) are real faces
        m = ((i >= 2) & (i <= nx + (c == 0) - 3) & (j >= 2) & (j <= ny + (c == 1) - 3)
             & (k >= 2) & (k <= nz + (c == 2) - 3))
        scale = np.abs(expect[m]).max()
        np.testing.assert_allclose(out[c][m], expect[m], rtol=0, atol=1e-14 * scale)
        # the check is not vacuous: the departure moved every value
        assert np.all(np.abs(f[c][m] - expect[m]) > 1e-6)
        checked += int(m.sum())
    assert checked > 500


def test_random_flow_generator():
    """synth.random_flow: the three face arrays in their sizes, values in
    [-amp, amp], wall-normal faces zero, the same arrays for the same seed."""
    import synth
    dims = (5, 4, 3)
    nx, ny, nz = dims
    u, v, w = synth.random_flow(dims, 11, amp=0.5)
    su, sv, sw, _ = oracle.face_shapes(dims)
    assert (u.size, v.size, w.size) == (su, sv, sw)
    for a in (u, v, w):
        assert np.abs(a).max() <= 0.5 and np.abs(a).max() > 0
    U, V, W = u.reshape(nz, ny, nx + 1), v.reshape(nz, ny + 1, nx), w.reshape(nz + 1, ny, nx)
    assert not U[:, :, 0].any() and not U[:, :, nx].any()
    assert not V[:, 0, :].any() and not V[:, ny, :].any()
    assert not W[0].any() and not W[nz].any()
    u2, v2, w2 = synth.random_flow(dims, 11, amp=0.5)
    assert np.array_equal(u, u2) and np.array_equal(v, v2) and np.array_equal(w, w2)
    assert not np.array_equal(u, synth.random_flow(dims, 12, amp=0.5)[0])
