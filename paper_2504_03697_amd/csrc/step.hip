// One fractional time step on the staggered grid (Sec. 3.1 of the paper):
// forces -> semi-Lagrangian advection -> (viscosity) -> pressure correction
// (divergence, Poisson solve, gradient correction).  Every stage is a device
// kernel; the Poisson solve is the library's CG (cfd_solve).
//
// Face layouts (x fastest over each component's own face grid):
//   u: (nx+1) x ny x nz at (i h, (j+1/2) h, (k+1/2) h)
//   v: nx x (ny+1) x nz at ((i+1/2) h, j h, (k+1/2) h)
//   w: nx x ny x (nz+1) at ((i+1/2) h, (j+1/2) h, k h)
// Wall-normal faces are zero.  A tangential value outside the domain is a
// ghost 2*U_wall - (mirror value), U_wall = lid_u for u on the wall y = ny*h,
// else 0; a ghost outside two walls resolves y first, then x, then z.
#include "common.h"

#include <cmath>

namespace cfd {

int solve_internal(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts *o,
                   double *x, cfd_solve_info *info, hipStream_t s);
double *scratch_partials(cfd_csr_t A);

struct StepGrid {
    int nx, ny, nz;
    double h, lid;
};

__device__ inline void fdims(const StepGrid &g, int c, int &dx, int &dy, int &dz) {
    dx = g.nx + (c == 0);
    dy = g.ny + (c == 1);
    dz = g.nz + (c == 2);
}

// Value of component c at face index (i, j, k), resolving ghosts.
__device__ inline double fval(const StepGrid &g, int c, const double *__restrict__ f, int i, int j, int k) {
    int dx, dy, dz;
    fdims(g, c, dx, dy, dz);
    double add = 0.0, sign = 1.0;
    if (j < 0 || j >= dy) {
        const double uw = (j >= dy && c == 0) ? g.lid : 0.0;
        j = j < 0 ? 0 : dy - 1;
        add = 2.0 * uw;
        sign = -1.0;
    }
    if (i < 0 || i >= dx) {
        i = i < 0 ? 0 : dx - 1;
        sign = -sign;
    }
    if (k < 0 || k >= dz) {
        k = k < 0 ? 0 : dz - 1;
        sign = -sign;
    }
    const double v = f[(int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * k)];
    return add + sign * v;
}

// Trilinear sample of component c at the physical point (x, y, z).
__device__ inline double sample(const StepGrid &g, int c, const double *__restrict__ f, double x, double y,
                                double z) {
    int dx, dy, dz;
    fdims(g, c, dx, dy, dz);
    const double fx = x / g.h - (c == 0 ? 0.0 : 0.5);
    const double fy = y / g.h - (c == 1 ? 0.0 : 0.5);
    const double fz = z / g.h - (c == 2 ? 0.0 : 0.5);
    const int lox = c == 0 ? 0 : -1, hix = c == 0 ? dx - 2 : dx - 1;
    const int loy = c == 1 ? 0 : -1, hiy = c == 1 ? dy - 2 : dy - 1;
    const int loz = c == 2 ? 0 : -1, hiz = c == 2 ? dz - 2 : dz - 1;
    int i0 = (int)floor(fx), j0 = (int)floor(fy), k0 = (int)floor(fz);
    i0 = i0 < lox ? lox : (i0 > hix ? hix : i0);
    j0 = j0 < loy ? loy : (j0 > hiy ? hiy : j0);
    k0 = k0 < loz ? loz : (k0 > hiz ? hiz : k0);
    double tx = fx - i0, ty = fy - j0, tz = fz - k0;
    tx = tx < 0 ? 0 : (tx > 1 ? 1 : tx);
    ty = ty < 0 ? 0 : (ty > 1 ? 1 : ty);
    tz = tz < 0 ? 0 : (tz > 1 ? 1 : tz);
    double s = 0.0;
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
                const double wgt = (a2 ? tx : 1 - tx) * (b2 ? ty : 1 - ty) * (c2 ? tz : 1 - tz);
                s += wgt * fval(g, c, f, i0 + a2, j0 + b2, k0 + c2);
            }
    return s;
}

__device__ inline bool wall_face(const StepGrid &g, int c, int i, int j, int k) {
    if (c == 0) return i == 0 || i == g.nx;
    if (c == 1) return j == 0 || j == g.ny;
    return k == 0 || k == g.nz;
}

// Map a flat face id over [u | v | w] to (component, i, j, k, local index).
__device__ inline bool face_of(const StepGrid &g, int64_t id, int &c, int &i, int &j, int &k, int64_t &loc) {
    const int64_t nu = (int64_t)(g.nx + 1) * g.ny * g.nz, nv = (int64_t)g.nx * (g.ny + 1) * g.nz,
                  nw = (int64_t)g.nx * g.ny * (g.nz + 1);
    if (id < nu) {
        c = 0;
        loc = id;
    } else if (id < nu + nv) {
        c = 1;
        loc = id - nu;
    } else if (id < nu + nv + nw) {
        c = 2;
        loc = id - nu - nv;
    } else {
        return false;
    }
    int dx, dy, dz;
    fdims(g, c, dx, dy, dz);
    i = (int)(loc % dx);
    j = (int)((loc / dx) % dy);
    k = (int)(loc / ((int64_t)dx * dy));
    return true;
}

struct Fields {
    double *u, *v, *w;
};

__global__ void __launch_bounds__(kBlock) force_kernel(StepGrid g, Fields f, double ax, double ay, double az) {
    const int64_t total = (int64_t)(g.nx + 1) * g.ny * g.nz + (int64_t)g.nx * (g.ny + 1) * g.nz +
                          (int64_t)g.nx * g.ny * (g.nz + 1);
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        int c, i, j, k;
        int64_t loc;
        face_of(g, id, c, i, j, k, loc);
        if (wall_face(g, c, i, j, k)) continue;
        double *dst = c == 0 ? f.u : (c == 1 ? f.v : f.w);
        dst[loc] += c == 0 ? ax : (c == 1 ? ay : az);
    }
}

// Semi-Lagrangian advection: first-order back-trace from the face position,
// trilinear sampling of all three components, departure point clamped to the
// closed domain, then the own component sampled there.
__global__ void __launch_bounds__(kBlock) advect_kernel(StepGrid g, double dt, Fields in, Fields out) {
    const int64_t total = (int64_t)(g.nx + 1) * g.ny * g.nz + (int64_t)g.nx * (g.ny + 1) * g.nz +
                          (int64_t)g.nx * g.ny * (g.nz + 1);
    const double X = g.nx * g.h, Y = g.ny * g.h, Z = g.nz * g.h;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        int c, i, j, k;
        int64_t loc;
        face_of(g, id, c, i, j, k, loc);
        double *dst = c == 0 ? out.u : (c == 1 ? out.v : out.w);
        if (wall_face(g, c, i, j, k)) {
            dst[loc] = 0.0;
            continue;
        }
        const double x = (i + (c == 0 ? 0.0 : 0.5)) * g.h;
        const double y = (j + (c == 1 ? 0.0 : 0.5)) * g.h;
        const double z = (k + (c == 2 ? 0.0 : 0.5)) * g.h;
        const double vx = sample(g, 0, in.u, x, y, z);
        const double vy = sample(g, 1, in.v, x, y, z);
        const double vz = sample(g, 2, in.w, x, y, z);
        double xd = x - dt * vx, yd = y - dt * vy, zd = z - dt * vz;
        xd = xd < 0 ? 0 : (xd > X ? X : xd);
        yd = yd < 0 ? 0 : (yd > Y ? Y : yd);
        zd = zd < 0 ? 0 : (zd > Z ? Z : zd);
        const double *src = c == 0 ? in.u : (c == 1 ? in.v : in.w);
        dst[loc] = sample(g, c, src, xd, yd, zd);
    }
}

// Explicit viscosity: out = in + dt*nu/h^2 * (sum of 6 face neighbours - 6 in).
__global__ void __launch_bounds__(kBlock) diffuse_kernel(StepGrid g, double coef, Fields in, Fields out) {
    const int64_t total = (int64_t)(g.nx + 1) * g.ny * g.nz + (int64_t)g.nx * (g.ny + 1) * g.nz +
                          (int64_t)g.nx * g.ny * (g.nz + 1);
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        int c, i, j, k;
        int64_t loc;
        face_of(g, id, c, i, j, k, loc);
        double *dst = c == 0 ? out.u : (c == 1 ? out.v : out.w);
        if (wall_face(g, c, i, j, k)) {
            dst[loc] = 0.0;
            continue;
        }
        const double *src = c == 0 ? in.u : (c == 1 ? in.v : in.w);
        const double ctr = src[loc];
        const double lap = fval(g, c, src, i - 1, j, k) + fval(g, c, src, i + 1, j, k) +
                           fval(g, c, src, i, j - 1, k) + fval(g, c, src, i, j + 1, k) +
                           fval(g, c, src, i, j, k - 1) + fval(g, c, src, i, j, k + 1) - 6.0 * ctr;
        dst[loc] = ctr + coef * lap;
    }
}

// b = scale * (sum of face-flux differences) per cell.
__global__ void __launch_bounds__(kBlock) divergence_kernel(StepGrid g, Fields f, double scale, double *__restrict__ b) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n; c += (int64_t)gridDim.x * kBlock) {
        const int64_t i = c % g.nx, j = (c / g.nx) % g.ny, k = c / ((int64_t)g.nx * g.ny);
        const int64_t nx = g.nx, ny = g.ny;
        const double du = f.u[(i + 1) + (nx + 1) * (j + ny * k)] - f.u[i + (nx + 1) * (j + ny * k)];
        const double dv = f.v[i + nx * ((j + 1) + (ny + 1) * k)] - f.v[i + nx * (j + (ny + 1) * k)];
        const double dw = f.w[i + nx * (j + ny * (k + 1))] - f.w[i + nx * (j + ny * k)];
        b[c] = (du + dv + dw) * scale;
    }
}

// Interior faces: f -= s * (p_right - p_left), s = dt/(rho h).
__global__ void __launch_bounds__(kBlock) correct_kernel(StepGrid g, Fields f, double s, const double *__restrict__ p) {
    const int64_t total = (int64_t)(g.nx + 1) * g.ny * g.nz + (int64_t)g.nx * (g.ny + 1) * g.nz +
                          (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t nx = g.nx, ny = g.ny;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        int c, i, j, k;
        int64_t loc;
        face_of(g, id, c, i, j, k, loc);
        if (wall_face(g, c, i, j, k)) continue;
        const int64_t hi = i + nx * (j + ny * (int64_t)k);
        const int64_t lo = c == 0 ? hi - 1 : (c == 1 ? hi - nx : hi - nx * ny);
        double *dst = c == 0 ? f.u : (c == 1 ? f.v : f.w);
        dst[loc] -= s * (p[hi] - p[lo]);
    }
}

struct StepWs {
    int64_t nu = 0, nv = 0, nw = 0, n = 0;
    double *ua = nullptr, *va = nullptr, *wa = nullptr, *b = nullptr;
};

void step_ws_free(void *p) {
    StepWs *s = (StepWs *)p;
    if (!s) return;
    double *dd[] = {s->ua, s->va, s->wa, s->b};
    for (double *d : dd) if (d) (void)hipFree(d);
    delete s;
}

static int step_impl(cfd_state *S, double dt, double tol, const cfd_solve_opts *opts, cfd_solve_info *info,
                     hipStream_t st) {
    cfd_csr_t A = S->A;
    const cfd_grid &gr = S->grid;
    if (!A) return fail(CFD_EINVAL, "cfd_step: state has no matrix");
    if (gr.nx != A->nx || gr.ny != A->ny || gr.nz != A->nz)
        return fail(CFD_EINVAL, "cfd_step: matrix was assembled for another grid");
    if (!S->u || !S->v || !S->w || !S->p) return fail(CFD_EINVAL, "cfd_step: null field");
    if (!(dt > 0.0)) return fail(CFD_EINVAL, "cfd_step: dt must be > 0");
    if (!(gr.h > 0.0) || !(S->rho > 0.0)) return fail(CFD_EINVAL, "cfd_step: h and rho must be > 0");
    if (S->nu < 0.0 || dt * S->nu * 6.0 / (gr.h * gr.h) > 1.0)
        return fail(CFD_EINVAL, "cfd_step: explicit viscosity unstable (need dt*nu*6/h^2 <= 1)");
    const int guess = opts ? opts->step_guess : CFD_GUESS_ZERO;
    if (guess != CFD_GUESS_ZERO && guess != CFD_GUESS_PREVIOUS) return fail(CFD_EINVAL, "cfd_step: unknown step_guess");
    if (guess == CFD_GUESS_PREVIOUS && opts->net)
        return fail(CFD_EINVAL, "cfd_step: give either a warm-start network or the previous-pressure guess");
    StepWs *w = (StepWs *)A->step_ws;
    if (!w) {
        w = new StepWs();
        A->step_ws = w;
        w->nu = (int64_t)(gr.nx + 1) * gr.ny * gr.nz;
        w->nv = (int64_t)gr.nx * (gr.ny + 1) * gr.nz;
        w->nw = (int64_t)gr.nx * gr.ny * (gr.nz + 1);
        w->n = (int64_t)gr.nx * gr.ny * gr.nz;
        CFD_HIP(hipMalloc(&w->ua, sizeof(double) * w->nu));
        CFD_HIP(hipMalloc(&w->va, sizeof(double) * w->nv));
        CFD_HIP(hipMalloc(&w->wa, sizeof(double) * w->nw));
        CFD_HIP(hipMalloc(&w->b, sizeof(double) * w->n));
    }
    const StepGrid g{gr.nx, gr.ny, gr.nz, gr.h, S->lid_u};
    const Fields f{S->u, S->v, S->w};
    const Fields fa{w->ua, w->va, w->wa};
    const int64_t faces = w->nu + w->nv + w->nw;
    const unsigned gf = (unsigned)std::min<int64_t>((faces + kBlock - 1) / kBlock, 65536);
    const unsigned gc = (unsigned)std::min<int64_t>((w->n + kBlock - 1) / kBlock, 65536);
    if (S->gx != 0.0 || S->gy != 0.0 || S->gz != 0.0)
        hipLaunchKernelGGL(force_kernel, dim3(gf), dim3(kBlock), 0, st, g, f, dt * S->gx, dt * S->gy, dt * S->gz);
    hipLaunchKernelGGL(advect_kernel, dim3(gf), dim3(kBlock), 0, st, g, dt, f, fa);
    if (S->nu != 0.0) {
        hipLaunchKernelGGL(diffuse_kernel, dim3(gf), dim3(kBlock), 0, st, g, dt * S->nu / (gr.h * gr.h), fa, f);
    } else {
        CFD_HIP(hipMemcpyAsync(S->u, w->ua, sizeof(double) * w->nu, hipMemcpyDeviceToDevice, st));
        CFD_HIP(hipMemcpyAsync(S->v, w->va, sizeof(double) * w->nv, hipMemcpyDeviceToDevice, st));
        CFD_HIP(hipMemcpyAsync(S->w, w->wa, sizeof(double) * w->nw, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(divergence_kernel, dim3(gc), dim3(kBlock), 0, st, g, f, -S->rho * gr.h / dt, w->b);
    CFD_HIP(hipGetLastError());
    int rc = cfd_rhs_prepare(A, w->b, st);
    if (rc != CFD_OK) return rc;
    if (S->rhs) CFD_HIP(hipMemcpyAsync(S->rhs, w->b, sizeof(double) * w->n, hipMemcpyDeviceToDevice, st));
    cfd_solve_info inf{};
    // previous-pressure guess: x0 and x are the same array (the solver reads
    // x0 only in its first kernel, before anything writes x)
    rc = solve_internal(A, w->b, guess == CFD_GUESS_PREVIOUS ? S->p : nullptr, tol, opts, S->p, &inf, st);
    if (info) *info = inf;
    if (rc != CFD_OK) return rc;
    hipLaunchKernelGGL(correct_kernel, dim3(gf), dim3(kBlock), 0, st, g, f, dt / (S->rho * gr.h), (const double *)S->p);
    CFD_HIP(hipGetLastError());
    CFD_HIP(hipStreamSynchronize(st));
    S->t += dt;
    S->step += 1;
    return CFD_OK;
}

}  // namespace cfd

extern "C" int cfd_step(cfd_state *state, double dt, double tol, const cfd_solve_opts *opts, cfd_solve_info *info,
                        void *stream) {
    if (!state) return cfd::fail(CFD_EINVAL, "cfd_step: null state");
    return cfd::step_impl(state, dt, tol, opts, info, (hipStream_t)stream);
}
