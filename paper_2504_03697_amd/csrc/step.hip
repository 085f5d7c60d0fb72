// One fractional time step on the staggered grid (Sec. 3.1 of the paper):
// forces -> semi-Lagrangian advection -> (viscosity) -> pressure correction
// (divergence, Poisson solve, gradient correction).  Every stage is a device
// kernel; advection and viscosity are one kernel (advdiff_kernel) writing
// the step's velocity buffers, which the divergence reads and the
// correction turns into the state's new velocities; the Poisson solve is
// the library's CG (cfd_solve).
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

// Load f at a byte offset.  Every face array of a grid the library
// assembles holds fewer than 2^29 entries (n < 2^31 / 7 cells), so its byte
// offsets fit in 32 bits; the address is then the array's base plus one
// 32-bit offset register.
__device__ inline double ld_at(const double *__restrict__ f, uint32_t off) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(f) + off);
}

// Byte offset of face (i, j, k) in a face grid dx x dy x dz.
__device__ inline uint32_t face_off(int dx, int dy, int i, int j, int k) {
    return 8u * ((uint32_t)i + (uint32_t)dx * ((uint32_t)j + (uint32_t)dy * (uint32_t)k));
}

// Trilinear sample of component C at the point (px, py, pz) in units of h.
// A node outside C's face grid is a ghost of the nearest face: mirrored
// (sign flipped) once per direction it lies outside, plus 2 U_wall when
// outside in y (U_wall = lid_u for u on the lid, else 0).  The rule factors
// by direction (clamped index and flip per direction, the y-add), so the 8
// loads are straight-line code; the interpolation is three rounds of linear
// interpolation, along x, then y, then z.
template <int C>
__device__ inline double sample(const StepGrid &g, const double *__restrict__ f, double px, double py, double pz) {
    int dx, dy, dz;
    fdims(g, C, dx, dy, dz);
    const double fx = px - (C == 0 ? 0.0 : 0.5);
    const double fy = py - (C == 1 ? 0.0 : 0.5);
    const double fz = pz - (C == 2 ? 0.0 : 0.5);
    const int lox = C == 0 ? 0 : -1, hix = C == 0 ? dx - 2 : dx - 1;
    const int loy = C == 1 ? 0 : -1, hiy = C == 1 ? dy - 2 : dy - 1;
    const int loz = C == 2 ? 0 : -1, hiz = C == 2 ? dz - 2 : dz - 1;
    int i0 = (int)floor(fx), j0 = (int)floor(fy), k0 = (int)floor(fz);
    i0 = i0 < lox ? lox : (i0 > hix ? hix : i0);
    j0 = j0 < loy ? loy : (j0 > hiy ? hiy : j0);
    k0 = k0 < loz ? loz : (k0 > hiz ? hiz : k0);
    double tx = fx - i0, ty = fy - j0, tz = fz - k0;
    tx = tx < 0 ? 0 : (tx > 1 ? 1 : tx);
    ty = ty < 0 ? 0 : (ty > 1 ? 1 : ty);
    tz = tz < 0 ? 0 : (tz > 1 ? 1 : tz);
    int ii[2], jj[2], kq[2];
    bool ox[2], oy[2], oz[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int i = i0 + t, j = j0 + t, k = k0 + t;
        ox[t] = i < 0 || i >= dx;
        oy[t] = j < 0 || j >= dy;
        oz[t] = k < 0 || k >= dz;
        ii[t] = i < 0 ? 0 : (i >= dx ? dx - 1 : i);
        jj[t] = j < 0 ? 0 : (j >= dy ? dy - 1 : j);
        kq[t] = k < 0 ? 0 : (k >= dz ? dz - 1 : k);
    }
    const double lid2 = 2.0 * g.lid;
    double vz[2];
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
        double vy[2];
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) {
            double vx[2];
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
                const double v = ld_at(f, face_off(dx, dy, ii[a2], jj[b2], kq[c2]));
                const double m = (ox[a2] != oy[b2]) != oz[c2] ? -v : v;
                vx[a2] = (C == 0 && j0 + b2 >= dy) ? lid2 + m : m;
            }
            vy[b2] = fma(tx, vx[1] - vx[0], vx[0]);
        }
        vz[c2] = fma(ty, vy[1] - vy[0], vy[0]);
    }
    return fma(tz, vz[1] - vz[0], vz[0]);
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

// ---------------------------------------------------------------- advection + viscosity
//
// Semi-Lagrangian advection (first-order back-trace from the face, departure
// point clamped to the closed domain, trilinear sample of the own component
// there) fused with the explicit viscosity step out = a + coef * Lap_h a of
// the advected field a.  One launch covers the interior faces of all three
// components (wall-normal faces stay zero in the output buffers).  A
// workgroup takes a tile of kAdTX x kAdTY faces of one component and marches
// kAdKZ planes along z: each plane of advected values, with a one-face halo
// in x and y (ghosts resolved as fval does for a stored field), goes into a
// ring of three LDS planes, so the 7-point Laplacian reads only LDS and the
// advected field never goes to memory.  The departure samples read the
// velocity through the caches; the tiles of one XCD are contiguous, so the
// halos they share sit in that XCD's L2.
constexpr int kAdThreads = 512;
constexpr int kAdTX = 64, kAdTY = 29;
constexpr int kAdHX = kAdTX + 2, kAdHY = kAdTY + 2;
constexpr int kAdHalo = kAdHX * kAdHY;  // 2046 entries: 4 passes of 512 threads
constexpr int kAdKZ = 16;
constexpr int kAdPasses = (kAdHalo + kAdThreads - 1) / kAdThreads;  // entries per thread and plane
constexpr int kAdPlane = kAdPasses * kAdThreads;                     // LDS slots per plane (2048)
constexpr int kAdBatch = 1;  // entries whose loads are issued together
static_assert(kAdPasses % kAdBatch == 0, "whole batches");

struct AdvTiles {
    int nxt[3], nyt[3];  // tiles across x and y, per component
    int start[4];        // first tile of each component; start[3] = all tiles
    int per_xcd;         // slots per XCD: the grid is 8 * per_xcd workgroups
};

// Velocity component D (!= C) at an interior face (i, j, k) of C: D's faces
// sit half a cell away along C and along D and level with it in the third
// direction, so the trilinear sample there is the mean of the four D-faces
// at offsets {-1, 0} along C and {0, +1} along D (all inside D's face grid
// for an interior face of C).
template <int C, int D>
__device__ inline double face_mean(const StepGrid &g, const double *__restrict__ f, int i, int j, int k) {
    int dx, dy, dz;
    fdims(g, D, dx, dy, dz);
    const int ci = C == 0 ? -1 : 0, cj = C == 1 ? -1 : 0, ck = C == 2 ? -1 : 0;
    const int di = D == 0 ? 1 : 0, dj = D == 1 ? 1 : 0, dk = D == 2 ? 1 : 0;
    const double s0 = ld_at(f, face_off(dx, dy, i + ci, j + cj, k + ck)) + ld_at(f, face_off(dx, dy, i, j, k));
    const double s1 = ld_at(f, face_off(dx, dy, i + ci + di, j + cj + dj, k + ck + dk)) +
                      ld_at(f, face_off(dx, dy, i + di, j + dj, k + dk));
    return 0.25 * (s0 + s1);
}

// A face of C whose advected value a halo entry needs: the departure point
// of that face in units of h (the face's position minus dt/h times the flow
// velocity there, clamped to the closed domain), and how the entry derives
// from the sample of C at it: entry = add + mul * sample.  Entries outside
// C's face grid are ghosts of the nearest face (the sample's rule); wall
// faces have mul = 0 (their advected value is zero) and the velocity is read
// at the nearest interior face so that every load stays inside the arrays.
struct AdvPoint {
    double px, py, pz, add, mul;
};

template <int C>
__device__ inline AdvPoint adv_point(const StepGrid &g, double dth, const Fields &in, int i, int j, int k) {
    int dx, dy, dz;
    fdims(g, C, dx, dy, dz);
    const bool jo = j < 0 || j >= dy, io = i < 0 || i >= dx, ko = k < 0 || k >= dz;
    AdvPoint P;
    P.add = (C == 0 && j >= dy) ? 2.0 * g.lid : 0.0;
    double sign = jo ? -1.0 : 1.0;
    sign = io ? -sign : sign;
    sign = ko ? -sign : sign;
    i = i < 0 ? 0 : (i >= dx ? dx - 1 : i);
    j = j < 0 ? 0 : (j >= dy ? dy - 1 : j);
    k = k < 0 ? 0 : (k >= dz ? dz - 1 : k);
    // along C the interior faces are 1 .. n - 1 (n = cells along C, >= 2 when
    // C has interior faces at all)
    const int nC = C == 0 ? g.nx : (C == 1 ? g.ny : g.nz);
    const int iC = C == 0 ? i : (C == 1 ? j : k);
    P.mul = (iC == 0 || iC == nC) ? 0.0 : sign;
    if (C == 0) i = i < 1 ? 1 : (i > nC - 1 ? nC - 1 : i);
    if (C == 1) j = j < 1 ? 1 : (j > nC - 1 ? nC - 1 : j);
    if (C == 2) k = k < 1 ? 1 : (k > nC - 1 ? nC - 1 : k);
    const double *fc = C == 0 ? in.u : (C == 1 ? in.v : in.w);
    const double own = ld_at(fc, face_off(dx, dy, i, j, k));
    const double vx = C == 0 ? own : face_mean<C, 0>(g, in.u, i, j, k);
    const double vy = C == 1 ? own : face_mean<C, 1>(g, in.v, i, j, k);
    const double vz = C == 2 ? own : face_mean<C, 2>(g, in.w, i, j, k);
    const double px = (i + (C == 0 ? 0.0 : 0.5)) - dth * vx;
    const double py = (j + (C == 1 ? 0.0 : 0.5)) - dth * vy;
    const double pz = (k + (C == 2 ? 0.0 : 0.5)) - dth * vz;
    P.px = px < 0 ? 0 : (px > g.nx ? g.nx : px);
    P.py = py < 0 ? 0 : (py > g.ny ? g.ny : py);
    P.pz = pz < 0 ? 0 : (pz > g.nz ? g.nz : pz);
    return P;
}

// One tile of component C.  Interior faces of C lie in [lo, n) in each
// direction (lo = 1 along C, else 0; n = cells along it); the halo planes
// hold indices x0 - 1 .. x0 + kAdTX and y0 - 1 .. y0 + kAdTY, of which those
// above n are never read.
template <int C>
__device__ void advdiff_tile(const StepGrid &g, double dth, double coef, const Fields &in, double *__restrict__ out,
                             int t, const AdvTiles &T, double (*ring)[kAdPlane]) {
    int dx, dy, dz;
    fdims(g, C, dx, dy, dz);
    const int nxt = T.nxt[C], nyt = T.nyt[C];
    const int xt = t % nxt, yt = (t / nxt) % nyt, zt = t / (nxt * nyt);
    const int x0 = (C == 0) + kAdTX * xt, y0 = (C == 1) + kAdTY * yt;
    const int z0 = (C == 2) + kAdKZ * zt, z1 = min(z0 + kAdKZ, g.nz);
    const int tid = threadIdx.x;
    const double *fc = C == 0 ? in.u : (C == 1 ? in.v : in.w);
    for (int kk = z0 - 1; kk <= z1; ++kk) {
        double *cur = ring[(kk + 3) % 3];
        // this thread's entries in batches of two phases each, so that each
        // phase's loads (the face velocities, then the departure samples) are
        // in flight together
#pragma unroll 1  // unrolled, later batches' loads are hoisted and spill
        for (int q0 = 0; q0 < kAdPasses; q0 += kAdBatch) {
            AdvPoint P[kAdBatch];
#pragma unroll
            for (int q = 0; q < kAdBatch; ++q) {
                const int e = tid + (q0 + q) * kAdThreads;
                P[q] = adv_point<C>(g, dth, in, x0 - 1 + e % kAdHX, y0 - 1 + e / kAdHX, kk);
            }
            // no branch between the samples (one would end the batch): every
            // slot of the padded plane is written, those past the tile's
            // halo or the grid are never read
            double a[kAdBatch];
#pragma unroll
            for (int q = 0; q < kAdBatch; ++q) a[q] = P[q].add + P[q].mul * sample<C>(g, fc, P[q].px, P[q].py, P[q].pz);
#pragma unroll
            for (int q = 0; q < kAdBatch; ++q) cur[tid + (q0 + q) * kAdThreads] = a[q];
        }
        __syncthreads();
        const int ko = kk - 1;  // its planes ko - 1, ko, ko + 1 are in the ring now
        if (ko >= z0) {
            const double *zm = ring[(ko + 2) % 3], *zo = ring[(ko + 3) % 3];
            for (int o = tid; o < kAdTX * kAdTY; o += kAdThreads) {
                const int i = x0 + o % kAdTX, j = y0 + o / kAdTX;
                if (i < g.nx && j < g.ny) {
                    const int e = (o / kAdTX + 1) * kAdHX + o % kAdTX + 1;
                    const double ctr = zo[e];
                    double v = ctr;
                    if (coef != 0.0) {
                        const double lap = zo[e - 1] + zo[e + 1] + zo[e - kAdHX] + zo[e + kAdHX] + zm[e] + cur[e] -
                                           6.0 * ctr;
                        v = ctr + coef * lap;
                    }
                    out[(int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * ko)] = v;
                }
            }
        }
        __syncthreads();
    }
}

// 6 waves per SIMD (3 workgroups per CU, as the LDS ring allows): 80 VGPRs
__global__ void __launch_bounds__(kAdThreads, 6) advdiff_kernel(StepGrid g, double dth, double coef, Fields in,
                                                             Fields out, AdvTiles T) {
    __shared__ double ring[3][kAdPlane];
    // XCD b % 8 takes tiles [(b % 8) * per_xcd, (b % 8 + 1) * per_xcd)
    // slot t holds tile t / 3 of component t % 3: the three components of
    // one region run side by side and share the velocity they read in L2
    // (component by component, each field was fetched three times)
    const int t = (int)(blockIdx.x & 7) * T.per_xcd + (int)(blockIdx.x >> 3);
    const int c = t % 3, s = t / 3;
    if (s >= T.start[c + 1] - T.start[c]) return;
    if (c == 0)
        advdiff_tile<0>(g, dth, coef, in, out.u, s, T, ring);
    else if (c == 1)
        advdiff_tile<1>(g, dth, coef, in, out.v, s, T, ring);
    else
        advdiff_tile<2>(g, dth, coef, in, out.w, s, T, ring);
}

static AdvTiles adv_tiles(const cfd_grid &gr) {
    AdvTiles T{};
    const int n[3] = {gr.nx, gr.ny, gr.nz};
    T.start[0] = 0;
    for (int c = 0; c < 3; ++c) {
        const int ex = n[0] - (c == 0), ey = n[1] - (c == 1), ez = n[2] - (c == 2);  // interior extents
        T.nxt[c] = (ex + kAdTX - 1) / kAdTX;
        T.nyt[c] = (ey + kAdTY - 1) / kAdTY;
        const int nzt = (ez + kAdKZ - 1) / kAdKZ;
        T.start[c + 1] = T.start[c] + T.nxt[c] * T.nyt[c] * nzt;
    }
    const int most = std::max(std::max(T.start[1] - T.start[0], T.start[2] - T.start[1]), T.start[3] - T.start[2]);
    T.per_xcd = (3 * most + 7) / 8;
    return T;
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

// Pressure correction of component C: dst = src - s (p_right - p_left) on
// interior faces, s = dt/(rho h); wall-normal faces 0.
template <int C>
__device__ inline void correct_face(const StepGrid &g, const double *__restrict__ src, double *__restrict__ dst,
                                    double s, const double *__restrict__ p, uint32_t loc) {
    int dx, dy, dz;
    fdims(g, C, dx, dy, dz);
    const uint32_t i = loc % (uint32_t)dx, r = loc / (uint32_t)dx;
    const uint32_t j = r % (uint32_t)dy, k = r / (uint32_t)dy;
    const bool wall = C == 0 ? (i == 0 || i == (uint32_t)g.nx)
                             : (C == 1 ? (j == 0 || j == (uint32_t)g.ny) : (k == 0 || k == (uint32_t)g.nz));
    if (wall) {
        dst[loc] = 0.0;
        return;
    }
    const int64_t nx = g.nx, ny = g.ny;
    const int64_t hi = i + nx * (j + ny * (int64_t)k);
    const int64_t lo = C == 0 ? hi - 1 : (C == 1 ? hi - nx : hi - nx * ny);
    dst[loc] = src[loc] - s * (p[hi] - p[lo]);
}

__global__ void __launch_bounds__(kBlock) correct_kernel(StepGrid g, Fields src, Fields dst, double s,
                                                         const double *__restrict__ p, uint32_t nu, uint32_t nv,
                                                         uint32_t nw) {
    const int64_t total = (int64_t)nu + nv + nw;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < total; id += (int64_t)gridDim.x * kBlock) {
        if (id < nu)
            correct_face<0>(g, src.u, dst.u, s, p, (uint32_t)id);
        else if (id < (int64_t)nu + nv)
            correct_face<1>(g, src.v, dst.v, s, p, (uint32_t)(id - nu));
        else
            correct_face<2>(g, src.w, dst.w, s, p, (uint32_t)(id - nu - nv));
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
        // wall-normal faces of the step's velocity buffers stay zero
        CFD_HIP(hipMemset(w->ua, 0, sizeof(double) * w->nu));
        CFD_HIP(hipMemset(w->va, 0, sizeof(double) * w->nv));
        CFD_HIP(hipMemset(w->wa, 0, sizeof(double) * w->nw));
    }
    const StepGrid g{gr.nx, gr.ny, gr.nz, gr.h, S->lid_u};
    const Fields f{S->u, S->v, S->w};
    const Fields fa{w->ua, w->va, w->wa};
    const int64_t faces = w->nu + w->nv + w->nw;
    const unsigned gf = (unsigned)std::min<int64_t>((faces + kBlock - 1) / kBlock, 65536);
    const unsigned gc = (unsigned)std::min<int64_t>((w->n + kBlock - 1) / kBlock, 65536);
    if (S->gx != 0.0 || S->gy != 0.0 || S->gz != 0.0)
        hipLaunchKernelGGL(force_kernel, dim3(gf), dim3(kBlock), 0, st, g, f, dt * S->gx, dt * S->gy, dt * S->gz);
    // advection and viscosity into the step's buffers; the divergence, and
    // after the solve the correction, read them there
    const AdvTiles T = adv_tiles(gr);
    if (std::max(std::max(w->nu, w->nv), w->nw) >= ((int64_t)1 << 29))
        return fail(CFD_EINVAL, "cfd_step: face arrays need 32-bit byte offsets (under 2^29 faces each)");
    if (T.start[3] > 0)
        hipLaunchKernelGGL(advdiff_kernel, dim3(8 * T.per_xcd), dim3(kAdThreads), 0, st, g, dt / gr.h,
                           dt * S->nu / (gr.h * gr.h), f, fa, T);
    hipLaunchKernelGGL(divergence_kernel, dim3(gc), dim3(kBlock), 0, st, g, fa, -S->rho * gr.h / dt, w->b);
    CFD_HIP(hipGetLastError());
    int rc = cfd_rhs_prepare(A, w->b, st);
    if (rc == CFD_OK && S->rhs)
        CFD_HIP(hipMemcpyAsync(S->rhs, w->b, sizeof(double) * w->n, hipMemcpyDeviceToDevice, st));
    cfd_solve_info inf{};
    // previous-pressure guess: x0 and x are the same array (the solver reads
    // x0 only in its first kernel, before anything writes x)
    if (rc == CFD_OK)
        rc = solve_internal(A, w->b, guess == CFD_GUESS_PREVIOUS ? S->p : nullptr, tol, opts, S->p, &inf, st);
    if (info) *info = inf;
    if (rc != CFD_OK) {
        // the state keeps the velocities before the correction
        const int err = rc;
        CFD_HIP(hipMemcpyAsync(S->u, w->ua, sizeof(double) * w->nu, hipMemcpyDeviceToDevice, st));
        CFD_HIP(hipMemcpyAsync(S->v, w->va, sizeof(double) * w->nv, hipMemcpyDeviceToDevice, st));
        CFD_HIP(hipMemcpyAsync(S->w, w->wa, sizeof(double) * w->nw, hipMemcpyDeviceToDevice, st));
        CFD_HIP(hipStreamSynchronize(st));
        return err;
    }
    hipLaunchKernelGGL(correct_kernel, dim3(gf), dim3(kBlock), 0, st, g, fa, f, dt / (S->rho * gr.h),
                       (const double *)S->p, (uint32_t)w->nu, (uint32_t)w->nv, (uint32_t)w->nw);
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
