/*
 * cfd_oracle.c -- plain, slow, obviously correct FP64 CPU reference of the
 * pressure-Poisson hot path of the lid-driven-cavity proxy app
 * (arXiv 2504.03697, "cfdSCOPE").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header or
 * constant with the HIP path.
 *
 * What it follows:
 *  - Sec. 3 (Eqs. 1-2): inviscid momentum + incompressibility; we add an
 *    optional viscosity nu (the paper's future-work item; nu=0 recovers it).
 *  - Sec. 3.1 "Computational Approach": staggered (MAC) grid, fractional
 *    step: forces -> semi-Lagrangian advection -> pressure correction
 *    (divergence, Poisson solve, gradient correction); the Poisson matrix is
 *    stored as CSR and solved by conjugate gradients.
 *  - Sec. 3.3 "Algorithmic changes": the matrix is symmetric and its
 *    sparsity pattern does not change between steps.
 *
 * Readings where the paper is silent:
 *  - Matrix: integer 7-point stencil A = -h^2 * Laplacian with homogeneous
 *    Neumann walls: diag = number of in-domain face neighbours, -1 per
 *    neighbour.  The h^2 scale lives in the right-hand side.
 *  - Pin: row `pin` becomes the unit row e_pin and the entries A[j,pin] of its
 *    neighbours are dropped (their diagonal is unchanged); b[pin] = 0.
 *    pin < 0 keeps the singular Neumann matrix.
 *  - CG: Hestenes-Stiefel, no preconditioner; stop when ||r_k|| <= tol*||b||
 *    on the recursive residual, confirm on the true residual b - A x and
 *    restart from it if the confirmation fails; b = 0 gives x = 0.
 *  - Lid: the wall y = max moves in +x with speed lid_u, imposed through
 *    ghost values (2*U_wall - inside); all other walls are no-slip.
 *
 * Every dot product is summed in a fixed order (ORA_CHUNKS contiguous
 * chunks summed serially, then the chunk sums in index order), so results
 * do not depend on the OpenMP thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads the parallel loops use (reported beside the timings). */
int ora_threads(void) { return omp_get_max_threads(); }

/* Set that thread count (timings only: every sum below runs in a fixed
 * order that does not depend on it, so the results do not change). */
void ora_set_threads(int t) {
    if (t > 0) omp_set_num_threads(t);
}

#define ORA_CHUNKS 256

/* ------------------------------------------------------------------ */
/* Matrix assembly (Sec. 3.1: Poisson system in CSR)                   */
/* ------------------------------------------------------------------ */

static int64_t cell(int i, int j, int k, int nx, int ny) {
    return (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * (int64_t)k);
}

/* Number of stored entries of the (optionally pinned) 7-point matrix,
 * counted by walking the rows exactly as ora_assemble does. */
int64_t ora_nnz(int nx, int ny, int nz, int64_t pin) {
    int64_t cnt = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t row = cell(i, j, k, nx, ny);
                if (row == pin) { cnt += 1; continue; }
                int64_t nb[6]; int m = 0;
                if (k > 0) nb[m++] = cell(i, j, k - 1, nx, ny);
                if (j > 0) nb[m++] = cell(i, j - 1, k, nx, ny);
                if (i > 0) nb[m++] = cell(i - 1, j, k, nx, ny);
                if (i < nx - 1) nb[m++] = cell(i + 1, j, k, nx, ny);
                if (j < ny - 1) nb[m++] = cell(i, j + 1, k, nx, ny);
                if (k < nz - 1) nb[m++] = cell(i, j, k + 1, nx, ny);
                cnt += 1;
                for (int q = 0; q < m; ++q) if (nb[q] != pin) cnt += 1;
            }
    return cnt;
}

/* Build the CSR arrays (caller allocates n+1 / nnz entries).  Columns are
 * ascending within a row: -z, -y, -x, diagonal, +x, +y, +z. */
void ora_assemble(int nx, int ny, int nz, int64_t pin,
                  int32_t *row_ptr, int32_t *col, double *val) {
    int64_t cnt = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t row = cell(i, j, k, nx, ny);
                row_ptr[row] = (int32_t)cnt;
                if (row == pin) { col[cnt] = (int32_t)row; val[cnt] = 1.0; ++cnt; continue; }
                int64_t lo[3]; int nlo = 0;
                int64_t hi[3]; int nhi = 0;
                if (k > 0) lo[nlo++] = cell(i, j, k - 1, nx, ny);
                if (j > 0) lo[nlo++] = cell(i, j - 1, k, nx, ny);
                if (i > 0) lo[nlo++] = cell(i - 1, j, k, nx, ny);
                if (i < nx - 1) hi[nhi++] = cell(i + 1, j, k, nx, ny);
                if (j < ny - 1) hi[nhi++] = cell(i, j + 1, k, nx, ny);
                if (k < nz - 1) hi[nhi++] = cell(i, j, k + 1, nx, ny);
                int degree = nlo + nhi;
                for (int q = 0; q < nlo; ++q)
                    if (lo[q] != pin) { col[cnt] = (int32_t)lo[q]; val[cnt] = -1.0; ++cnt; }
                col[cnt] = (int32_t)row; val[cnt] = (double)degree; ++cnt;
                for (int q = 0; q < nhi; ++q)
                    if (hi[q] != pin) { col[cnt] = (int32_t)hi[q]; val[cnt] = -1.0; ++cnt; }
            }
    row_ptr[(int64_t)nx * ny * nz] = (int32_t)cnt;
}

/* ------------------------------------------------------------------ */
/* Basic linear algebra (Table 1: spmv, dot, vector updates)           */
/* ------------------------------------------------------------------ */

/* y = A x */
void ora_spmv(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += val[e] * x[col[e]];
        y[i] = s;
    }
}

/* x^T y in a fixed summation order (independent of the thread count). */
double ora_dot(int64_t n, const double *x, const double *y) {
    double part[ORA_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < ORA_CHUNKS; ++c) {
        int64_t lo = n * c / ORA_CHUNKS, hi = n * (c + 1) / ORA_CHUNKS;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += x[i] * y[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < ORA_CHUNKS; ++c) s += part[c];
    return s;
}

/* y += a x */
static void axpy(int64_t n, double a, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] += a * x[i];
}

/* r = b - A x */
static void residual(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                     const double *b, const double *x, double *r) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += val[e] * x[col[e]];
        r[i] = b[i] - s;
    }
}

/* Right-hand-side consistency: subtract the mean, then b[pin] = 0. */
void ora_rhs_prepare(int64_t n, double *b, int64_t pin) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += b[i];
    double mean = s / (double)n;
    for (int64_t i = 0; i < n; ++i) b[i] -= mean;
    if (pin >= 0 && pin < n) b[pin] = 0.0;
}

/* ------------------------------------------------------------------ */
/* Conjugate gradients (Sec. 3.1), unpreconditioned                     */
/* ------------------------------------------------------------------ */

enum { ORA_OK = 0, ORA_ENOCONV = -4, ORA_EBREAKDOWN = -5, ORA_ENONFINITE = -6 };

/*
 * Solve A x = b.  x0 may be NULL (zero guess).  Returns a status code;
 * *iters = number of products q = A p, *relres = ||b - A x|| / ||b|| of
 * the returned x (0 when b = 0).
 */
int ora_cg(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
           const double *b, const double *x0, double tol, int max_iters,
           double *x, int *iters, double *relres) {
    double *r = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    int status = ORA_OK, k = 0;
    double bnorm = sqrt(ora_dot(n, b, b));
    if (x0) memcpy(x, x0, sizeof(double) * n); else memset(x, 0, sizeof(double) * n);
    *iters = 0;
    if (!isfinite(bnorm)) { status = ORA_ENONFINITE; *relres = NAN; goto out; }
    if (bnorm == 0.0) { memset(x, 0, sizeof(double) * n); *relres = 0.0; goto out; }

    residual(n, rp, col, val, b, x, r);
    double rho = ora_dot(n, r, r);
    if (!isfinite(rho)) { status = ORA_ENONFINITE; goto fin; }
    if (sqrt(rho) <= tol * bnorm) goto fin;
    memcpy(p, r, sizeof(double) * n);
    for (;;) {
        if (k >= max_iters) { status = ORA_ENOCONV; break; }
        ora_spmv(n, rp, col, val, p, q);
        double pq = ora_dot(n, p, q);
        ++k;
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORA_EBREAKDOWN; break; }
        double alpha = rho / pq;
        axpy(n, alpha, p, x);
        axpy(n, -alpha, q, r);
        double rho_new = ora_dot(n, r, r);
        if (!isfinite(rho_new)) { status = ORA_ENONFINITE; break; }
        if (sqrt(rho_new) <= tol * bnorm) {
            /* confirm on the true residual; restart from it if it fails */
            residual(n, rp, col, val, b, x, r);
            rho_new = ora_dot(n, r, r);
            if (sqrt(rho_new) <= tol * bnorm) break;
            memcpy(p, r, sizeof(double) * n);
            rho = rho_new;
            continue;
        }
        double beta = rho_new / rho;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
fin:
    residual(n, rp, col, val, b, x, r);
    *relres = sqrt(ora_dot(n, r, r)) / bnorm;
out:
    *iters = k;
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Preconditioned CG (Sec. 3.1: PCG with a DIC or a Jacobi              */
/* preconditioner; Sec. 3.3: DIC's recurrences run in a fixed order)    */
/* ------------------------------------------------------------------ */

/*
 * Elimination order of the cells.  redblack = 0: natural (cell index);
 * redblack = 1: the cells with i+j+k even ("red") first, then the others,
 * each colour in cell-index order.  ord[t] is the cell at position t and
 * pos[m] the position of cell m.
 */
void ora_order(int nx, int ny, int nz, int redblack, int64_t *ord, int64_t *pos) {
    int64_t n = (int64_t)nx * ny * nz, t = 0;
    for (int pass = 0; pass < (redblack ? 2 : 1); ++pass)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    if (redblack && ((i + j + k) & 1) != pass) continue;
                    int64_t m = cell(i, j, k, nx, ny);
                    ord[t] = m;
                    pos[m] = t;
                    ++t;
                }
    (void)n;
}

/*
 * Diagonal-based incomplete Cholesky: M = (D + L) D^{-1} (D + U), where L
 * and U hold the entries a_mj of A whose cell j comes before / after m in
 * the order, and D is chosen so that diag(M) = diag(A):
 *   d_m = a_mm - sum_{j before m} a_mj^2 / d_j,
 * evaluated along the order.  Returns 0, or -1 if a pivot is not positive.
 */
int ora_dic_factor(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                   const int64_t *ord, const int64_t *pos, double *d) {
    for (int64_t t = 0; t < n; ++t) {
        int64_t m = ord[t];
        double dm = 0.0, s = 0.0;
        for (int64_t e = rp[m]; e < rp[m + 1]; ++e) {
            int64_t j = col[e];
            if (j == m) dm += val[e];
            else if (pos[j] < t) s += val[e] * val[e] / d[j];
        }
        d[m] = dm - s;
        if (!(d[m] > 0.0)) return -1;
    }
    return 0;
}

/* z = M^{-1} r: forward substitution (D + L) w = r along the order, then
 * backward substitution (D + U) z = D w against it (work: n doubles). */
void ora_dic_apply(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                   const int64_t *ord, const int64_t *pos, const double *d,
                   const double *r, double *z, double *work) {
    double *w = work;
    for (int64_t t = 0; t < n; ++t) {
        int64_t m = ord[t];
        double s = r[m];
        for (int64_t e = rp[m]; e < rp[m + 1]; ++e)
            if (pos[col[e]] < t) s -= val[e] * w[col[e]];
        w[m] = s / d[m];
    }
    for (int64_t t = n - 1; t >= 0; --t) {
        int64_t m = ord[t];
        double s = 0.0;
        for (int64_t e = rp[m]; e < rp[m + 1]; ++e)
            if (pos[col[e]] > t) s += val[e] * z[col[e]];
        z[m] = w[m] - s / d[m];
    }
}

enum { ORA_PRECOND_NONE = 0, ORA_PRECOND_JACOBI = 1, ORA_PRECOND_DIC = 2 };

/* z = M^{-1} r for the chosen preconditioner (Jacobi: M = diag(A)). */
static void precond_apply(int kind, int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                          const int64_t *ord, const int64_t *pos, const double *d,
                          const double *r, double *z, double *work) {
    if (kind == ORA_PRECOND_DIC) {
        ora_dic_apply(n, rp, col, val, ord, pos, d, r, z, work);
    } else if (kind == ORA_PRECOND_JACOBI) {
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / d[i];
    } else {
        memcpy(z, r, sizeof(double) * n);
    }
}

/*
 * Preconditioned CG on A x = b, same contract as ora_cg (stop on the
 * recursive ||r|| <= tol*||b||, confirm on the true residual, restart from
 * it if the confirmation fails).  kind: ORA_PRECOND_*; ord/pos: elimination
 * order for DIC (ignored otherwise).  Returns ORA_EBREAKDOWN also when the
 * DIC factorisation meets a non-positive pivot or r^T z <= 0.
 */
int ora_pcg(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
            const double *b, const double *x0, double tol, int max_iters, int kind,
            const int64_t *ord, const int64_t *pos, double *x, int *iters, double *relres) {
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    double *work = (double *)malloc(sizeof(double) * n);
    int status = ORA_OK, k = 0;
    double bnorm = sqrt(ora_dot(n, b, b));
    if (x0) memcpy(x, x0, sizeof(double) * n); else memset(x, 0, sizeof(double) * n);
    *iters = 0;
    if (!isfinite(bnorm)) { status = ORA_ENONFINITE; *relres = NAN; goto out; }
    if (bnorm == 0.0) { memset(x, 0, sizeof(double) * n); *relres = 0.0; goto out; }
    if (kind == ORA_PRECOND_DIC) {
        if (ora_dic_factor(n, rp, col, val, ord, pos, d) != 0) { status = ORA_EBREAKDOWN; goto fin; }
    } else if (kind == ORA_PRECOND_JACOBI) {
        for (int64_t i = 0; i < n; ++i) {
            d[i] = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
                if (col[e] == i) d[i] += val[e];
            if (!(d[i] > 0.0)) { status = ORA_EBREAKDOWN; goto fin; }
        }
    }

    residual(n, rp, col, val, b, x, r);
    if (!isfinite(ora_dot(n, r, r))) { status = ORA_ENONFINITE; goto fin; }
    if (sqrt(ora_dot(n, r, r)) <= tol * bnorm) goto fin;
    precond_apply(kind, n, rp, col, val, ord, pos, d, r, z, work);
    double rho = ora_dot(n, r, z);
    memcpy(p, z, sizeof(double) * n);
    for (;;) {
        if (k >= max_iters) { status = ORA_ENOCONV; break; }
        if (!(rho > 0.0)) { status = ORA_EBREAKDOWN; break; }
        ora_spmv(n, rp, col, val, p, q);
        double pq = ora_dot(n, p, q);
        ++k;
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORA_EBREAKDOWN; break; }
        double alpha = rho / pq;
        axpy(n, alpha, p, x);
        axpy(n, -alpha, q, r);
        double rr = ora_dot(n, r, r);
        if (!isfinite(rr)) { status = ORA_ENONFINITE; break; }
        if (sqrt(rr) <= tol * bnorm) {
            residual(n, rp, col, val, b, x, r);
            if (sqrt(ora_dot(n, r, r)) <= tol * bnorm) break;
            precond_apply(kind, n, rp, col, val, ord, pos, d, r, z, work);
            rho = ora_dot(n, r, z);
            memcpy(p, z, sizeof(double) * n);
            continue;
        }
        precond_apply(kind, n, rp, col, val, ord, pos, d, r, z, work);
        double rho_new = ora_dot(n, r, z);
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
fin:
    residual(n, rp, col, val, b, x, r);
    *relres = sqrt(ora_dot(n, r, r)) / bnorm;
out:
    *iters = k;
    free(r); free(z); free(p); free(q); free(d); free(work);
    return status;
}

/* ------------------------------------------------------------------ */
/* One fractional time step on the MAC grid (Sec. 3.1)                  */
/* ------------------------------------------------------------------ */
/*
 * Layout (x fastest):
 *   u (x-faces): (nx+1) * ny * nz, u[i + (nx+1)*(j + ny*k)], at (i h, (j+.5)h, (k+.5)h)
 *   v (y-faces): nx * (ny+1) * nz, v[i + nx*(j + (ny+1)*k)], at ((i+.5)h, j h, (k+.5)h)
 *   w (z-faces): nx * ny * (nz+1), w[i + nx*(j + ny*k)],     at ((i+.5)h, (j+.5)h, k h)
 *   p (cells):   nx * ny * nz
 * Wall-normal faces are zero.  Tangential values outside the domain are
 * ghosts: g = 2*U_wall - inside, where U_wall = lid_u for u on the wall
 * y = ny*h and 0 otherwise.  A ghost outside two walls resolves the y wall
 * first, then x, then z.
 */

typedef struct {
    int nx, ny, nz;
    double h, lid;
} ogrid;

/* component c in {0,1,2}; face-grid dims */
static void fdims(const ogrid *g, int c, int *dx, int *dy, int *dz) {
    *dx = g->nx + (c == 0); *dy = g->ny + (c == 1); *dz = g->nz + (c == 2);
}

/* value of component c at integer face index (i,j,k), possibly a ghost */
static double fval(const ogrid *g, int c, const double *f, int i, int j, int k) {
    int dx, dy, dz; fdims(g, c, &dx, &dy, &dz);
    if (j < 0 || j >= dy) {            /* only for c != 1: tangential in y */
        int jm = j < 0 ? 0 : dy - 1;
        double uw = (j >= dy && c == 0) ? g->lid : 0.0;
        return 2.0 * uw - fval(g, c, f, i, jm, k);
    }
    if (i < 0 || i >= dx) {            /* only for c != 0 */
        int im = i < 0 ? 0 : dx - 1;
        return -fval(g, c, f, im, j, k);
    }
    if (k < 0 || k >= dz) {            /* only for c != 2 */
        int km = k < 0 ? 0 : dz - 1;
        return -fval(g, c, f, i, j, km);
    }
    return f[(int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * k)];
}

/* trilinear sample of component c at physical point (x,y,z) */
static double sample(const ogrid *g, int c, const double *f, double x, double y, double z) {
    int dx, dy, dz; fdims(g, c, &dx, &dy, &dz);
    double fx = x / g->h - (c == 0 ? 0.0 : 0.5);
    double fy = y / g->h - (c == 1 ? 0.0 : 0.5);
    double fz = z / g->h - (c == 2 ? 0.0 : 0.5);
    /* lowest corner index: staggered direction clamps to [0, d-2], the
     * cell-centred directions to [-1, d-1] (ghost layers on both sides) */
    int lox = c == 0 ? 0 : -1, hix = c == 0 ? dx - 2 : dx - 1;
    int loy = c == 1 ? 0 : -1, hiy = c == 1 ? dy - 2 : dy - 1;
    int loz = c == 2 ? 0 : -1, hiz = c == 2 ? dz - 2 : dz - 1;
    int i0 = (int)floor(fx), j0 = (int)floor(fy), k0 = (int)floor(fz);
    if (i0 < lox) i0 = lox; if (i0 > hix) i0 = hix;
    if (j0 < loy) j0 = loy; if (j0 > hiy) j0 = hiy;
    if (k0 < loz) k0 = loz; if (k0 > hiz) k0 = hiz;
    double tx = fx - i0, ty = fy - j0, tz = fz - k0;
    if (tx < 0) tx = 0; if (tx > 1) tx = 1;
    if (ty < 0) ty = 0; if (ty > 1) ty = 1;
    if (tz < 0) tz = 0; if (tz > 1) tz = 1;
    double s = 0.0;
    for (int c2 = 0; c2 < 2; ++c2)
        for (int b2 = 0; b2 < 2; ++b2)
            for (int a2 = 0; a2 < 2; ++a2) {
                double wgt = (a2 ? tx : 1 - tx) * (b2 ? ty : 1 - ty) * (c2 ? tz : 1 - tz);
                s += wgt * fval(g, c, f, i0 + a2, j0 + b2, k0 + c2);
            }
    return s;
}

/* physical position of face (i,j,k) of component c */
static void fpos(const ogrid *g, int c, int i, int j, int k, double *x, double *y, double *z) {
    *x = (i + (c == 0 ? 0.0 : 0.5)) * g->h;
    *y = (j + (c == 1 ? 0.0 : 0.5)) * g->h;
    *z = (k + (c == 2 ? 0.0 : 0.5)) * g->h;
}

static int is_wall_face(const ogrid *g, int c, int i, int j, int k) {
    if (c == 0) return i == 0 || i == g->nx;
    if (c == 1) return j == 0 || j == g->ny;
    return k == 0 || k == g->nz;
}

/* Semi-Lagrangian advection (first-order back-trace, trilinear sampling,
 * departure point clamped to the closed domain). */
void ora_advect(int nx, int ny, int nz, double h, double lid, double dt,
                const double *u, const double *v, const double *w,
                double *un, double *vn, double *wn) {
    ogrid g = {nx, ny, nz, h, lid};
    const double *f[3] = {u, v, w};
    double *out[3] = {un, vn, wn};
    double X = nx * h, Y = ny * h, Z = nz * h;
    for (int c = 0; c < 3; ++c) {
        int dx, dy, dz; fdims(&g, c, &dx, &dy, &dz);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < dz; ++k)
            for (int j = 0; j < dy; ++j)
                for (int i = 0; i < dx; ++i) {
                    int64_t id = (int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * k);
                    if (is_wall_face(&g, c, i, j, k)) { out[c][id] = 0.0; continue; }
                    double x, y, z; fpos(&g, c, i, j, k, &x, &y, &z);
                    double vx = sample(&g, 0, u, x, y, z);
                    double vy = sample(&g, 1, v, x, y, z);
                    double vz = sample(&g, 2, w, x, y, z);
                    double xd = x - dt * vx, yd = y - dt * vy, zd = z - dt * vz;
                    if (xd < 0) xd = 0; if (xd > X) xd = X;
                    if (yd < 0) yd = 0; if (yd > Y) yd = Y;
                    if (zd < 0) zd = 0; if (zd > Z) zd = Z;
                    out[c][id] = sample(&g, c, f[c], xd, yd, zd);
                }
    }
}

/* Explicit viscous update f_out = f + dt*nu*Lap_h f on interior faces
 * (7-point Laplacian over face neighbours, ghosts at tangential walls). */
void ora_diffuse(int nx, int ny, int nz, double h, double lid, double dt, double nu,
                 const double *u, const double *v, const double *w,
                 double *un, double *vn, double *wn) {
    ogrid g = {nx, ny, nz, h, lid};
    const double *f[3] = {u, v, w};
    double *out[3] = {un, vn, wn};
    double coef = dt * nu / (h * h);
    for (int c = 0; c < 3; ++c) {
        int dx, dy, dz; fdims(&g, c, &dx, &dy, &dz);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < dz; ++k)
            for (int j = 0; j < dy; ++j)
                for (int i = 0; i < dx; ++i) {
                    int64_t id = (int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * k);
                    if (is_wall_face(&g, c, i, j, k)) { out[c][id] = 0.0; continue; }
                    double ctr = f[c][id];
                    double lap = fval(&g, c, f[c], i - 1, j, k) + fval(&g, c, f[c], i + 1, j, k)
                               + fval(&g, c, f[c], i, j - 1, k) + fval(&g, c, f[c], i, j + 1, k)
                               + fval(&g, c, f[c], i, j, k - 1) + fval(&g, c, f[c], i, j, k + 1)
                               - 6.0 * ctr;
                    out[c][id] = ctr + coef * lap;
                }
    }
}

/* D = sum of face-flux differences per cell (no 1/h factor). */
void ora_divergence(int nx, int ny, int nz, const double *u, const double *v, const double *w,
                    double *D) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t c = (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * k);
                double du = u[(int64_t)(i + 1) + (int64_t)(nx + 1) * (j + (int64_t)ny * k)]
                          - u[(int64_t)i + (int64_t)(nx + 1) * (j + (int64_t)ny * k)];
                double dv = v[(int64_t)i + (int64_t)nx * ((j + 1) + (int64_t)(ny + 1) * k)]
                          - v[(int64_t)i + (int64_t)nx * (j + (int64_t)(ny + 1) * k)];
                double dw = w[(int64_t)i + (int64_t)nx * (j + (int64_t)ny * (k + 1))]
                          - w[(int64_t)i + (int64_t)nx * (j + (int64_t)ny * k)];
                D[c] = du + dv + dw;
            }
}

/* Interior faces: f -= (dt/(rho h)) * (p_right - p_left). */
void ora_correct(int nx, int ny, int nz, double h, double rho, double dt, const double *p,
                 double *u, double *v, double *w) {
    double s = dt / (rho * h);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            for (int i = 1; i < nx; ++i)
                u[(int64_t)i + (int64_t)(nx + 1) * (j + (int64_t)ny * k)] -=
                    s * (p[cell(i, j, k, nx, ny)] - p[cell(i - 1, j, k, nx, ny)]);
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                v[(int64_t)i + (int64_t)nx * (j + (int64_t)(ny + 1) * k)] -=
                    s * (p[cell(i, j, k, nx, ny)] - p[cell(i, j - 1, k, nx, ny)]);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                w[(int64_t)i + (int64_t)nx * (j + (int64_t)ny * k)] -=
                    s * (p[cell(i, j, k, nx, ny)] - p[cell(i, j, k - 1, nx, ny)]);
}

/*
 * One full time step, in the paper's order: forces (g*dt on interior
 * faces) -> advection -> viscosity (reading; nu=0 skips it) -> pressure
 * correction.  The Poisson right-hand side is b = -(rho h/dt) D, made
 * consistent (mean removed, b[pin] = 0) and solved from a zero guess.
 * u, v, w, p are updated in place.  Returns the CG status.
 */
int ora_step(int nx, int ny, int nz, double h, double lid, double nu, double rho,
             double gx, double gy, double gz, double dt,
             const int32_t *rp, const int32_t *col, const double *val, int64_t pin,
             double tol, int max_iters,
             double *u, double *v, double *w, double *p, int *iters, double *relres) {
    int64_t nu_ = (int64_t)(nx + 1) * ny * nz, nv_ = (int64_t)nx * (ny + 1) * nz,
            nw_ = (int64_t)nx * ny * (nz + 1), n = (int64_t)nx * ny * nz;
    double *ua = (double *)malloc(sizeof(double) * nu_);
    double *va = (double *)malloc(sizeof(double) * nv_);
    double *wa = (double *)malloc(sizeof(double) * nw_);
    double *b = (double *)malloc(sizeof(double) * n);
    ogrid g = {nx, ny, nz, h, lid};
    /* forces */
    if (gx != 0.0 || gy != 0.0 || gz != 0.0) {
        double gg[3] = {gx, gy, gz};
        double *f[3] = {u, v, w};
        for (int c = 0; c < 3; ++c) {
            int dx, dy, dz; fdims(&g, c, &dx, &dy, &dz);
            for (int k = 0; k < dz; ++k)
                for (int j = 0; j < dy; ++j)
                    for (int i = 0; i < dx; ++i)
                        if (!is_wall_face(&g, c, i, j, k))
                            f[c][(int64_t)i + (int64_t)dx * ((int64_t)j + (int64_t)dy * k)] += dt * gg[c];
        }
    }
    ora_advect(nx, ny, nz, h, lid, dt, u, v, w, ua, va, wa);
    if (nu != 0.0) {
        ora_diffuse(nx, ny, nz, h, lid, dt, nu, ua, va, wa, u, v, w);
    } else {
        memcpy(u, ua, sizeof(double) * nu_);
        memcpy(v, va, sizeof(double) * nv_);
        memcpy(w, wa, sizeof(double) * nw_);
    }
    ora_divergence(nx, ny, nz, u, v, w, b);
    double scale = -rho * h / dt;
    for (int64_t i = 0; i < n; ++i) b[i] *= scale;
    ora_rhs_prepare(n, b, pin);
    int st = ora_cg(n, rp, col, val, b, NULL, tol, max_iters, p, iters, relres);
    ora_correct(nx, ny, nz, h, rho, dt, p, u, v, w);
    free(ua); free(va); free(wa); free(b);
    return st;
}

/* ------------------------------------------------------------------ */
/* Warm-start network: 3-D convolution with replicate padding           */
/* ------------------------------------------------------------------ */
/*
 * Activations: X[v*cin + ci], v = voxel index (x fastest).
 * Weights:     W[(t*cin + ci)*cout + co], t = (dz+1)*9 + (dy+1)*3 + (dx+1).
 * Output:      Y[v*cout + co] = sum_t sum_ci X[clamp(v + d_t), ci] * W[t,ci,co].
 * Replicate padding: an out-of-range neighbour index is clamped to the
 * nearest in-range one.
 */
static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

void ora_conv3d_fwd(int nx, int ny, int nz, int cin, int cout,
                    const double *X, const double *W, double *Y) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t v = cell(i, j, k, nx, ny);
                for (int co = 0; co < cout; ++co) {
                    double s = 0.0;
                    for (int t = 0; t < 27; ++t) {
                        int ddx = t % 3 - 1, ddy = (t / 3) % 3 - 1, ddz = t / 9 - 1;
                        int64_t src = cell(clampi(i + ddx, 0, nx - 1), clampi(j + ddy, 0, ny - 1),
                                           clampi(k + ddz, 0, nz - 1), nx, ny);
                        for (int ci = 0; ci < cin; ++ci)
                            s += X[src * cin + ci] * W[((int64_t)t * cin + ci) * cout + co];
                    }
                    Y[v * cout + co] = s;
                }
            }
}

/* Adjoint of ora_conv3d_fwd w.r.t. X: scatter dY through the clamped taps. */
void ora_conv3d_bwd_data(int nx, int ny, int nz, int cin, int cout,
                         const double *dY, const double *W, double *dX) {
    int64_t n = (int64_t)nx * ny * nz;
    memset(dX, 0, sizeof(double) * n * cin);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t v = cell(i, j, k, nx, ny);
                for (int t = 0; t < 27; ++t) {
                    int ddx = t % 3 - 1, ddy = (t / 3) % 3 - 1, ddz = t / 9 - 1;
                    int64_t src = cell(clampi(i + ddx, 0, nx - 1), clampi(j + ddy, 0, ny - 1),
                                       clampi(k + ddz, 0, nz - 1), nx, ny);
                    for (int ci = 0; ci < cin; ++ci) {
                        double s = 0.0;
                        for (int co = 0; co < cout; ++co)
                            s += dY[v * cout + co] * W[((int64_t)t * cin + ci) * cout + co];
                        dX[src * cin + ci] += s;
                    }
                }
            }
}

/* Gradient w.r.t. W: dW[t,ci,co] = sum_v X[clamp(v+d_t),ci] * dY[v,co]. */
void ora_conv3d_bwd_weight(int nx, int ny, int nz, int cin, int cout,
                           const double *X, const double *dY, double *dW) {
#pragma omp parallel for schedule(static)
    for (int t = 0; t < 27; ++t) {
        int ddx = t % 3 - 1, ddy = (t / 3) % 3 - 1, ddz = t / 9 - 1;
        for (int ci = 0; ci < cin; ++ci)
            for (int co = 0; co < cout; ++co) {
                double s = 0.0;
                for (int k = 0; k < nz; ++k)
                    for (int j = 0; j < ny; ++j)
                        for (int i = 0; i < nx; ++i) {
                            int64_t v = cell(i, j, k, nx, ny);
                            int64_t src = cell(clampi(i + ddx, 0, nx - 1), clampi(j + ddy, 0, ny - 1),
                                               clampi(k + ddz, 0, nz - 1), nx, ny);
                            s += X[src * cin + ci] * dY[v * cout + co];
                        }
                dW[((int64_t)t * cin + ci) * cout + co] = s;
            }
    }
}

/* Adam update (Kingma & Ba 2015, Algorithm 1), step t >= 1, in place. */
void ora_adam(int64_t count, double *theta, double *m, double *v, const double *g,
              double lr, double beta1, double beta2, double eps, int t) {
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t i = 0; i < count; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
