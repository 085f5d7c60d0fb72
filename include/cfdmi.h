/*
 * cfdmi.h -- C ABI of the MI355X pressure-Poisson library.
 *
 * The library implements the hot path of the lid-driven-cavity proxy app of
 * arXiv 2504.03697 ("cfdSCOPE"): the pressure-Poisson solve that each
 * fractional time step performs (Sec. 3.1: the Poisson equation is stored
 * as a CSR matrix and solved by conjugate gradients; Table 1: spmv, dot and
 * the vector updates dominate the solver's time), plus the time step that
 * produces its right-hand side and a learned warm start for the solve.
 *
 * Conventions for every function below:
 *  - Return value: CFD_OK (0) on success, a negative CFD_E* code on failure;
 *    cfd_last_error() then returns a message (thread-local, valid until the
 *    next call on that thread).
 *  - Pointers named as device pointers must point to device memory of the
 *    current HIP device (for example torch tensors' data_ptr()); the caller
 *    owns them.  Opaque handles (cfd_csr_t, cfd_net_t) own their device
 *    workspaces and free them in *_destroy.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All device
 *    work is enqueued on it.  Functions that return host-side results
 *    (cfd_solve, cfd_step, cfd_net_train_step) synchronise that stream before
 *    returning; the others return without synchronising.
 *  - Grids are nx*ny*nz cubic cells of side h.  Cell arrays are indexed
 *    idx = i + nx*(j + ny*k) (x fastest).  Face velocities live on the
 *    staggered grid: u[(nx+1)*ny*nz], v[nx*(ny+1)*nz], w[nx*ny*(nz+1)], each
 *    indexed x fastest over its own face dimensions.
 *  - Boundary vectors are float64; float32 and bfloat16 are internal only,
 *    except in the explicitly typed kernel-level entry points.
 *  - Results are deterministic: the same inputs on the same device give
 *    bitwise identical outputs (all reductions run in a fixed order).
 */
#ifndef CFDMI_H
#define CFDMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CFD_OK = 0,
    CFD_EINVAL = -1,      /* bad argument (sizes, null pointers, options)    */
    CFD_ENOMEM = -2,      /* device or pinned-host allocation failed          */
    CFD_EHIP = -3,        /* a HIP runtime call failed                        */
    CFD_ENOCONV = -4,     /* max_iters reached; x holds the last iterate      */
    CFD_EBREAKDOWN = -5,  /* p^T A p <= 0: matrix not positive definite       */
    CFD_ENONFINITE = -6   /* NaN/Inf met in the right-hand side or iteration  */
};

typedef struct cfd_grid {
    int32_t nx, ny, nz;   /* cells per direction, each >= 1                   */
    double h;             /* cell size (unit cube: 1/N)                       */
} cfd_grid;

/* ------------------------------------------------------------------ */
/* Matrix (Sec. 3.1 CSR storage; Sec. 3.3: the pattern is fixed)        */
/* ------------------------------------------------------------------ */

typedef struct cfd_csr *cfd_csr_t;

/*
 * Assemble, on the device, the 7-point Poisson matrix of the grid in CSR
 * form (Sec. 3.1).  Values are the integer stencil -h^2*Laplacian with
 * homogeneous Neumann walls: the diagonal holds the number of in-domain face
 * neighbours (0..6), each neighbour contributes -1, columns ascend within a
 * row.  pin >= 0 pins that cell: its row becomes the unit row and its
 * neighbours' entries in that column are dropped (a symmetric positive
 * definite matrix); pin < 0 keeps the singular Neumann matrix (valid for
 * cfd_spmv; cfd_solve rejects it).  The values are stored once, in float32
 * (they are small integers, exact in float32); float64 products of them are
 * exact, so every float64 kernel reads the same array.
 * Errors: CFD_EINVAL if a dimension is < 1, pin >= n, or nnz >= 2^31.
 * The handle is freed with cfd_csr_destroy.
 */
int cfd_assemble(const cfd_grid *grid, int64_t pin, void *stream, cfd_csr_t *out);

/* Number of rows (cells) and stored entries. */
int cfd_csr_info(cfd_csr_t A, int64_t *n, int64_t *nnz);

/*
 * Copy the CSR arrays into caller-owned device buffers of n+1, nnz and nnz
 * entries (val receives the values converted to float64, exactly).  Any of
 * the three may be NULL.
 */
int cfd_csr_export(cfd_csr_t A, int32_t *row_ptr, int32_t *col, double *val, void *stream);

void cfd_csr_destroy(cfd_csr_t A);

/*
 * y = A x (Table 1 "spmv") on device vectors of n entries.
 * precision 0: x, y are double*, float64 products and sums.
 * precision 1: x, y are float*,  float32 values, float32 accumulation.
 * x and y must not overlap.
 */
int cfd_spmv(cfd_csr_t A, int32_t precision, const void *x, void *y, void *stream);

/*
 * y = A x from symmetric storage, the layout of Sec. 3.3 (the matrix is
 * symmetric, so only the diagonal and the upper triangle hold values): a
 * CSR of the diagonal and upper entries with their values, plus the column
 * pattern of the lower triangle; the value of lower entry (i, j) is looked
 * up as entry (j, i) among row j's upper entries.  The storage is built from
 * the handle's matrix on the first call (kept with the handle; the build
 * synchronizes the stream once and scans the row counts on the host).
 * Arguments, precisions and result bits are those of cfd_spmv: each row sums
 * its terms in ascending column order, as cfd_spmv does.
 * Errors: CFD_EINVAL (null argument, bad precision), CFD_ENOMEM, CFD_EHIP.
 */
int cfd_spmv_sym(cfd_csr_t A, int32_t precision, const void *x, void *y, void *stream);

/*
 * Make a right-hand side consistent with the pinned matrix, in place on the
 * device: subtract its mean (in float64, fixed summation order), then set
 * b[pin] = 0.  For the singular matrix only the mean is removed.
 */
int cfd_rhs_prepare(cfd_csr_t A, double *b, void *stream);

/*
 * cfd_rhs_prepare for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result bits, with the partial sums in a fixed 8 KiB
 * device array of the library instead of the matrix handle's workspace, so
 * the call allocates nothing (cfd_rhs_prepare allocates that workspace on
 * its first call).  Limit: the reduction grid of n must fit the 1024 partial
 * sums the array holds, true for every n on a device with at most 256 compute
 * units; otherwise CFD_EINVAL.  Call it with A's device current (else
 * CFD_EINVAL).  Every call on one GPU uses that GPU's one array: calls that
 * overlap on the same GPU (concurrent streams or threads) race and must not
 * be issued.
 */
int cfd_rhs_prepare_noalloc(cfd_csr_t A, double *b, void *stream);

/* ------------------------------------------------------------------ */
/* Solver (Sec. 3.1: conjugate gradients, unpreconditioned or with DIC) */
/* ------------------------------------------------------------------ */

typedef struct cfd_net *cfd_net_t;

enum { CFD_PREC_FP64 = 0, CFD_PREC_MIXED = 1 };
enum { CFD_FORM_PINNED = 0, CFD_FORM_PROJECTED = 1 };
enum { CFD_GUESS_ZERO = 0, CFD_GUESS_PREVIOUS = 1 };
enum { CFD_PRECOND_NONE = 0, CFD_PRECOND_DIC_RB = 1 };
enum { CFD_DRIVER_AUTO = 0, CFD_DRIVER_STEPS = 1, CFD_DRIVER_PERSISTENT = 2, CFD_DRIVER_RESIDENT = 3 };

typedef struct cfd_solve_opts {
    int32_t precision;   /* CFD_PREC_FP64: CG in float64 throughout (the
                            matrix values are read from the float32 copy:
                            they are exact, so every product is the same).
                            CFD_PREC_MIXED: float32 matrix values, float32
                            SpMV and vector updates; float64 dot products,
                            step lengths, solution accumulation and true
                            residual (reliable-update refinement).          */
    int32_t max_iters;   /* cap on products q = A p; <= 0 means 100000       */
    double  ru_delta;    /* mixed only: refresh the float64 residual when the
                            recursive residual drops below ru_delta times its
                            maximum since the last refresh; <= 0 means 0.1   */
    cfd_net_t net;       /* non-NULL: the initial guess is the network's
                            prediction scaled by the A-optimal factor
                            (x0 must then be NULL)                           */
    int32_t chunk;       /* iterations enqueued between host polls; <= 0: 16 */
    int32_t timing;      /* nonzero: time sampled launches of the CG SpMV
                            kernel with HIP events (see cfd_solve_info)      */
    int32_t formulation; /* CFD_FORM_PINNED: CG on the stored pinned matrix.
                            CFD_FORM_PROJECTED: CG on the consistent Neumann
                            system A_neu x = c (c_i = b_i - b_pin for the
                            pin's neighbours, c_pin = -sum of the others),
                            whose solutions differ from the pinned solution
                            by a constant; x is shifted so x_pin = b_pin.
                            Same answer, without the pinned cell's isolated
                            small eigenvalue.                                */
    int32_t step_guess;  /* cfd_step only (ignored by cfd_solve):
                            CFD_GUESS_ZERO: the pressure solve starts from
                            zero (or from the network when `net` is set).
                            CFD_GUESS_PREVIOUS: it starts from the pressure
                            already in state->p, the previous step's (the
                            paper's pressure is a field carried from step to
                            step, starting uniform, Sec. 3); CFD_EINVAL
                            together with `net`.                             */
    int32_t precond;     /* CFD_PRECOND_NONE: plain CG (the default).
                            CFD_PRECOND_DIC_RB: CG preconditioned with the
                            paper's diagonal-based incomplete Cholesky
                            factor (Sec. 3.1), eliminating the cells in
                            red-black order (i+j+k even first) so that its
                            recurrences run in parallel (the dependency
                            Sec. 3.3 names).  Computed in the equivalent form
                            of Jacobi-preconditioned CG on the black cells'
                            Schur complement S = D_b - B^T D_r^{-1} B, the
                            red cells recovered at the end; `iters` counts
                            products with S, and the stopping test is the
                            same ||b - A x|| <= tol ||b||.  Both precisions
                            and formulations, x0 and the network apply; the
                            red-black copy of the matrix (float32 values,
                            exact) is built on the first such solve of
                            each formulation and kept with the handle.      */
    int32_t debug_breakdown_at; /* testing only; 0 in normal use.  k > 0: the
                            k-th iteration's step length is rejected as if
                            p^T A p <= 0, so the solve ends with
                            CFD_EBREAKDOWN and the iterate of k-1 updates
                            (the error path, exercised on demand).        */
    double  stop_margin; /* the solve runs until the float64 true residual
                            is <= stop_margin * tol * ||b|| (values > 1 act
                            as 1).  <= 0 means the default: CFD_PREC_FP64 1;
                            CFD_PREC_MIXED 0.05 when the right-hand side's
                            Rayleigh quotient b^T A b / b^T b exceeds 0.5,
                            else 1 (computed on the device, one sweep).
                            float32 rounding noise leaves error in the
                            lowest modes that a residual at tol does not
                            show, most where b holds little of them: at a
                            1e-10 residual the mixed path measured <= 1.3e-10
                            relative pressure error on smooth right-hand
                            sides (quotient ~0.16), 0.4e-9..1.4e-9 on cavity
                            steps (~2) and 1e-9..3e-8 on white noise (~6);
                            <= 3e-10 on all of them at 0.05 * 1e-10.       */
    int32_t driver;      /* unpreconditioned solves only (the DIC path always
                            launches per step):
                            CFD_DRIVER_STEPS: one kernel launch per step
                            (SpMV, vector update, refresh), the host
                            polling the device state every `chunk`
                            iterations.  CFD_DRIVER_PERSISTENT: one
                            cooperative launch runs every iteration, its
                            steps separated by grid barriers (CFD_EINVAL if
                            the device cannot launch cooperatively).
                            CFD_DRIVER_RESIDENT: grids of at most 4096 cells
                            (16^3), both precisions: one workgroup runs the
                            whole solve with the matrix and vectors in
                            registers and LDS (CFD_EINVAL for a larger
                            grid).
                            CFD_DRIVER_AUTO (0): resident up to 4096 cells;
                            else persistent for grids of at most 24^3
                            cells (mixed) or 19^3 cells (float64), where
                            launch overhead sets the iteration time; else
                            one launch per step.                           */
    int32_t barrier_spins; /* persistent driver: polls before a grid barrier
                            wait gives up (<= 0: about 4M, ~0.3 s); the
                            solve then ends with CFD_EHIP.  Testing only.  */
} cfd_solve_opts;

typedef struct cfd_solve_info {
    int32_t iters;          /* products q = A p performed                     */
    int32_t updates;        /* float64 true-residual refreshes performed      */
    int32_t status;         /* CFD_OK or the error code returned              */
    int32_t used_fallback;  /* warm start rejected; zero guess used instead   */
    double  rel_residual;   /* ||b - A x|| / ||b|| of the returned x (float64) */
    double  init_residual;  /* ||b - A x0|| / ||b|| of the initial guess       */
    double  gamma;          /* warm-start scale (0 when not used)             */
    double  seconds;        /* device time from entry to exit (HIP events)    */
    double  spmv_ms;        /* mean duration of the sampled CG SpMV launches  */
    int32_t spmv_samples;   /* number of launches behind spmv_ms              */
    int32_t pad_;
    double  stop_margin;    /* the stopping margin this solve applied (the
                               true residual was taken to <= stop_margin*tol) */
} cfd_solve_info;

/*
 * Solve A x = b for the pinned matrix A to ||b - A x|| <= tol * ||b||
 * (float64 true residual), starting from x0 (device, may be NULL = zero
 * guess, may alias x).  b, x0, x: device double[n]; x must not overlap b,
 * and x0 must either be x itself or not overlap it (CFD_EINVAL).  On CFD_ENOCONV,
 * CFD_EBREAKDOWN and CFD_ENONFINITE, x holds the last iterate and info is
 * filled.  b = 0 returns x = 0 after 0 iterations.  b must be consistent
 * (see cfd_rhs_prepare).  Synchronises the stream before returning.
 */
int cfd_solve(cfd_csr_t A, const double *b, const double *x0, double tol,
              const cfd_solve_opts *opts, double *x, cfd_solve_info *info, void *stream);

/* ------------------------------------------------------------------ */
/* Time step (Sec. 3.1 fractional step on the staggered grid)           */
/* ------------------------------------------------------------------ */

typedef struct cfd_state {
    cfd_grid grid;
    double *u, *v, *w;   /* device face velocities (sizes above)             */
    double *p;           /* device cell pressure, n entries                  */
    double nu;           /* kinematic viscosity (0 = the paper's Euler model) */
    double rho;          /* density                                          */
    double lid_u;        /* speed of the lid: the wall y = ny*h moves in +x   */
    double gx, gy, gz;   /* constant body force ("applyForces")              */
    double t;            /* simulated time, advanced by dt                   */
    int64_t step;        /* step counter, advanced by 1                      */
    cfd_csr_t A;         /* pinned matrix assembled for `grid`               */
    double *rhs;         /* optional device double[n]: receives the step's
                            consistent Poisson right-hand side (NULL: none)  */
} cfd_state;

/*
 * One fractional time step (Sec. 3.1), in place:
 *  forces (u += dt*g on interior faces) -> semi-Lagrangian advection
 *  (first-order back-trace, trilinear sampling, departure point clamped to
 *  the domain) -> explicit viscosity (u += dt*nu*Lap_h u) -> pressure
 *  correction: D = sum of face-flux differences, b = -(rho*h/dt)*D made
 *  consistent, A p = b solved to tol with `opts` (from a zero guess, the
 *  network's prediction, or the previous pressure: opts->step_guess), then
 *  interior faces u -= (dt/(rho*h))*(p_right - p_left).
 * Walls are no-slip; tangential values outside the domain are ghosts
 * 2*U_wall - inside (U_wall = lid_u for u on the lid, else 0).
 * Errors: CFD_EINVAL if dt <= 0 or dt*nu*6/h^2 > 1 (explicit viscosity
 * unstable), plus every cfd_solve error; after a solve error u, v, w hold
 * the velocities before the pressure correction, p the solver's last
 * iterate, and t and step are not advanced.  Synchronises the stream.
 */
int cfd_step(cfd_state *state, double dt, double tol, const cfd_solve_opts *opts,
             cfd_solve_info *info, void *stream);

/* ------------------------------------------------------------------ */
/* Learned warm start: 3-D convolutional network                        */
/* ------------------------------------------------------------------ */
/*
 * Layers l = 0..L-1: 3x3x3 convolutions with replicate (clamped) padding
 * and no bias, channels 1 -> C -> ... -> C -> 1, ReLU after all but the
 * last.  Weights of layer l: [27][c_in][c_out] with tap t = (dz+1)*9 +
 * (dy+1)*3 + (dx+1); output[v][co] = sum_t sum_ci in[clamp(v+d_t)][ci] *
 * W[t][ci][co].  Master weights are float32; the forward and backward
 * passes run in bfloat16 (round to nearest even) with float32 accumulation
 * on the matrix cores.  Inference normalises by s = rms(b): y = s*f(b/s).
 */

/* Create a network with C channels (C = 16) and L = 4 layers, weights from
 * `init` (host float32, cfd_net_param_count values; NULL = all zero). */
int cfd_net_create(int32_t channels, int32_t layers, const float *init, cfd_net_t *out);
int64_t cfd_net_param_count(int32_t channels, int32_t layers);
void cfd_net_destroy(cfd_net_t net);

/* y = s * f(b/s), s = rms(b) (y = 0 when b = 0).  b, y: device double[n]. */
int cfd_net_forward(cfd_net_t net, const cfd_grid *grid, const double *b, double *y, void *stream);

/*
 * One training pair of the warm start from a right-hand side b and its
 * pressure p (device double[n]): input = b / rms(b) and target =
 * (p - mean p) / rms(p - mean p), device float[n] each (0 where the divisor
 * is 0).  The network is bias-free, hence positively homogeneous, so the
 * input scale loses nothing; the target scale does not matter to the solver
 * either (the prediction is rescaled by the A-optimal factor), and unit RMS
 * keeps the loss of every pair and every grid size at the same scale.  Uses
 * the network's scratch; does not synchronise.
 */
int cfd_net_training_pair(cfd_net_t net, const cfd_grid *grid, const double *b, const double *p,
                          float *input, float *target, void *stream);

/*
 * One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean squared error between f(input) and target, averaged over the batch
 * and the voxels.  input, target: device float[batch*n] (already
 * normalised).  *loss receives the loss before the update.  Synchronises.
 */
int cfd_net_train_step(cfd_net_t net, const cfd_grid *grid, int32_t batch,
                       const float *input, const float *target, float lr,
                       float *loss, void *stream);

/* Gradient of that loss w.r.t. the weights at the current weights, without
 * updating them (host float32 output, cfd_net_param_count values). */
int cfd_net_gradient(cfd_net_t net, const cfd_grid *grid, int32_t batch,
                     const float *input, const float *target, float *grad_host,
                     float *loss, void *stream);

int cfd_net_get_params(cfd_net_t net, float *host_buf, int64_t count);
int cfd_net_set_params(cfd_net_t net, const float *host_buf, int64_t count);

/*
 * Kernel-level entry points of one convolution layer (test and tuning use).
 * x: device bf16 bits (uint16) [n][cin]; w: device bf16 bits [27][cin][cout];
 * y: device float [n][cout], float32 accumulation, ReLU applied if relu != 0.
 * cin, cout in {1, 16}.
 */
int cfd_conv3d_forward(const cfd_grid *grid, int32_t cin, int32_t cout,
                       const uint16_t *x, const uint16_t *w, float *y, int32_t relu,
                       void *stream);
/* dx[v][ci] = sum over (u, t) with clamp(u + d_t) = v of sum_co dy[u][co] W[t][ci][co]
 * (the adjoint of cfd_conv3d_forward).  dy: bf16 bits [n][cout]; dx: float [n][cin]. */
int cfd_conv3d_backward_data(const cfd_grid *grid, int32_t cin, int32_t cout,
                             const uint16_t *dy, const uint16_t *w, float *dx, void *stream);
/* dw[t][ci][co] = sum_v x[clamp(v + d_t)][ci] * dy[v][co]; dw: float [27][cin][cout]. */
int cfd_conv3d_backward_weight(const cfd_grid *grid, int32_t cin, int32_t cout,
                               const uint16_t *x, const uint16_t *dy, float *dw, void *stream);

const char *cfd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CFDMI_H */
