// Conjugate-gradient solver (Sec. 3.1 of the paper; Table 1's pcg loop with
// its spmv, dot and vector updates), device-resident.
//
// One iteration is two kernels:
//   A: fold the pending x update, form the new direction p = r + beta p_old
//      on the fly while gathering it for q = A p (double-buffered p), write
//      p, q and the partial sums of p^T q;
//   B: alpha = rho / p^T q, r -= alpha q, partial sums of r^T r.
// Every kernel starts by reducing the partial sums of the previous one in a
// fixed order (every workgroup computes the same bits), so the scalars
// alpha, beta, the convergence test and the control decisions never leave the
// device and no atomics or grid barriers are needed.  The control state is
// double-buffered by launch sequence number: kernel t reads S[t&1] and
// workgroup 0 writes S[(t+1)&1].
//
// A third kernel F ends each chunk of iterations enqueued by the host.  It
// does nothing unless the iteration asked for a refresh (converged on the
// recursive residual, reliable-update trigger, iteration cap, breakdown):
// then it recomputes the true residual b - A x' in float64 for the folded
// iterate x' gathered on the fly.  The next A kernel writes x' into x and
// decides: converged, stop with an error, or continue.
//
// Mixed precision (reliable updates): the matrix values, r, p and q are
// float32, normalised by the residual scale s; the solution x is accumulated
// in float64 (x += s alpha p for every iteration, in order), and b, the true
// residual, every dot product and the scalars are float64.  The x updates are
// deferred: the directions stay in a ring of kDefer float32 buffers with their
// step lengths s alpha queued in the control state, and the B kernel that
// fills the queue applies all kDefer updates to x in one read-modify-write
// pass, oldest first.  That is the float64 x of updating it every iteration,
// for a quarter of the x traffic.  When ||r|| falls below ru_delta
// times its maximum since the last refresh, x' = x + s alpha p and
// r64 = b - A x' are formed in float64; the
// float32 recurrence restarts from r = r64 / ||r64|| keeping the search
// direction (rescaled into the new units).
#include "common.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace cfd {

// Mixed path: x updates queued before one pass applies them.  The A kernel
// writes its direction into the ring slot after the current one; at that
// point at most kDefer - 1 queued directions occupy the other slots.
constexpr int kDefer = 4;
constexpr int kRing = kDefer;

// Persistent driver.  Each grid barrier costs a few microseconds (every
// workgroup writes back and invalidates its XCD's L2 so that the others see
// its writes), which only beats two kernel launches per iteration on the
// smallest grids: measured per iteration (white noise, projected) at 17^3
// 15.6 us against 16.2 (FP64) and 15.9 against 19.8 (mixed) with one launch
// per step, at 20^3 15.8 against 13.6 (FP64) and 15.2 against 16.7 (mixed),
// at 24^3 19.1 against 19.7 (mixed), at 28^3 21.2 against 18.6 (mixed).  So
// mixed grids up to 24^3 cells and float64 grids up to 19^3 use it by
// default (CFD_DRIVER_AUTO).  At most 32 workgroups take part
// (fewer barrier arrivals; measured best from 24^3 to 64^3).  A barrier wait
// gives up after kBarrierSpins polls (about 0.3 s; a step of such a grid
// takes microseconds).
constexpr int64_t kPersistMaxRows = 24 * 24 * 24;    // mixed precision
constexpr int64_t kPersistMaxRows64 = 19 * 19 * 19;  // float64: one launch per step is faster from 20^3
constexpr int kPersistMaxGroups = 32;
constexpr int64_t kBarrierSpins = 1 << 22;

// Stopping margin: the solve runs until the true residual reaches
// tol * margin.  float32 rounding leaves error in the lowest modes that a
// residual at tol cannot show (their share of the residual is lambda_min
// times their share of the error), and it weighs most where b, hence x,
// holds little of those modes: measured at a 1e-10 residual, the mixed
// path's pressure error was <= 1.3e-10 on Gaussian-smoothed right-hand sides
// (128^3, 256^3), but 0.4e-9..1.4e-9 on cavity steps and 1e-9..3e-8 on white
// noise (96^3-160^3); with margin 0.05 all were <= 3e-10.  The Rayleigh
// quotient b^T A b / b^T b tells them apart: 0.16 smoothed, ~2 cavity, ~6
// white noise.  So the mixed path's default margin is 0.05 when it exceeds
// kRoughRq, else 1; float64 CG (the plain method, the oracle's iteration)
// keeps 1.
constexpr double kMixedStopMargin = 0.05;
constexpr double kRoughRq = 0.5;

enum Mode : int32_t { MODE_INIT = 0, MODE_NORMAL = 1, MODE_REFRESH = 2 };
enum Reason : int32_t { R_NONE = 0, R_CONVERGED = 1, R_REFRESH = 2, R_NOCONV = 3, R_BREAKDOWN = 4, R_NONFINITE = 5 };

struct CgState {
    int32_t done;      // 1 once the solve has finished
    int32_t status;    // CFD_* code at exit
    int32_t mode;      // what the next A kernel starts from
    int32_t pending;   // 1: F must fold x and recompute the true residual
    int32_t reason;    // why a refresh was requested
    int32_t iters;     // products q = A p so far
    int32_t updates;   // refreshes performed
    int32_t pcur;      // which p buffer holds the current direction
    int32_t fallback;  // warm start rejected
    int32_t npend;     // mixed: x updates not yet applied (directions in the ring)
    double rho;        // r^T r of the residual that generated the current p
    double rho_new;    // latest recursive r^T r (when a refresh is pending)
    double alpha;      // step length not yet folded into x (0 = none)
    double bnorm;      // ||b||
    double scale;      // s: true residual = s * r (mixed); 1 in float64
    double rmax;       // max ||r|| since the last refresh (mixed, normalised)
    double relres;     // last true relative residual
    double init_relres;
    double gamma;      // warm-start scale
    double xpin;       // folded iterate at the pinned cell (projected formulation)
    double margin;     // stopping margin of this solve
    double sa[kDefer]; // mixed: step lengths s alpha of the pending updates, oldest first
};

struct SolveArgs {
    int64_t n;
    const int32_t *rp, *col;
    const float *v32;       // matrix values: small integers, exact in float32
    double tol, ru_delta;
    int32_t max_iters;
    int32_t break_at;       // testing: iteration whose step length is treated as a breakdown (-1: none)
    int32_t Ga, Gb, Gf;
    int64_t pin;
    int32_t proj;           // 1: CG on the consistent Neumann system, shifted at exit
    int32_t nnb;            // in-domain neighbours of the pinned cell
    int32_t x_vec2;         // x is 16-byte aligned (paired float64 access)
    int64_t nb[6];
    int64_t nxny;
    const double *b;        // right-hand side of the pinned system
    double *c;              // consistent Neumann right-hand side (projected), else b
    double *x;
    const double *x0;       // initial guess (NULL = none)
    const double *y;        // warm-start prediction (NULL = none)
    double *r, *p0, *p1, *q;          // float64 path (r doubles as r64 in mixed)
    float *r32, *q32;
    float *p32[kRing];      // mixed: ring of direction buffers
    double *partA, *partB, *partF, *partF2, *partG1, *partG2, *partFp, *partS;
    double *partR, *partRb; // b^T A b and b^T b partial sums (stopping margin)
    double *tolv;           // [effective tolerance tol * margin, margin], set on the device per solve
    CgState *S;
    unsigned *bar;          // persistent driver: grid barrier [arrivals, generation, error]
    int64_t spin_limit;     // persistent driver: polls before a barrier wait gives up
};

struct Workspace {
    int64_t n = 0;
    int gmax = 0;
    double *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    float *r32 = nullptr, *q32 = nullptr;
    float *p32[kRing] = {};
    double *y = nullptr;
    double *c = nullptr;     // consistent right-hand side (projected formulation)
    double *part = nullptr;  // 11 * gmax doubles
    double *tolv = nullptr;  // effective tolerance and stopping margin
    unsigned *bar = nullptr; // grid barrier of the persistent driver
    CgState *S = nullptr;
    CgState *host = nullptr; // pinned, 2 entries
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evc[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ta, tb;
    struct RbMatrix *rb[2] = {nullptr, nullptr};  // red-black matrices (pinned, projected)
};

void rb_free(struct RbMatrix *m);

void workspace_free(Workspace *ws) {
    if (!ws) return;
    for (RbMatrix *m : ws->rb) rb_free(m);
    double *dd[] = {ws->r, ws->p0, ws->p1, ws->q, ws->y, ws->c, ws->part};
    for (double *p : dd) if (p) (void)hipFree(p);
    float *ff[] = {ws->r32, ws->q32};
    for (float *p : ff) if (p) (void)hipFree(p);
    for (float *p : ws->p32) if (p) (void)hipFree(p);
    if (ws->S) (void)hipFree(ws->S);
    if (ws->bar) (void)hipFree(ws->bar);
    if (ws->tolv) (void)hipFree(ws->tolv);
    if (ws->host) (void)hipHostFree(ws->host);
    hipEvent_t ee[] = {ws->ev0, ws->ev1, ws->evc[0], ws->evc[1]};
    for (hipEvent_t e : ee) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ws->ta) (void)hipEventDestroy(e);
    for (hipEvent_t e : ws->tb) (void)hipEventDestroy(e);
    delete ws;
}

template <class T>
static hipError_t alloc(T **p, int64_t count) {
    if (*p) return hipSuccess;
    return hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
}

// Allocate what the requested path needs (kept until cfd_csr_destroy).
static int ensure_workspace(cfd_csr_t A, bool fp64, bool mixed, bool warm, bool proj = false) {
    if (!A->ws) {
        A->ws = new Workspace();
        A->ws->n = A->n;
        A->ws->gmax = std::max(grid_tiles(A->n, 8), grid_vec(A->n));  // no grid has more than 8 per CU
    }
    Workspace *w = A->ws;
    const int64_t n = A->n;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = alloc(&w->part, (int64_t)w->gmax * 11);
    if (e == hipSuccess) e = alloc(&w->tolv, 2);
    if (e == hipSuccess) e = alloc(&w->S, 2);
    if (e == hipSuccess) e = alloc(&w->bar, 4);
    if (e == hipSuccess && !w->host) e = hipHostMalloc((void **)&w->host, sizeof(CgState) * 2, 0);
    if (e == hipSuccess) e = alloc(&w->r, n);
    if (fp64) {
        if (e == hipSuccess) e = alloc(&w->p0, n);
        if (e == hipSuccess) e = alloc(&w->p1, n);
        if (e == hipSuccess) e = alloc(&w->q, n);
    }
    if (mixed) {
        if (e == hipSuccess) e = alloc(&w->r32, n);
        for (int k = 0; k < kRing && e == hipSuccess; ++k) e = alloc(&w->p32[k], n);
        if (e == hipSuccess) e = alloc(&w->q32, n);
    }
    if (warm && e == hipSuccess) e = alloc(&w->y, n);
    if (proj && e == hipSuccess) e = alloc(&w->c, n);
    if (e == hipSuccess && !w->ev0) e = hipEventCreate(&w->ev0);
    if (e == hipSuccess && !w->ev1) e = hipEventCreate(&w->ev1);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        if (!w->evc[i]) e = hipEventCreateWithFlags(&w->evc[i], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "solver workspace allocation");
    return CFD_OK;
}

double *scratch_partials(cfd_csr_t A) {
    if (ensure_workspace(A, false, false, false) != CFD_OK) return nullptr;
    return A->ws->part + 6 * (int64_t)A->ws->gmax;
}

double *warm_buffer(cfd_csr_t A) {
    if (ensure_workspace(A, false, false, true) != CFD_OK) return nullptr;
    return A->ws->y;
}

// ---------------------------------------------------------------- kernels

#define CG_SHARED(VT)                                  \
    __shared__ __align__(16) int32_t s_col[kSlabLds];  \
    __shared__ __align__(16) VT s_val[kSlabLds];       \
    __shared__ double red[kBlock / 64]
// The same for a kernel of B threads sweeping tiles of B rows.
#define CG_SHARED_B(VT, B)                                  \
    __shared__ __align__(16) int32_t s_col[slab_lds<B>()];  \
    __shared__ __align__(16) VT s_val[slab_lds<B>()];       \
    __shared__ double red[(B) / 64]

__device__ inline bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// The control state, staged once per workgroup in LDS as st.  Read by value
// in every lane, its 160 bytes (and the next state built from it) went
// through per-lane scratch: at 64^3 that was three times the vector traffic
// of the float64 B kernel.
#define CG_STATE(t)                                \
    __shared__ CgState s_st;                       \
    if (threadIdx.x == 0) s_st = a.S[(t) & 1];     \
    __syncthreads();                               \
    const CgState &st = s_st

// Projected formulation.  The stored matrix is the pinned one, A_pin; the
// Neumann matrix differs from it only in the pinned row (which becomes
// deg*e_pin - sum of its neighbours) and in the pinned column (-1 in each
// neighbour row).  Row i of A_neu w is therefore row i of A_pin w plus this
// correction (nonzero in at most 7 rows).
template <class T, class G>
__device__ inline T neu_fix(const SolveArgs &a, int64_t i, T acc, G &&g) {
    if (!a.proj) return acc;
    const int64_t d = i - a.pin;
    if (d > a.nxny || d < -a.nxny) return acc;
    if (d == 0) {
        T s = (T)(a.nnb - 1) * g((int32_t)a.pin);
        for (int q = 0; q < a.nnb; ++q) s -= g((int32_t)a.nb[q]);
        return acc + s;
    }
    for (int q = 0; q < a.nnb; ++q)
        if (i == a.nb[q]) return acc - g((int32_t)a.pin);
    return acc;
}

__device__ inline bool is_pin_nb(const SolveArgs &a, int64_t i) {
    for (int q = 0; q < a.nnb; ++q)
        if (i == a.nb[q]) return true;
    return false;
}

// Initial residual r = c - A x0 (x0 = gamma*y for a warm start), x = x0,
// partial sums of ||r||^2 (full and without the pinned row) and ||b||^2;
// fresh control state.  In mixed mode r is the float64 buffer r64 and d is
// cleared.  Projected formulation: the consistent Neumann right-hand side is
// c_i = b_i - b_pin [i neighbours the pin], c_pin = -sum_{i != pin} c_i, so
// that A_neu x = c with x_pin = b_pin is the pinned solution.
template <bool MIXED>
__global__ void __launch_bounds__(kBlock) cg_init(SolveArgs a, int64_t t) {
    CG_SHARED(float);
    double gamma = 1.0;
    int fallback = 0;
    const double *guess = a.x0;
    if (a.y) {
        // A-optimal scale of the prediction: gamma = c^T y / y^T A y; zero
        // guess if it is not finite or y^T A y <= 0.
        const double yay = reduce_partials(a.partG1, a.Gf, red);
        const double by = reduce_partials(a.partG2, a.Gf, red);
        gamma = by / yay;
        if (!(yay > 0.0) || !std::isfinite(gamma)) {
            gamma = 0.0;
            fallback = 1;
        }
        guess = gamma != 0.0 ? a.y : nullptr;
    }
    const double bpin = a.b[a.pin];
    double cpin = bpin;
    if (a.proj) {
        const double sb = reduce_partials(a.partS, a.Gb, red);
        cpin = -(sb - bpin) + (double)a.nnb * bpin;
    }
    const bool have = guess != nullptr;
    double rr = 0.0, rp = 0.0, bb = 0.0;
    auto xg = [&](int32_t j) -> double {
        if (!have) return 0.0;
        if (a.y) return (j == a.pin) ? 0.0 : gamma * guess[j];
        return guess[j];
    };
    csr_sweep<float>(a.rp, a.col, a.v32, a.n, s_col, s_val, [&](int64_t i, int rs, int re) {
        double acc = 0.0;
        if (have) acc = neu_fix(a, i, row_product<double>(s_col, s_val, rs, re, xg), xg);
        const double bi = a.b[i];
        double ci = bi;
        if (a.proj) {
            ci = (i == a.pin) ? cpin : (is_pin_nb(a, i) ? bi - bpin : bi);
            a.c[i] = ci;
        }
        const double ri = ci - acc;
        a.r[i] = ri;
        if (a.x != a.x0 || a.y) a.x[i] = xg((int32_t)i);
        rr = fma(ri, ri, rr);
        if (!(a.proj && i == a.pin)) rp = fma(ri, ri, rp);
        bb = fma(bi, bi, bb);
    });
    rr = block_sum(rr, red);
    rp = block_sum(rp, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        a.partF[blockIdx.x] = rr;
        a.partFp[blockIdx.x] = rp;
        a.partF2[blockIdx.x] = bb;
    }
    if (lead()) {
        CgState ns{};
        ns.mode = MODE_INIT;
        ns.scale = 1.0;
        ns.gamma = a.y ? gamma : 0.0;
        ns.fallback = fallback;
        ns.xpin = xg((int32_t)a.pin);
        a.S[(t + 1) & 1] = ns;
        if (a.bar) a.bar[0] = a.bar[1] = a.bar[2] = 0u;  // fresh grid barrier for the persistent driver
    }
}

// Fold the pending update into x for row i.  The refresh kernel gathers
// exactly these expressions, so the residual it computed is that of the x
// written here.
__device__ inline double folded64(const SolveArgs &a, int64_t j, double alpha, const double *p) {
    return alpha != 0.0 ? fma(alpha, p[j], a.x[j]) : a.x[j];
}

// Mixed path.  Ring buffer k of the directions (uniform select, so the
// argument block stays in registers).
__device__ inline const float *ring(const SolveArgs &a, int k) {
    const float *p = a.p32[0];
#pragma unroll
    for (int q = 1; q < kRing; ++q) p = (k == q) ? a.p32[q] : p;
    return p;
}
// Buffer of pending update e (0 = oldest); the newest is the current direction.
__device__ inline int pend_slot(const CgState &st, int e) {
    return (st.pcur - (st.npend - 1 - e) + kRing) % kRing;
}
// x + every pending update, oldest first: the float64 x that per-iteration
// updates would hold.
__device__ inline double folded32(const SolveArgs &a, const CgState &st, int64_t j) {
    double xj = a.x[j];
#pragma unroll
    for (int e = 0; e < kDefer; ++e)
        if (e < st.npend && st.sa[e] != 0.0) xj = fma(st.sa[e], (double)ring(a, pend_slot(st, e))[j], xj);
    return xj;
}

// Decision taken at the start of every A kernel from the reduced residual
// norm.  Identical in every workgroup.
struct Decision {
    bool stop;        // no iteration in this kernel
    bool zero_x;      // b == 0: the answer is x = 0
    bool fold;        // fold the refreshed update into x (refresh mode)
    CgState ns;       // state to publish
    double beta;      // direction coefficient (normal mode)
    double cref;      // mixed refresh: coefficient on the old direction
    double inv_s;     // mixed refresh: 1 / new scale
    double shift;     // projected formulation, final x: + (b_pin - x_pin)
};

// The decision from the reduced sums: rr = ||r||^2 (normal mode: the
// recursive residual); after cg_init or a refresh also rrp (the pinned
// system's ||r||^2) and, after cg_init, bb = ||b||^2.
template <bool MIXED>
__device__ inline Decision decide_core(const SolveArgs &a, const CgState &st, double rr_in, double rrp_in,
                                       double bb_in) {
    Decision D;
    D.stop = false;
    D.zero_x = false;
    D.fold = false;
    D.beta = 0.0;
    D.cref = 0.0;
    D.inv_s = 1.0;
    D.shift = 0.0;
    CgState ns = st;
    if (st.mode == MODE_NORMAL) {
        const double rr = rr_in;
        const double nr = sqrt(rr);
        const double thr = a.tolv[0] * st.bnorm;
        int reason = R_NONE;
        if (!std::isfinite(rr)) reason = R_NONFINITE;
        else if (nr * st.scale <= thr) reason = R_CONVERGED;
        else if (MIXED && nr < a.ru_delta * st.rmax) reason = R_REFRESH;
        else if (st.iters >= a.max_iters) reason = R_NOCONV;
        if (reason != R_NONE) {
            ns.pending = 1;
            ns.reason = reason;
            ns.rho_new = rr;
            D.stop = true;
        } else {
            D.beta = rr / st.rho;
            ns.rho = rr;
            ns.rmax = std::max(st.rmax, nr);
        }
    } else {
        // rr: ||r||^2 of the system being iterated; rrp: ||r||^2 of the pinned
        // system at the (shifted) iterate, which decides convergence
        const double rr = rr_in, rrp = rrp_in;
        if (st.mode == MODE_INIT) {
            ns.bnorm = sqrt(bb_in);
            ns.margin = a.tolv[1];
        } else {
            D.fold = true;  // refresh (float64 path): this A kernel folds x += alpha p
        }
        const double tr = sqrt(rr), trp = sqrt(rrp);
        const double bn = ns.bnorm;
        ns.reason = R_NONE;
        ns.alpha = 0.0;
        if (!std::isfinite(bn) || !std::isfinite(rr) || !std::isfinite(rrp)) {
            ns.done = 1;
            ns.status = CFD_ENONFINITE;
            ns.relres = NAN;
        } else if (bn == 0.0) {
            ns.done = 1;
            ns.status = CFD_OK;
            ns.relres = 0.0;
            D.zero_x = true;
        } else {
            ns.relres = trp / bn;
            if (st.mode == MODE_INIT) ns.init_relres = ns.relres;
            if (trp <= a.tolv[0] * bn) {
                ns.done = 1;
                ns.status = CFD_OK;
            } else if (st.reason == R_NOCONV || st.iters >= a.max_iters) {
                ns.done = 1;
                ns.status = CFD_ENOCONV;
            } else if (st.reason == R_BREAKDOWN) {
                ns.done = 1;
                ns.status = CFD_EBREAKDOWN;
            } else if (st.reason == R_NONFINITE) {
                ns.done = 1;
                ns.status = CFD_ENONFINITE;
            }
        }
        if (ns.done) {
            D.stop = true;
            if (a.proj && !D.zero_x) D.shift = a.b[a.pin] - st.xpin;
        } else if (MIXED) {
            // restart the float32 recurrence from r64 / ||r64||, keeping the
            // old direction (rescaled into the new units) after a refresh:
            // beta = rho_new / (rho_old (s_old/s_new)^2) with rho_new = 1, and
            // the rescaled direction p_old * s_old / s_new.
            D.inv_s = 1.0 / tr;
            D.cref = (st.mode == MODE_INIT) ? 0.0 : tr / (st.scale * st.rho);
            ns.scale = tr;
            ns.rho = 1.0;
            ns.rmax = 1.0;
        } else {
            D.beta = 0.0;  // float64: restart from the true residual
            ns.rho = rr;
        }
    }
    D.ns = ns;
    return D;
}

// The decision at the start of an A step, from the partial sums the
// previous step left (identical in every workgroup).
template <bool MIXED, int B = kBlock>
__device__ inline Decision decide(const SolveArgs &a, const CgState &st, double *red) {
    if (st.mode == MODE_NORMAL) return decide_core<MIXED>(a, st, reduce_partials<B>(a.partB, a.Gb, red), 0.0, 0.0);
    const double rr = reduce_partials<B>(a.partF, a.Gf, red);
    const double rrp = reduce_partials<B>(a.partFp, a.Gf, red);
    const double bb = st.mode == MODE_INIT ? reduce_partials<B>(a.partF2, a.Gf, red) : 0.0;
    return decide_core<MIXED>(a, st, rr, rrp, bb);
}

// Bodies of the solver's kernels, shared by the launch-per-step driver (one
// kernel per step, below) and the persistent driver (cg_persist): each takes
// the control state every workgroup holds and returns the next one (the same
// bits in every thread).

// The solve has ended (float64): x = 0 (b == 0) or x with the pending update
// folded in, plus the projected formulation's shift.
__device__ __forceinline__ void a64_final(const SolveArgs &a, const CgState &st, const Decision &D) {
    const double *pold = st.pcur ? a.p1 : a.p0;
    const double alpha = st.alpha;
    if (D.zero_x || D.fold || a.proj)
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock)
            a.x[i] = D.zero_x ? 0.0
                   : (a.proj && i == a.pin) ? a.b[a.pin]
                   : (D.fold ? folded64(a, i, alpha, pold) : a.x[i]) + D.shift;
}

// A step, float64.  Normal: x += alpha p_old; p = r + beta p_old; q = A p.
// Init/refresh: (fold x) p = r; q = A p.  The matrix values come from the
// float32 copy: they are small integers, so each float64 product, and the
// result, is bit-identical to the one with the float64 copy, at 4 B per entry
// less.  The same holds for every kernel of the solver that reads values.
__device__ __forceinline__ CgState a64_next(const CgState &st, const Decision &D) {
    CgState ns = D.ns;
    ns.mode = MODE_NORMAL;
    ns.iters = st.iters + 1;
    ns.pcur = 1 - st.pcur;
    ns.alpha = 0.0;
    return ns;
}

__device__ __forceinline__ CgState a64_body(const SolveArgs &a, const CgState &st, const Decision &D, double *red,
                                            int32_t *s_col, float *s_val) {
    const double *pold = st.pcur ? a.p1 : a.p0;
    const double alpha = st.alpha;  // pending update (normal mode or refresh fold)
    double *pnew = st.pcur ? a.p0 : a.p1;
    const bool normal = st.mode == MODE_NORMAL;
    const bool fold = normal || D.fold;
    const double beta = D.beta;
    double pq = 0.0;
    auto wg = [&](int32_t j) -> double { return normal ? fma(beta, pold[j], a.r[j]) : a.r[j]; };
    // the streamed sweep: 3 % faster here than csr_sweep (256^3), no spills.
    // Each row's direction w_i is formed from its r and p_old, loaded a tile
    // ahead, and staged in LDS with the slab; the row products take the
    // neighbours inside the tile from there (the same value wg forms).
    __shared__ double s_w[kBlock];
    int64_t w0 = 0;
    int wn = 0;
    auto own = [&](int64_t i) -> f64x2 {
        f64x2 o;
        o.x = a.r[i];
        o.y = normal ? pold[i] : 0.0;
        return o;
    };
    auto stage = [&](int64_t r0, int nr, const f64x2 &o) {
        w0 = r0;
        wn = nr;
        if ((int)threadIdx.x < nr) s_w[threadIdx.x] = normal ? fma(beta, o.y, o.x) : o.x;
    };
    auto wl = [&](int32_t j) -> double {
        const uint32_t d = (uint32_t)((int64_t)j - w0);
        return d < (uint32_t)wn ? s_w[d] : wg(j);
    };
    csr_stream_rows_staged<float>(a.rp, a.col, a.v32, 0, a.n, s_col, s_val, own, stage,
                                  [&](int64_t i, int rs, int re, f64x2 o) {
        const double acc = neu_fix(a, i, row_product<double>(s_col, s_val, rs, re, wl), wg);
        const double wi = normal ? fma(beta, o.y, o.x) : o.x;
        if (fold && alpha != 0.0) store_stream(a.x + i, folded64(a, i, alpha, pold));
        store_stream(pnew + i, wi);
        store_stream(a.q + i, acc);
        pq = fma(wi, acc, pq);
    });
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) a.partA[blockIdx.x] = pq;
    CgState ns = D.ns;
    ns.mode = MODE_NORMAL;
    ns.iters = st.iters + 1;
    ns.pcur = 1 - st.pcur;
    ns.alpha = 0.0;
    return ns;
}

__global__ void __launch_bounds__(kBlock) cg_a64(SolveArgs a, int64_t t) {
    CG_SHARED(float);
    const CgState st = a.S[t & 1];
    CgState *out = &a.S[(t + 1) & 1];
    if (st.done || st.pending) {
        if (lead()) *out = st;
        return;
    }
    const Decision D = decide<false>(a, st, red);
    if (D.stop) {
        if (D.ns.done) a64_final(a, st, D);
        if (lead()) *out = D.ns;
        return;
    }
    // the next state depends on nothing the sweep computes: published first,
    // it need not stay live (in scratch) across the sweep
    if (lead()) *out = a64_next(st, D);
    (void)a64_body(a, st, D, red, s_col, s_val);
}

// The solve has ended (mixed): x = 0, or x plus the queued updates, plus the
// projected formulation's shift.
template <int B = kBlock>
__device__ __forceinline__ void a32_final(const SolveArgs &a, const CgState &st, const Decision &D) {
    if (D.zero_x || st.npend > 0 || a.proj)
        for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * B) {
            a.x[i] = D.zero_x ? 0.0
                   : (a.proj && i == a.pin) ? a.b[a.pin]
                   : folded32(a, st, i) + D.shift;
        }
}

// A step, mixed.  Normal: p = r + beta p_old; q = A p (float32).
// Init/refresh: r = r64 / s_new; p = r + cref p_old; q = A p.  x is written
// only when the solve ends (queued updates, projected shift); the B steps
// apply the queue otherwise.
template <int B = kBlock>
__device__ __forceinline__ CgState a32_body(const SolveArgs &a, const CgState &st, const Decision &D, double *red,
                                            int32_t *s_col, float *s_val) {
    const float *pold = ring(a, st.pcur);
    float *pnew = const_cast<float *>(ring(a, (st.pcur + 1) % kRing));
    const bool normal = st.mode == MODE_NORMAL;
    const bool use_p = normal || st.mode == MODE_REFRESH;
    const float cf = normal ? (float)D.beta : (float)D.cref;
    const double inv_s = D.inv_s;
    double pq = 0.0;
    auto rg = [&](int64_t j) -> float { return normal ? a.r32[j] : (float)(a.r[j] * inv_s); };
    auto wg = [&](int32_t j) -> float { return use_p ? fmaf(cf, pold[j], rg(j)) : rg(j); };
    // own row's r and p_old, loaded a tile ahead with the CSR slab (measured
    // 7.6% faster at 256^3 than loading them in the row body).  Each row's
    // direction w_i goes to LDS with the slab, so the row products take the
    // neighbours inside the tile (+-1, and one of +-nx) from there instead
    // of gathering r and p_old (the same value, formed the same way).
    __shared__ float s_w[B];
    auto own = [&](int64_t i) -> float2 { return make_float2(rg(i), use_p ? pold[i] : 0.0f); };
    const int64_t ntiles = (a.n + B - 1) / B;
    const TileRange tr = tile_range(ntiles);
    const int tid = threadIdx.x;
    SlabPipe<float, B> P;
    float2 next{};
    if (tr.first < tr.end) {
        P.fetch(a.rp, a.col, a.v32, a.n, tr.first);
        if (tid < P.nr) next = own(P.r0 + tid);
    }
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t r0 = P.r0;
        const int nr = P.nr, rs = P.rs, re = P.re;
        const float2 o = next;
        const float wi = use_p ? fmaf(cf, o.y, o.x) : o.x;
        P.commit(s_col, s_val);
        if (tid < nr) s_w[tid] = wi;
        __syncthreads();
        if (t + tr.step < tr.end) {
            P.fetch(a.rp, a.col, a.v32, a.n, t + tr.step);
            if (tid < P.nr) next = own(P.r0 + tid);
        }
        if (tid < nr) {
            const int64_t i = r0 + tid;
            auto wl = [&](int32_t j) -> float {
                const uint32_t d = (uint32_t)((int64_t)j - r0);
                return d < (uint32_t)nr ? s_w[d] : wg(j);
            };
            const float acc = neu_fix(a, i, row_product<float>(s_col, s_val, rs, re, wl), wg);
            if (!normal) store_stream(a.r32 + i, o.x);
            store_stream(pnew + i, wi);
            store_stream(a.q32 + i, acc);
            pq = fma((double)wi, (double)acc, pq);
        }
        __syncthreads();
    }
    pq = block_sum<B>(pq, red);
    if (threadIdx.x == 0) a.partA[blockIdx.x] = pq;
    CgState ns = D.ns;
    ns.mode = MODE_NORMAL;
    ns.iters = st.iters + 1;
    ns.pcur = (st.pcur + 1) % kRing;
    ns.alpha = 0.0;
    return ns;
}

// A kernel, mixed: workgroups of B threads sweeping tiles of B rows.  The
// kernel is latency-bound: 8 waves per SIMD (64 VGPRs per lane, the most a
// SIMD holds at that size) measured fastest at 256^3.
template <int B>
__global__ void __launch_bounds__(B, 8) cg_a32(SolveArgs a, int64_t t) {
    CG_SHARED_B(float, B);
    const CgState st = a.S[t & 1];
    CgState *out = &a.S[(t + 1) & 1];
    if (st.done || st.pending) {
        if (lead()) *out = st;
        return;
    }
    const Decision D = decide<true, B>(a, st, red);
    if (D.stop) {
        if (D.ns.done) a32_final<B>(a, st, D);
        if (lead()) *out = D.ns;
        return;
    }
    const CgState ns = a32_body<B>(a, st, D, red, s_col, s_val);
    if (lead()) *out = ns;
}

// B step: alpha = rho / p^T q; r -= alpha q; partial sums of r^T r.
// Returns false (and touches nothing) when the step length is rejected.
template <bool MIXED>
__device__ __forceinline__ bool b_core(const SolveArgs &a, const CgState &st, double *red, double &alpha,
                                       double &sa_new) {
    const double pq = reduce_partials(a.partA, a.Ga, red);
    alpha = st.rho / pq;
    if (!(pq > 0.0) || !std::isfinite(alpha) || st.iters == a.break_at) return false;
    double rr = 0.0;
    sa_new = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (MIXED) {
        // Queue x += s alpha p for this iteration's direction (the ring's
        // current slot).  When that fills the queue, apply all kDefer updates
        // to x here, oldest first; the older directions sit in the slots
        // before the current one.
        sa_new = st.scale * alpha;
        if (st.npend == kDefer - 1) {
            const float *pe[kDefer];
            double se[kDefer];
#pragma unroll
            for (int e = 0; e < kDefer; ++e) {
                pe[e] = ring(a, (st.pcur - (kDefer - 1 - e) + kRing) % kRing);
                se[e] = e < kDefer - 1 ? st.sa[e] : sa_new;
            }
            const int64_t n2 = a.x_vec2 ? a.n / 2 : 0;
            f64x2 *x2 = reinterpret_cast<f64x2 *>(a.x);
            for (int64_t v = first; v < n2; v += stride) {
                f64x2 xv = __builtin_nontemporal_load(x2 + v);
#pragma unroll
                for (int e = 0; e < kDefer; ++e) {
                    const f32x2 pv = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(pe[e]) + v);
                    if (se[e] != 0.0) {
                        xv.x = fma(se[e], (double)pv.x, xv.x);
                        xv.y = fma(se[e], (double)pv.y, xv.y);
                    }
                }
                store_stream(x2 + v, xv);
            }
            for (int64_t i = n2 * 2 + first; i < a.n; i += stride) {
                double xi = a.x[i];
#pragma unroll
                for (int e = 0; e < kDefer; ++e)
                    if (se[e] != 0.0) xi = fma(se[e], (double)pe[e][i], xi);
                a.x[i] = xi;
            }
        }
        const float af = (float)alpha;
        const int64_t nv = a.n / 4;
        f32x4 *r4 = reinterpret_cast<f32x4 *>(a.r32);
        const f32x4 *q4 = reinterpret_cast<const f32x4 *>(a.q32);
        for (int64_t v = first; v < nv; v += stride) {
            // plain loads (measured faster than non-temporal ones here: the
            // lines they leave cached serve the next A kernel), streamed store
            f32x4 r = r4[v];
            const f32x4 q = q4[v];
            r.x = fmaf(-af, q.x, r.x);
            r.y = fmaf(-af, q.y, r.y);
            r.z = fmaf(-af, q.z, r.z);
            r.w = fmaf(-af, q.w, r.w);
            store_stream(r4 + v, r);
            rr = fma((double)r.x, (double)r.x, rr);
            rr = fma((double)r.y, (double)r.y, rr);
            rr = fma((double)r.z, (double)r.z, rr);
            rr = fma((double)r.w, (double)r.w, rr);
        }
        for (int64_t i = nv * 4 + first; i < a.n; i += stride) {
            const float r = fmaf(-af, a.q32[i], a.r32[i]);
            a.r32[i] = r;
            rr = fma((double)r, (double)r, rr);
        }
    } else {
        const int64_t nv = a.n / 2;
        f64x2 *r2 = reinterpret_cast<f64x2 *>(a.r);
        const f64x2 *q2 = reinterpret_cast<const f64x2 *>(a.q);
        for (int64_t v = first; v < nv; v += stride) {
            f64x2 r = r2[v];
            const f64x2 q = q2[v];
            r.x = fma(-alpha, q.x, r.x);
            r.y = fma(-alpha, q.y, r.y);
            store_stream(r2 + v, r);
            rr = fma(r.x, r.x, rr);
            rr = fma(r.y, r.y, rr);
        }
        for (int64_t i = nv * 2 + first; i < a.n; i += stride) {
            const double r = fma(-alpha, a.q[i], a.r[i]);
            a.r[i] = r;
            rr = fma(r, r, rr);
        }
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) a.partB[blockIdx.x] = rr;
    return true;
}

// The state after a B step (ok: its step length was accepted).
template <bool MIXED>
__device__ __forceinline__ CgState b_next(const CgState &st, bool ok, double alpha, double sa_new) {
    CgState ns = st;
    if (!ok) {
        ns.pending = 1;
        ns.reason = R_BREAKDOWN;
        ns.alpha = 0.0;
        // mixed: this iteration's direction is not queued, so the newest
        // queued update is the one before it; point pcur back at it
        // (pend_slot() counts the queue back from pcur)
        if (MIXED) ns.pcur = (st.pcur - 1 + kRing) % kRing;
        return ns;
    }
    ns.alpha = alpha;
    if (MIXED) {
        if (st.npend < kDefer - 1) {
#pragma unroll
            for (int e = 0; e < kDefer - 1; ++e)
                if (e == st.npend) ns.sa[e] = sa_new;
            ns.npend = st.npend + 1;
        } else {
            ns.npend = 0;  // applied in b_core
        }
    }
    return ns;
}

template <bool MIXED>
__global__ void __launch_bounds__(kBlock) cg_b(SolveArgs a, int64_t t) {
    __shared__ double red[kBlock / 64];
    CG_STATE(t);
    CgState *out = &a.S[(t + 1) & 1];
    if (st.done || st.pending) {
        if (lead()) *out = st;
        return;
    }
    double alpha, sa_new;
    const bool ok = b_core<MIXED>(a, st, red, alpha, sa_new);
    if (lead()) *out = b_next<MIXED>(st, ok, alpha, sa_new);
}

// F kernel: when a refresh is pending, r = c - A x' in float64 with the
// folded iterate x' = x + alpha p (float64) or x plus every pending
// s alpha p (mixed) gathered on the fly.  x itself is only written by the next A kernel (which
// never gathers x), so no workgroup can see a half-updated x here.
template <bool MIXED>
__device__ __forceinline__ CgState f_body(const SolveArgs &a, const CgState &st, double *red, int32_t *s_col,
                                          float *s_val) {
    const double alpha = st.alpha;
    const double *p64 = st.pcur ? a.p1 : a.p0;
    auto xg = [&](int32_t j) -> double {
        if constexpr (MIXED) return folded32(a, st, j);
        else return folded64(a, j, alpha, p64);
    };
    double rr = 0.0, rp = 0.0;
    csr_sweep<float>(a.rp, a.col, a.v32, a.n, s_col, s_val, [&](int64_t i, int rs, int re) {
        const double acc = neu_fix(a, i, row_product<double>(s_col, s_val, rs, re, xg), xg);
        const double ri = a.c[i] - acc;
        a.r[i] = ri;
        rr = fma(ri, ri, rr);
        if (!(a.proj && i == a.pin)) rp = fma(ri, ri, rp);
    });
    rr = block_sum(rr, red);
    rp = block_sum(rp, red);
    if (threadIdx.x == 0) {
        a.partF[blockIdx.x] = rr;
        a.partFp[blockIdx.x] = rp;
    }
    CgState ns = st;
    ns.pending = 0;
    ns.mode = MODE_REFRESH;
    ns.updates = st.updates + 1;
    ns.xpin = xg((int32_t)a.pin);  // nobody writes x, p or d in this step
    return ns;
}

template <bool MIXED>
__global__ void __launch_bounds__(kBlock) cg_refresh(SolveArgs a, int64_t t) {
    CG_SHARED(float);
    CG_STATE(t);
    CgState *out = &a.S[(t + 1) & 1];
    if (st.done || !st.pending) {
        if (lead()) *out = st;
        return;
    }
    const CgState ns = f_body<MIXED>(a, st, red, s_col, s_val);
    if (lead()) *out = ns;
}

// ---------------------------------------------------------------- persistent driver
//
// One cooperative launch runs the whole iteration: every workgroup is
// resident, and the steps that the launch-per-step driver puts in separate
// kernels (A, B, refresh) are separated by grid barriers instead.  Every
// workgroup keeps the control state itself: the decisions are taken from
// partial sums reduced in a fixed order, so all workgroups hold the same bits
// and leave the loop together.  For grids small enough that the launches,
// not the memory traffic, set the iteration time.

// Grid barrier: arrivals are counted in bar[0]; the last to arrive resets the
// count and advances the generation in bar[1], which the others poll.  The
// fences before arriving and after leaving make every write issued before the
// barrier visible to every workgroup after it (agent scope: across the XCDs'
// L2 caches).  The wait is bounded: after spin_limit polls it sets bar[2]
// and fails, and so does every barrier after it, so all workgroups leave.
__device__ inline bool grid_sync(const SolveArgs &a, unsigned &seen) {
    __shared__ int ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned *count = a.bar, *gen = a.bar + 1, *err = a.bar + 2;
        const unsigned target = seen + 1;
        __threadfence();
        if (atomicAdd(count, 1u) == gridDim.x - 1) {
            atomicExch(count, 0u);
            __threadfence();
            atomicExch(gen, target);
        } else {
            int64_t spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > a.spin_limit) {
                    atomicExch(err, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ok = 0;
        seen = target;
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

// The same steps, decisions and arithmetic as the launch-per-step driver
// (with one grid size for every step, so the partial sums group differently).
// Reads the state cg_init left in S[t & 1], writes the final one to
// S[(t + 1) & 1]; x is written before it returns.
template <bool MIXED>
__global__ void __launch_bounds__(kBlock) cg_persist(SolveArgs a, int64_t t) {
    CG_SHARED(float);
    CgState st = a.S[t & 1];
    unsigned seen = 0;
    bool ok = true;
    while (!st.done) {
        if (st.pending) {
            st = f_body<MIXED>(a, st, red, s_col, s_val);
            if (!(ok = grid_sync(a, seen))) break;
            continue;
        }
        const Decision D = decide<MIXED>(a, st, red);
        if (D.stop) {
            if (D.ns.done) {
                if (MIXED) a32_final(a, st, D);
                else a64_final(a, st, D);
            }
            st = D.ns;
            continue;
        }
        st = MIXED ? a32_body(a, st, D, red, s_col, s_val) : a64_body(a, st, D, red, s_col, s_val);
        if (!(ok = grid_sync(a, seen))) break;
        double alpha, sa_new;
        const bool stepped = b_core<MIXED>(a, st, red, alpha, sa_new);
        st = b_next<MIXED>(st, stepped, alpha, sa_new);
        if (!(ok = grid_sync(a, seen))) break;
    }
    if (!ok) {
        st.done = 1;
        st.status = CFD_EHIP;
    }
    if (lead()) a.S[(t + 1) & 1] = st;
}

// ---------------------------------------------------------------- resident driver
//
// Float64, small grids (up to kResMaxRows cells): one workgroup runs the
// whole solve after cg_init, with no grid barrier and no global round trip
// per step.  Thread t owns rows t, t + kResThreads, ...: their columns (as
// 16-bit offsets from the row, |col - i| < n <= kResMaxRows), x, r and q
// stay in its registers, the matrix values in LDS, and the direction (or x
// during a refresh) in LDS, where the row products gather it.  Thread 0 holds the control state in LDS and takes each
// decision with decide_core, the launch-per-step driver's rules; the
// per-row arithmetic is that driver's too.  The sums are reduced over one
// workgroup instead of per-workgroup partial sums, and x takes each step
// x += alpha p at once rather than at the next A step (the same fma).
constexpr int kResThreads = 1024;
constexpr int kResRows = 4;
constexpr int64_t kResMaxRows = (int64_t)kResThreads * kResRows;

enum ResOp : int32_t { OP_END = 0, OP_REFRESH = 1, OP_STEP = 2, OP_FINAL = 3 };

struct ResCtl {
    CgState st;
    double beta, shift, alpha;
    double cref, inv_s, sa;  // mixed: restart coefficient, 1 / s, s alpha
    int32_t op, normal, use_p, zero_x, update;
};

// Thread 0: the next operation from the control state and the latest sums.
// Not inlined: the decision's temporaries then take call-clobbered
// registers instead of competing with the rows each thread keeps.  The
// arguments are the fields of SolveArgs that the decision reads.
template <bool MIXED>
__device__ __noinline__ void res_control(double *tolv, double ru_delta, int32_t max_iters, int32_t proj,
                                         double bpin, ResCtl *cp, double rr, double rrp, double bb) {
    SolveArgs a{};
    a.tolv = tolv;
    a.ru_delta = ru_delta;
    a.max_iters = max_iters;
    a.proj = proj;
    a.b = &bpin;
    a.pin = 0;
    ResCtl &c = *cp;
    for (;;) {
        if (c.st.done) {
            c.op = OP_END;
            return;
        }
        if (c.st.pending) {
            c.op = OP_REFRESH;
            return;
        }
        const Decision D = decide_core<MIXED>(a, c.st, rr, rrp, bb);
        if (D.stop) {
            c.st = D.ns;
            if (D.ns.done) {
                c.op = OP_FINAL;
                c.zero_x = D.zero_x;
                c.shift = D.shift;
                return;
            }
            continue;  // a refresh is pending
        }
        c.op = OP_STEP;
        c.beta = D.beta;
        c.cref = D.cref;
        c.inv_s = D.inv_s;
        c.normal = c.st.mode == MODE_NORMAL;
        c.use_p = c.st.mode == MODE_NORMAL || c.st.mode == MODE_REFRESH;
        c.st = D.ns;
        return;
    }
}

// f(integral_constant<int, k>) for k = 0 .. K-1: the row slot is a
// compile-time index, so the per-row arrays stay in registers.
template <int K, class F>
__device__ __forceinline__ void res_for(F &&f) {
    if constexpr (K > 0) {
        res_for<K - 1>(f);
        f(std::integral_constant<int, K - 1>{});
    }
}

// MIXED: the launch-per-step mixed path's arithmetic (a32_body, b_core,
// f_body): float32 r, q and direction, the direction gathered as float32,
// x and the refreshed residual r64 in float64; x takes s alpha p at once
// (the same fma, in the same order, as the queue applies it).
template <bool MIXED>
__global__ void __launch_bounds__(kResThreads) cg_resident(SolveArgs a, int64_t t) {
    typedef typename std::conditional<MIXED, float, double>::type VT;
    __shared__ float s_val[kResRows * kMaxRowNnz * kResThreads];  // [row slot][entry][thread]
    __shared__ double s_v[kResMaxRows];  // the direction (as VT), or x during a refresh
    __shared__ double red[kResThreads / 64];
    __shared__ ResCtl ctl;
    VT *s_p = reinterpret_cast<VT *>(s_v);
    const int tid = threadIdx.x;
    const int64_t n = a.n;
    constexpr int kPacked = (kMaxRowNnz + 1) / 2;
    uint32_t cc[kResRows][kPacked];  // two 16-bit column offsets per word
    // per row slot k, 4 bits at 4k: the row length (0..7), and bit 3 set for
    // the rows the projected formulation corrects (the pin and its neighbours)
    uint32_t meta = 0u;
    // float64: r in r64; mixed: r in units of s in r32, and the float64
    // residual of cg_init and of each refresh in a.r (read back by the same
    // thread in the step after it: out of the registers the loop carries)
    double x[kResRows];
    double r64[kResRows];
    VT r32[kResRows], q[kResRows];
    VT pk[kResRows];  // mixed: this thread's rows of the direction
    auto row = [&](auto kc) -> int64_t { return tid + (int64_t)decltype(kc)::value * kResThreads; };
    res_for<kResRows>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int64_t i = row(kc);
        const bool own = i < n;
        const int32_t e0 = own ? a.rp[i] : 0;
        const int len = own ? a.rp[i + 1] - e0 : 0;
        const bool fix = own && a.proj && (i == a.pin || is_pin_nb(a, i));
        meta |= ((uint32_t)len | (fix ? 8u : 0u)) << (4 * k);
#pragma unroll
        for (int w = 0; w < kPacked; ++w) cc[k][w] = 0u;
#pragma unroll
        for (int e = 0; e < kMaxRowNnz; ++e) {
            const int32_t off = e < len ? a.col[e0 + e] - (int32_t)i : 0;
            cc[k][e / 2] |= ((uint32_t)off & 0xffffu) << (16 * (e & 1));
            s_val[(k * kMaxRowNnz + e) * kResThreads + tid] = e < len ? a.v32[e0 + e] : 0.0f;
        }
        x[k] = own ? a.x[i] : 0.0;
        r64[k] = (!MIXED && own) ? a.r[i] : 0.0;
        r32[k] = q[k] = pk[k] = (VT)0;
    });
    // row k of A (A_neu in the projected formulation) times the vector in
    // s_v (float64: the direction or x) or, mixed, in s_p (the direction)
    auto sv64 = [&](int32_t j) -> double { return s_v[j]; };
    auto svp = [&](int32_t j) -> VT { return s_p[j]; };
    auto rowprod = [&](auto kc, auto g) {
        using T = decltype(g(0));
        constexpr int k = decltype(kc)::value;
        const int32_t i = (int32_t)row(kc);
        const uint32_t m = (meta >> (4 * k)) & 15u;
        const int len = (int)(m & 7u);
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < kMaxRowNnz; ++e)
            if (e < len) {
                const int32_t j = i + (int32_t)(int16_t)(cc[k][e / 2] >> (16 * (e & 1)));
                acc = fma(T(s_val[(k * kMaxRowNnz + e) * kResThreads + tid]), g(j), acc);
            }
        return (m & 8u) ? neu_fix(a, (int64_t)i, acc, g) : acc;
    };
    // the first decision reduces the partial sums cg_init left
    if (tid == 0) ctl.st = a.S[t & 1];
    __syncthreads();
    double rr = 0.0, rrp = 0.0, bb = 0.0;
    if (!ctl.st.done && !ctl.st.pending) {
        if (ctl.st.mode == MODE_NORMAL) {
            rr = reduce_partials<kResThreads>(a.partB, a.Gb, red);
        } else {
            rr = reduce_partials<kResThreads>(a.partF, a.Gf, red);
            rrp = reduce_partials<kResThreads>(a.partFp, a.Gf, red);
            if (ctl.st.mode == MODE_INIT) bb = reduce_partials<kResThreads>(a.partF2, a.Gf, red);
        }
    }
    const double bpin = a.proj ? a.b[a.pin] : 0.0;
    for (;;) {
        if (tid == 0) res_control<MIXED>(a.tolv, a.ru_delta, a.max_iters, a.proj, bpin, &ctl, rr, rrp, bb);
        __syncthreads();
        const int32_t op = ctl.op;
        if (op == OP_END) break;
        if (op == OP_FINAL) {
            const bool zx = ctl.zero_x;
            const double sh = ctl.shift;
            res_for<kResRows>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const int64_t i = row(kc);
                if (i < n) a.x[i] = zx ? 0.0 : (a.proj && i == a.pin) ? a.b[a.pin] : x[k] + sh;
            });
            break;
        }
        if constexpr (MIXED) {
            if (op == OP_REFRESH) {
                // r64 = c - A x at the current iterate (x gathered from s_v)
                res_for<kResRows>([&](auto kc) {
                    const int64_t i = row(kc);
                    if (i < n) s_v[i] = x[decltype(kc)::value];
                });
                __syncthreads();
                double s1 = 0.0, s2 = 0.0;
                res_for<kResRows>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    const int64_t i = row(kc);
                    if (i < n) {
                        const double ri = a.c[i] - rowprod(kc, sv64);
                        a.r[i] = ri;
                        s1 = fma(ri, ri, s1);
                        if (!(a.proj && i == a.pin)) s2 = fma(ri, ri, s2);
                    }
                });
                const double xpin = s_v[a.pin];
                rr = block_sum<kResThreads>(s1, red);
                rrp = block_sum<kResThreads>(s2, red);
                bb = 0.0;
                if (tid == 0) {
                    ctl.st.pending = 0;
                    ctl.st.mode = MODE_REFRESH;
                    ctl.st.updates += 1;
                    ctl.st.xpin = xpin;
                }
                continue;
            }
        }
        // Float64: one pass serves the refresh (r = c - A x, x gathered from
        // s_v) and the A step (p = r + beta p_old, after a restart p = r,
        // into s_v; q = A p; p^T q).  Mixed A step: r = r64 / s after a
        // restart; p = r + beta p_old (normal), r + cref p_old (refresh) or
        // r (first step); q = A p; p^T q.
        const bool refresh = !MIXED && op == OP_REFRESH;
        const bool normal = ctl.normal != 0;
        const double beta = ctl.beta;
        if constexpr (MIXED) {
            const bool use_p = ctl.use_p != 0;
            const float cf = normal ? (float)beta : (float)ctl.cref;
            const double inv_s = ctl.inv_s;
            res_for<kResRows>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const int64_t i = row(kc);
                if (i < n) {
                    if (!normal) r32[k] = (float)(a.r[i] * inv_s);
                    pk[k] = use_p ? fmaf(cf, pk[k], r32[k]) : r32[k];
                    s_p[i] = pk[k];
                }
            });
        } else {
            res_for<kResRows>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const int64_t i = row(kc);
                if (i < n) s_v[i] = refresh ? x[k] : normal ? fma(beta, s_v[i], r64[k]) : r64[k];
            });
        }
        __syncthreads();
        double s1 = 0.0, s2 = 0.0;
        res_for<kResRows>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int64_t i = row(kc);
            if (i < n) {
                const VT prod = rowprod(kc, svp);
                if (refresh) {
                    const double ri = a.c[i] - (double)prod;
                    r64[k] = ri;
                    s1 = fma(ri, ri, s1);
                    if (!(a.proj && i == a.pin)) s2 = fma(ri, ri, s2);
                } else {
                    q[k] = prod;
                    s1 = fma((double)s_p[i], (double)prod, s1);  // p^T q
                }
            }
        });
        if (refresh) {
            const double xpin = s_v[a.pin];
            rr = block_sum<kResThreads>(s1, red);
            rrp = block_sum<kResThreads>(s2, red);
            bb = 0.0;
            if (tid == 0) {
                ctl.st.pending = 0;
                ctl.st.mode = MODE_REFRESH;
                ctl.st.updates += 1;
                ctl.st.xpin = xpin;
            }
            continue;
        }
        const double pq = block_sum<kResThreads>(s1, red);
        // B step: alpha = rho / p^T q; x += (s) alpha p; r -= alpha q; ||r||^2
        if (tid == 0) {
            ctl.st.mode = MODE_NORMAL;
            ctl.st.iters += 1;
            ctl.st.alpha = 0.0;
            const double alpha = ctl.st.rho / pq;
            if (!(pq > 0.0) || !std::isfinite(alpha) || ctl.st.iters == a.break_at) {
                ctl.st.pending = 1;
                ctl.st.reason = R_BREAKDOWN;
                ctl.update = 0;
            } else {
                ctl.update = 1;
                ctl.alpha = alpha;
                ctl.sa = ctl.st.scale * alpha;
            }
        }
        __syncthreads();
        if (ctl.update) {
            const double alpha = ctl.alpha, sa = ctl.sa;
            double s1 = 0.0;
            res_for<kResRows>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const int64_t i = row(kc);
                if (i < n) {
                    if constexpr (MIXED) {
                        x[k] = fma(sa, (double)pk[k], x[k]);
                        r32[k] = fmaf(-(float)alpha, q[k], r32[k]);
                        s1 = fma((double)r32[k], (double)r32[k], s1);
                    } else {
                        x[k] = fma(alpha, s_v[i], x[k]);  // s_v still holds p
                        r64[k] = fma(-alpha, q[k], r64[k]);
                        s1 = fma(r64[k], r64[k], s1);
                    }
                }
            });
            rr = block_sum<kResThreads>(s1, red);
        }
        rrp = bb = 0.0;
    }
    if (tid == 0) a.S[(t + 1) & 1] = ctl.st;
}

// Warm start: partial sums of y^T A y and c^T y for gamma, with y[pin] = 0
// (then y^T A_neu y = y^T A_pin y, and c^T y = b^T y - b_pin * sum of y over
// the pin's neighbours in the projected formulation).
__global__ void __launch_bounds__(kBlock) warm_gamma(SolveArgs a) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    __shared__ double red[kBlock / 64];
    auto yg = [&](int32_t j) -> double { return j == a.pin ? 0.0 : a.y[j]; };
    double yay = 0.0, by = 0.0;
    csr_sweep<float>(a.rp, a.col, a.v32, a.n, s_col, s_val, [&](int64_t i, int rs, int re) {
        const double ay = row_product<double>(s_col, s_val, rs, re, yg);
        const double yi = yg((int32_t)i);
        yay = fma(yi, ay, yay);
        const double ci = (a.proj && is_pin_nb(a, i)) ? a.b[i] - a.b[a.pin] : a.b[i];
        by = fma(ci, yi, by);
    });
    yay = block_sum(yay, red);
    by = block_sum(by, red);
    if (threadIdx.x == 0) {
        a.partG1[blockIdx.x] = yay;
        a.partG2[blockIdx.x] = by;
    }
}

// Stopping margin (see kRoughRq): partial sums of b^T A b (the pinned
// matrix) and b^T b.
__global__ void __launch_bounds__(kBlock) rhs_rayleigh(SolveArgs a) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    __shared__ double red[kBlock / 64];
    auto bg = [&](int32_t j) -> double { return a.b[j]; };
    double bab = 0.0, bb = 0.0;
    csr_sweep<float>(a.rp, a.col, a.v32, a.n, s_col, s_val, [&](int64_t i, int rs, int re) {
        const double bi = a.b[i];
        bab = fma(bi, row_product<double>(s_col, s_val, rs, re, bg), bab);
        bb = fma(bi, bi, bb);
    });
    bab = block_sum(bab, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        a.partR[blockIdx.x] = bab;
        a.partRb[blockIdx.x] = bb;
    }
}

// One workgroup: tolv = [tol * margin, margin]; margin = the caller's when
// given (> 0), else 0.05 for the mixed path when b^T A b / b^T b > kRoughRq
// (count > 0: the partial sums of rhs_rayleigh), else 1.
__global__ void __launch_bounds__(kBlock) stop_tol(SolveArgs a, double fixed, int mixed, int count) {
    __shared__ double red[kBlock / 64];
    double m = 1.0;
    if (fixed > 0.0) {
        m = fixed < 1.0 ? fixed : 1.0;
    } else if (mixed) {
        const double bab = reduce_partials(a.partR, count, red);
        const double bb = reduce_partials(a.partRb, count, red);
        m = (bb > 0.0 && bab > kRoughRq * bb) ? kMixedStopMargin : 1.0;
    }
    if (threadIdx.x == 0) {
        a.tolv[0] = a.tol * m;
        a.tolv[1] = m;
    }
}

// Launch the two kernels above for a solve whose natural-order arguments are
// in g (rp, col, v32, b, n, partR, partRb, tolv, tol, Gf).
static void launch_stop_tol(const SolveArgs &g, const cfd_solve_opts &opts, bool mixed, hipStream_t s) {
    const bool rq = opts.stop_margin <= 0.0 && mixed;
    if (rq) hipLaunchKernelGGL(rhs_rayleigh, dim3(g.Gf), dim3(kBlock), 0, s, g);
    hipLaunchKernelGGL(stop_tol, dim3(1), dim3(kBlock), 0, s, g, opts.stop_margin, mixed ? 1 : 0, rq ? g.Gf : 0);
}

// Partial sums of b (projected formulation: sum of b for c_pin).
__global__ void __launch_bounds__(kBlock) rhs_sum(SolveArgs a) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) s += a.b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) a.partS[blockIdx.x] = s;
}

int net_predict(cfd_net_t net, const cfd_grid *grid, const double *b, double *y, hipStream_t s);

// ---------------------------------------------------------------- host driver

// Workgroups per CU that can be resident at once for a kernel, capped at 8.
// The SpMV-shaped kernels use a static, XCD-contiguous tile schedule, so
// every workgroup must be resident: a queued one would run its whole tile
// range after the others finished.
template <class K>
static int resident_per_cu(K kernel, int block = kBlock) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess || nb < 1) nb = 1;
    return std::min(nb, 8);
}

// Rows per tile (and threads per workgroup) of the mixed A kernel.  HBM
// streams a workgroup's CSR slab faster the more contiguous bytes it spans;
// at 512 rows (4 workgroups per CU, the same 64 VGPRs per lane as 8 of 256)
// each slab covers about 14 KB of each of the column and value arrays.
constexpr int kA32Rows = 512;

struct Grids {
    int a64, f64, a32, f32;
};

// Workgroups per CU of the float64 A kernel: measured at 256^3 (full solves,
// per-launch time) 0.50 ms at 4 per CU, 0.46 at 5, 0.43 at 6 and 0.62 at 7,
// the most that fit; past 6 the float64 neighbour planes it gathers no
// longer stay in the XCD's L2.
constexpr int kA64PerCu = 6;

static const Grids &solver_grids() {
    static Grids g = [] {
        Grids r;
        r.a64 = std::min(resident_per_cu(cg_a64), kA64PerCu);
        r.f64 = std::min(resident_per_cu(cg_init<false>), resident_per_cu(cg_refresh<false>));
        r.a32 = resident_per_cu(cg_a32<kA32Rows>, kA32Rows);
        r.f32 = std::min(std::min(resident_per_cu(cg_init<true>), resident_per_cu(cg_refresh<true>)),
                         resident_per_cu(warm_gamma));
        return r;
    }();
    return g;
}

static int rb_solve_impl(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts &opts,
                         double *x, cfd_solve_info *info, hipStream_t s);



// Run the persistent driver after cg_init (launch sequence number t) and
// fill info.  The whole solve is one launch, so no per-launch timings.
// Run the resident driver after cg_init and fill info the same way.
static int finish_single_launch(int64_t t, Workspace *w, cfd_solve_info *info, hipStream_t s);

static int resident_run(SolveArgs &a, bool mixed, int64_t t, Workspace *w, cfd_solve_info *info, hipStream_t s) {
    if (mixed) hipLaunchKernelGGL(cg_resident<true>, dim3(1), dim3(kResThreads), 0, s, a, t);
    else hipLaunchKernelGGL(cg_resident<false>, dim3(1), dim3(kResThreads), 0, s, a, t);
    CFD_HIP(hipGetLastError());
    return finish_single_launch(t, w, info, s);
}

static int persist_run(SolveArgs &a, bool mixed, int64_t t, Workspace *w, cfd_solve_info *info, hipStream_t s) {
    void *args[] = {(void *)&a, (void *)&t};
    const void *kern = mixed ? (const void *)cg_persist<true> : (const void *)cg_persist<false>;
    CFD_HIP(hipLaunchCooperativeKernel(kern, dim3(a.Ga), dim3(kBlock), args, 0, s));
    return finish_single_launch(t, w, info, s);
}

static int finish_single_launch(int64_t t, Workspace *w, cfd_solve_info *info, hipStream_t s) {
    CFD_HIP(hipMemcpyAsync(&w->host[0], &w->S[(t + 1) & 1], sizeof(CgState), hipMemcpyDeviceToHost, s));
    CFD_HIP(hipEventRecord(w->ev1, s));
    CFD_HIP(hipEventSynchronize(w->ev1));
    float ms = 0.0f;
    CFD_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
    const CgState fs = w->host[0];
    cfd_solve_info inf{};
    inf.iters = fs.iters;
    inf.updates = fs.updates;
    inf.status = fs.done ? fs.status : CFD_EHIP;
    inf.used_fallback = fs.fallback;
    inf.rel_residual = fs.relres;
    inf.init_residual = fs.init_relres;
    inf.gamma = fs.gamma;
    inf.stop_margin = fs.margin;
    inf.seconds = ms * 1e-3;
    if (info) *info = inf;
    if (inf.status != CFD_OK) {
        const char *what = inf.status == CFD_ENOCONV ? "max_iters reached"
                         : inf.status == CFD_EBREAKDOWN ? "breakdown: p^T A p <= 0"
                         : inf.status == CFD_ENONFINITE ? "non-finite value in the solve"
                         : inf.status == CFD_EHIP ? "single-launch driver: a grid barrier wait timed out"
                                                  : "solver error";
        return fail(inf.status, std::string("cfd_solve: ") + what);
    }
    return CFD_OK;
}

static int solve_impl(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts *o,
                      double *x, cfd_solve_info *info, hipStream_t s) {
    cfd_solve_opts opts{};
    if (o) opts = *o;
    // x is written while b (and x0, unless it is x itself) are still read
    auto overlap = [&](const double *u, const double *v) { return u < v + A->n && v < u + A->n; };
    if (overlap(x, b)) return fail(CFD_EINVAL, "cfd_solve: x must not overlap b");
    if (x0 && x0 != x && overlap(x, x0)) return fail(CFD_EINVAL, "cfd_solve: x0 must be x itself or not overlap it");
    const bool mixed = opts.precision == CFD_PREC_MIXED;
    if (opts.precision != CFD_PREC_FP64 && !mixed) return fail(CFD_EINVAL, "cfd_solve: unknown precision");
    if (A->pin < 0) return fail(CFD_EINVAL, "cfd_solve: the singular Neumann matrix needs a pinned cell");
    if (!(tol >= 0.0)) return fail(CFD_EINVAL, "cfd_solve: tol must be >= 0");
    if (opts.net && x0) return fail(CFD_EINVAL, "cfd_solve: give either x0 or a warm-start network");
    const int max_iters = opts.max_iters > 0 ? opts.max_iters : 100000;
    const double delta = opts.ru_delta > 0.0 ? opts.ru_delta : 0.1;
    const int K = opts.chunk > 0 ? opts.chunk : 16;
    if (opts.formulation != CFD_FORM_PINNED && opts.formulation != CFD_FORM_PROJECTED)
        return fail(CFD_EINVAL, "cfd_solve: unknown formulation");
    const bool proj = opts.formulation == CFD_FORM_PROJECTED;
    if (opts.precond != CFD_PRECOND_NONE && opts.precond != CFD_PRECOND_DIC_RB)
        return fail(CFD_EINVAL, "cfd_solve: unknown preconditioner");
    if (opts.precond == CFD_PRECOND_DIC_RB) return rb_solve_impl(A, b, x0, tol, opts, x, info, s);
    int rc = ensure_workspace(A, !mixed, mixed, opts.net != nullptr, proj);
    if (rc != CFD_OK) return rc;
    Workspace *w = A->ws;

    SolveArgs a{};
    a.n = A->n;
    a.rp = A->rp;
    a.col = A->col;
    a.v32 = A->val32;
    a.tol = tol;
    a.ru_delta = delta;
    a.max_iters = max_iters;
    a.break_at = opts.debug_breakdown_at > 0 ? opts.debug_breakdown_at : -1;
    const Grids &gr = solver_grids();
    a.Ga = mixed ? grid_tiles(A->n, gr.a32, kA32Rows) : grid_tiles(A->n, gr.a64);
    a.Gb = grid_vec(A->n);
    a.Gf = grid_tiles(A->n, mixed ? gr.f32 : std::min(gr.f64, resident_per_cu(warm_gamma)));
    a.pin = A->pin;
    a.proj = proj ? 1 : 0;
    a.nxny = (int64_t)A->nx * A->ny;
    a.nnb = 0;
    {
        const int64_t p = A->pin, nx = A->nx, ny = A->ny, nz = A->nz;
        const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
        const int64_t cand[6] = {k > 0 ? p - nx * ny : -1, j > 0 ? p - nx : -1, i > 0 ? p - 1 : -1,
                                 i < nx - 1 ? p + 1 : -1, j < ny - 1 ? p + nx : -1, k < nz - 1 ? p + nx * ny : -1};
        for (int q = 0; q < 6; ++q)
            if (cand[q] >= 0) a.nb[a.nnb++] = cand[q];
    }
    a.b = b;
    a.c = proj ? w->c : const_cast<double *>(b);
    a.x = x;
    a.x_vec2 = ((uintptr_t)x % 16) == 0 ? 1 : 0;
    a.x0 = x0;
    a.y = nullptr;
    a.r = w->r;
    a.p0 = w->p0;
    a.p1 = w->p1;
    a.q = w->q;
    a.r32 = w->r32;
    for (int k = 0; k < kRing; ++k) a.p32[k] = w->p32[k];
    a.q32 = w->q32;
    const int64_t gm = w->gmax;
    a.partA = w->part;
    a.partB = w->part + gm;
    a.partF = w->part + 2 * gm;
    a.partF2 = w->part + 3 * gm;
    a.partG1 = w->part + 4 * gm;
    a.partG2 = w->part + 5 * gm;
    a.partFp = w->part + 7 * gm;
    a.partS = w->part + 8 * gm;
    a.partR = w->part + 9 * gm;
    a.partRb = w->part + 10 * gm;
    a.tolv = w->tolv;
    a.S = w->S;
    a.bar = w->bar;
    a.spin_limit = opts.barrier_spins > 0 ? opts.barrier_spins : kBarrierSpins;

    // Driver: one cooperative launch for the whole iteration (small grids,
    // where launches set the pace), or one launch per step.
    if (opts.driver != CFD_DRIVER_AUTO && opts.driver != CFD_DRIVER_STEPS && opts.driver != CFD_DRIVER_PERSISTENT &&
        opts.driver != CFD_DRIVER_RESIDENT)
        return fail(CFD_EINVAL, "cfd_solve: unknown driver");
    if (opts.driver == CFD_DRIVER_RESIDENT && A->n > kResMaxRows)
        return fail(CFD_EINVAL, "cfd_solve: the resident driver takes grids of at most " +
                                    std::to_string(kResMaxRows) + " cells");
    const bool resident = opts.driver == CFD_DRIVER_RESIDENT ||
                          (opts.driver == CFD_DRIVER_AUTO && A->n <= kResMaxRows);
    bool persist = !resident && (opts.driver == CFD_DRIVER_PERSISTENT ||
                                 (opts.driver == CFD_DRIVER_AUTO &&
                                  A->n <= (mixed ? kPersistMaxRows : kPersistMaxRows64)));
    if (persist) {
        int coop = 0;
        CFD_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, A->device));
        if (!coop) {
            if (opts.driver == CFD_DRIVER_PERSISTENT)
                return fail(CFD_EINVAL, "cfd_solve: the device does not support cooperative launches");
            persist = false;
        }
    }
    if (persist) {
        // every step on one grid that is resident all at once
        const int G = std::min(kPersistMaxGroups,
                               grid_tiles(A->n, mixed ? resident_per_cu(cg_persist<true>) : resident_per_cu(cg_persist<false>)));
        a.Ga = a.Gb = a.Gf = G;
    }

    CFD_HIP(hipEventRecord(w->ev0, s));
    launch_stop_tol(a, opts, mixed, s);
    if (opts.net) {
        cfd_grid g{A->nx, A->ny, A->nz, A->h};
        rc = net_predict(opts.net, &g, b, w->y, s);
        if (rc != CFD_OK) return rc;
        a.y = w->y;
        hipLaunchKernelGGL(warm_gamma, dim3(a.Gf), dim3(kBlock), 0, s, a);
    }
    if (proj) hipLaunchKernelGGL(rhs_sum, dim3(a.Gb), dim3(kBlock), 0, s, a);
    int64_t t = 0;
    if (mixed) hipLaunchKernelGGL(cg_init<true>, dim3(a.Gf), dim3(kBlock), 0, s, a, t);
    else hipLaunchKernelGGL(cg_init<false>, dim3(a.Gf), dim3(kBlock), 0, s, a, t);
    ++t;
    CFD_HIP(hipGetLastError());
    if (resident) return resident_run(a, mixed, t, w, info, s);
    if (persist) return persist_run(a, mixed, t, w, info, s);

    // Enqueue chunks of K iterations + one refresh kernel; poll the state of
    // the previous chunk while the current one runs.
    const int pool = opts.timing ? 256 : 0;
    while ((int)w->ta.size() < pool) {
        hipEvent_t e0, e1;
        CFD_HIP(hipEventCreate(&e0));
        CFD_HIP(hipEventCreate(&e1));
        w->ta.push_back(e0);
        w->tb.push_back(e1);
    }
    std::vector<char> sampled;
    std::vector<char> live;  // chunk ended with the solve still running
    const int64_t cap = (int64_t)max_iters + 64;  // every chunk iterates at least once until done
    int64_t c = 0;
    bool finished = false;
    CgState final_state{};
    for (;; ++c) {
        if (c > cap) return fail(CFD_EHIP, "cfd_solve: solver control did not terminate");
        bool smp = false;
        for (int i = 0; i < K; ++i) {
            const bool time_it = (i == 1 || K == 1) && c < pool;
            if (time_it) {
                smp = true;
                if (mixed)
                    hipExtLaunchKernelGGL(cg_a32<kA32Rows>, dim3(a.Ga), dim3(kA32Rows), 0, s, w->ta[c], w->tb[c], 0, a,
                                          t);
                else
                    hipExtLaunchKernelGGL(cg_a64, dim3(a.Ga), dim3(kBlock), 0, s, w->ta[c], w->tb[c], 0, a, t);
            } else if (mixed) {
                hipLaunchKernelGGL(cg_a32<kA32Rows>, dim3(a.Ga), dim3(kA32Rows), 0, s, a, t);
            } else {
                hipLaunchKernelGGL(cg_a64, dim3(a.Ga), dim3(kBlock), 0, s, a, t);
            }
            ++t;
            if (mixed) hipLaunchKernelGGL(cg_b<true>, dim3(a.Gb), dim3(kBlock), 0, s, a, t);
            else hipLaunchKernelGGL(cg_b<false>, dim3(a.Gb), dim3(kBlock), 0, s, a, t);
            ++t;
        }
        if (mixed) hipLaunchKernelGGL(cg_refresh<true>, dim3(a.Gf), dim3(kBlock), 0, s, a, t);
        else hipLaunchKernelGGL(cg_refresh<false>, dim3(a.Gf), dim3(kBlock), 0, s, a, t);
        ++t;
        CFD_HIP(hipGetLastError());
        sampled.push_back(smp);
        live.push_back(0);
        const int slot = (int)(c & 1);
        CFD_HIP(hipMemcpyAsync(&w->host[slot], &w->S[t & 1], sizeof(CgState), hipMemcpyDeviceToHost, s));
        CFD_HIP(hipEventRecord(w->evc[slot], s));
        if (c >= 1) {
            const int prev = (int)((c - 1) & 1);
            CFD_HIP(hipEventSynchronize(w->evc[prev]));
            const CgState ps = w->host[prev];
            live[c - 1] = !ps.done;
            if (ps.done) {
                finished = true;
                break;
            }
        }
    }
    (void)finished;
    CFD_HIP(hipEventSynchronize(w->evc[c & 1]));
    final_state = w->host[c & 1];
    live[c] = !final_state.done;
    CFD_HIP(hipEventRecord(w->ev1, s));
    CFD_HIP(hipEventSynchronize(w->ev1));
    float ms = 0.0f;
    CFD_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));

    cfd_solve_info inf{};
    inf.iters = final_state.iters;
    inf.updates = final_state.updates;
    inf.status = final_state.done ? final_state.status : CFD_EHIP;
    inf.used_fallback = final_state.fallback;
    inf.rel_residual = final_state.relres;
    inf.init_residual = final_state.init_relres;
    inf.gamma = final_state.gamma;
    inf.stop_margin = final_state.margin;
    inf.seconds = ms * 1e-3;
    double tot = 0.0;
    int ns = 0;
    for (int64_t i = 0; i < (int64_t)sampled.size() && i < pool; ++i) {
        if (!sampled[i] || !live[i]) continue;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, w->ta[i], w->tb[i]) == hipSuccess) {
            tot += e;
            ++ns;
        }
    }
    inf.spmv_ms = ns ? tot / ns : 0.0;
    inf.spmv_samples = ns;
    if (info) *info = inf;
    if (!final_state.done) return fail(CFD_EHIP, "cfd_solve: solver did not finish");
    if (inf.status != CFD_OK) {
        const char *what = inf.status == CFD_ENOCONV ? "max_iters reached"
                         : inf.status == CFD_EBREAKDOWN ? "breakdown: p^T A p <= 0"
                         : inf.status == CFD_ENONFINITE ? "non-finite value in the solve"
                                                        : "solver error";
        return fail(inf.status, std::string("cfd_solve: ") + what);
    }
    return CFD_OK;
}

// ================================================================ preconditioned solve
//
// The paper's PCG uses a diagonal-based incomplete Cholesky preconditioner
// (Sec. 3.1): M = (D + L) D^{-1} (D + U), L and U the entries of A before and
// after each row in the elimination order, D chosen so that diag(M) =
// diag(A).  Its recurrences follow that order, which keeps the paper's
// version serial (Sec. 3.3).  Here the order is red-black (cells with i+j+k
// even first).  A 7-point cell only neighbours cells of the other colour, so
// the red block of A is diagonal: the red pivots are a_rr and the black ones
// the diagonal of the Schur complement S = D_b - B^T D_r^{-1} B.  In this
// order M^{-1} A is similar to diag(I, D_S^{-1/2} S D_S^{-1/2}) (Eisenstat's
// form of the preconditioned operator), so PCG with M is Jacobi-
// preconditioned CG with S on the black unknowns, the red ones following
// from x_r = D_r^{-1} (b_r - B x_b).  That is what runs: per iteration one
// sweep over the red rows (y = D_r^{-1} B p) and one over the black rows
// (q = D_b p - B^T y), each over half of the matrix, on black-length
// vectors.  With x_r recovered the red rows of b - A x vanish, so the full
// residual is the Schur residual and the stopping test is unchanged.
//
// The matrix is stored once more in red-black order (cfd_csr handle, built
// on the first preconditioned solve of each formulation): perm/iperm map
// natural <-> red-black indices, red rows first, and each row holds its
// diagonal entry first.

struct RbMatrix {
    int64_t n = 0, nr = 0, nnz = 0;
    int gmax = 0;
    int32_t *perm = nullptr, *iperm = nullptr;  // natural -> red-black, and back
    int32_t *rp = nullptr, *col = nullptr;      // CSR in red-black order, diagonal first
    float *v32 = nullptr;                       // values: small integers, exact in float32
    double *d64 = nullptr;                      // diagonal of S (black rows)
    float *d32 = nullptr;
    // solve buffers; black length unless noted
    double *bp = nullptr;                       // right-hand side in red-black order (n)
    double *bS = nullptr, *xb = nullptr, *r64 = nullptr;
    double *y64 = nullptr, *yb = nullptr;       // red length
    double *z64 = nullptr, *p64[2] = {nullptr, nullptr}, *q64 = nullptr;
    float *z32 = nullptr, *q32 = nullptr, *y32 = nullptr;  // y32: red length
    float *ring32 = nullptr;                    // mixed: kRing directions, nb_pad apart
    int64_t nb_pad = 0;
    double *part = nullptr;                     // 7 * gmax partial sums
    struct RbState *S = nullptr, *host = nullptr;
};

// Control state of the preconditioned solve: the CG state (same fields and
// meaning; kept in its own buffers).
struct RbState {
    CgState cg;
};

// The red-black solver's state staged in LDS, as CG_STATE does.
#define RB_STATE(t)                                \
    __shared__ RbState s_st;                       \
    if (threadIdx.x == 0) s_st = a.S[(t) & 1];     \
    __syncthreads();                               \
    const RbState &st = s_st

void rb_free(RbMatrix *m) {
    if (!m) return;
    void *pp[] = {m->perm, m->iperm, m->rp, m->col, m->v32, m->d64, m->d32, m->bp, m->bS, m->xb,
                  m->r64, m->y64, m->yb, m->z64, m->p64[0], m->p64[1], m->q64, m->z32, m->ring32,
                  m->q32, m->y32, m->part, m->S};
    for (void *p : pp) if (p) (void)hipFree(p);
    if (m->host) (void)hipHostFree(m->host);
    delete m;
}

// Matrix entries of row p (cell m) in red-black order: the diagonal, then
// the in-domain neighbours in the order -z, -y, -x, +x, +y, +z.  pin >= 0:
// the pinned matrix (unit row at pin, pin column dropped); pin < 0: the
// singular Neumann matrix.
__global__ void __launch_bounds__(kBlock) rb_fill(int64_t n, int nx, int ny, int nz, int64_t pin,
                                                  const int32_t *perm, const int32_t *iperm, const int32_t *rp,
                                                  int32_t *col, float *v32) {
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        const int64_t m = iperm[p];
        int64_t e = rp[p];
        if (m == pin) {
            col[e] = (int32_t)p;
            v32[e] = 1.0f;
            continue;
        }
        const int64_t nxny = (int64_t)nx * ny;
        const int i = (int)(m % nx), j = (int)((m / nx) % ny), k = (int)(m / nxny);
        const int64_t cand[6] = {k > 0 ? m - nxny : -1, j > 0 ? m - nx : -1, i > 0 ? m - 1 : -1,
                                 i < nx - 1 ? m + 1 : -1, j < ny - 1 ? m + nx : -1, k < nz - 1 ? m + nxny : -1};
        int deg = 0;
        for (int q = 0; q < 6; ++q) deg += cand[q] >= 0;
        col[e] = (int32_t)p;
        v32[e] = (float)deg;
        ++e;
        for (int q = 0; q < 6; ++q) {
            if (cand[q] < 0 || cand[q] == pin) continue;
            col[e] = perm[cand[q]];
            v32[e] = -1.0f;
            ++e;
        }
    }
}

// Diagonal of the Schur complement for the black rows p in [nr, n):
// a_pp - sum over the row's (red) neighbours j of a_pj^2 / a_jj.  In the
// singular Neumann matrix of a grid only 2 or 3 cells long in a single
// direction, a black cell between two end cells has a vanishing Schur row
// (S is positive semidefinite, so a zero diagonal means a zero row); its
// Jacobi scale is then 1, which leaves that unknown at its initial value.
__global__ void __launch_bounds__(kBlock) rb_schur_diag(int64_t n, int64_t nr, const int32_t *rp, const int32_t *col,
                                                        const float *v32, double *d64, float *d32) {
    for (int64_t p = nr + (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n; p += (int64_t)gridDim.x * kBlock) {
        double d = (double)v32[rp[p]];
        for (int32_t e = rp[p] + 1; e < rp[p + 1]; ++e) {
            const double v = (double)v32[e];
            d -= v * v / (double)v32[rp[col[e]]];
        }
        if (!(d > 0.0)) d = 1.0;
        d64[p - nr] = d;
        d32[p - nr] = (float)d;
    }
}

// Build the red-black matrix of A (proj: the Neumann matrix, else the pinned
// one).  The permutation and the row pointers are computed on the host (one
// pass over the cells), the entries on the device.
static int rb_build(cfd_csr_t A, bool proj, int gmax, hipStream_t s, RbMatrix **out) {
    const int nx = A->nx, ny = A->ny, nz = A->nz;
    const int64_t n = A->n, nxny = (int64_t)nx * ny;
    const int64_t pin = proj ? -1 : A->pin;
    std::vector<int32_t> perm(n), iperm(n), rp(n + 1);
    int64_t nr = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) nr += ((i + j + k) & 1) == 0;
    {
        int64_t rc = 0, bc = nr, m = 0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i, ++m) {
                    const int64_t p = ((i + j + k) & 1) == 0 ? rc++ : bc++;
                    perm[m] = (int32_t)p;
                    iperm[p] = (int32_t)m;
                }
    }
    int64_t e = 0;
    rp[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int64_t m = iperm[p];
        int64_t len;
        if (m == pin) {
            len = 1;
        } else {
            const int i = (int)(m % nx), j = (int)((m / nx) % ny), k = (int)(m / nxny);
            const int64_t cand[6] = {k > 0 ? m - nxny : -1, j > 0 ? m - nx : -1, i > 0 ? m - 1 : -1,
                                     i < nx - 1 ? m + 1 : -1, j < ny - 1 ? m + nx : -1, k < nz - 1 ? m + nxny : -1};
            len = 1;
            for (int q = 0; q < 6; ++q) len += cand[q] >= 0 && cand[q] != pin;
        }
        e += len;
        if (e > (int64_t)INT32_MAX - kPad) return fail(CFD_EINVAL, "cfd_solve: red-black matrix exceeds int32 indexing");
        rp[p + 1] = (int32_t)e;
    }
    RbMatrix *M = new RbMatrix();
    M->n = n;
    M->nr = nr;
    M->nnz = e;
    M->gmax = gmax;
    hipError_t h = hipSuccess;
    if (h == hipSuccess) h = alloc(&M->perm, n);
    if (h == hipSuccess) h = alloc(&M->iperm, n);
    if (h == hipSuccess) h = alloc(&M->rp, n + 1);
    if (h == hipSuccess) h = alloc(&M->col, e + kPad);
    if (h == hipSuccess) h = alloc(&M->v32, e + kPad);
    if (h == hipSuccess) h = alloc(&M->d64, n - nr);
    if (h == hipSuccess) h = alloc(&M->d32, n - nr);
    if (h == hipSuccess) h = hipMemcpy(M->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
    if (h == hipSuccess) h = hipMemcpy(M->iperm, iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
    if (h == hipSuccess) h = hipMemcpy(M->rp, rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice);
    if (h == hipSuccess) h = hipMemsetAsync(M->col + e, 0, sizeof(int32_t) * kPad, s);
    if (h == hipSuccess) h = hipMemsetAsync(M->v32 + e, 0, sizeof(float) * kPad, s);
    if (h != hipSuccess) {
        rb_free(M);
        return hip_fail(h, "cfd_solve: red-black matrix");
    }
    const unsigned g = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(rb_fill, dim3(g), dim3(kBlock), 0, s, n, nx, ny, nz, pin, (const int32_t *)M->perm,
                       (const int32_t *)M->iperm, (const int32_t *)M->rp, M->col, M->v32);
    hipLaunchKernelGGL(rb_schur_diag, dim3(g), dim3(kBlock), 0, s, n, nr, (const int32_t *)M->rp,
                       (const int32_t *)M->col, (const float *)M->v32, M->d64, M->d32);
    h = hipGetLastError();
    if (h != hipSuccess) {
        rb_free(M);
        return hip_fail(h, "cfd_solve: red-black matrix");
    }
    *out = M;
    return CFD_OK;
}

static int rb_buffers(RbMatrix *M, bool mixed) {
    const int64_t nb = M->n - M->nr, nr = M->nr;
    hipError_t h = hipSuccess;
    if (h == hipSuccess) h = alloc(&M->bp, M->n);
    if (h == hipSuccess) h = alloc(&M->bS, nb);
    if (h == hipSuccess) h = alloc(&M->xb, nb);
    if (h == hipSuccess) h = alloc(&M->r64, nb);
    if (h == hipSuccess) h = alloc(&M->y64, nr);
    if (h == hipSuccess) h = alloc(&M->yb, nr);
    if (h == hipSuccess) h = alloc(&M->part, (int64_t)M->gmax * 7);
    if (h == hipSuccess) h = alloc(&M->S, 2);
    if (h == hipSuccess && !M->host) h = hipHostMalloc((void **)&M->host, sizeof(RbState) * 2, 0);
    if (mixed) {
        if (h == hipSuccess) h = alloc(&M->z32, nb);
        M->nb_pad = (nb + 63) / 64 * 64;
        if (h == hipSuccess) h = alloc(&M->ring32, kRing * M->nb_pad);
        if (h == hipSuccess) h = alloc(&M->q32, nb);
        if (h == hipSuccess) h = alloc(&M->y32, nr);
    } else {
        if (h == hipSuccess) h = alloc(&M->z64, nb);
        if (h == hipSuccess) h = alloc(&M->p64[0], nb);
        if (h == hipSuccess) h = alloc(&M->p64[1], nb);
        if (h == hipSuccess) h = alloc(&M->q64, nb);
    }
    if (h != hipSuccess) return hip_fail(h, "cfd_solve: red-black solver buffers");
    return CFD_OK;
}

struct RbArgs {
    int64_t n, nr, nb;
    const int32_t *rp, *col;
    const float *v32;       // matrix values (small integers, exact in float32)
    const double *d64;
    const float *d32;
    const int32_t *perm, *iperm;
    double ru_delta;
    const double *tolv;     // [effective tolerance, stopping margin] (see SolveArgs)
    int32_t max_iters;
    int32_t break_at;       // testing: as in SolveArgs
    int32_t G1, G2, Gv;     // red and black sweeps of the iteration, black vector kernels
    int32_t Gf1, Gf2;       // red and black sweeps of the initial residual and the refresh
    int32_t Gw, Gs;         // partial counts of the warm-start and right-hand-side sums
    int64_t pin;
    int32_t proj, nnb;
    int64_t nbr[6];         // natural indices of the pin's neighbours
    const double *b;
    double *x;
    const double *x0, *y;   // initial guess or warm-start prediction (NULL = none)
    double *bp, *bS, *xb, *r64, *y64, *yb;
    double *z64, *p64a, *p64b, *q64;
    float *z32, *q32, *y32;
    float *ring32;          // mixed: ring of kRing direction buffers, nb_pad apart
    int64_t nb_pad;
    double *partA, *partB, *partB2, *partF, *partFp, *partFz, *partF2;
    const double *partG1, *partG2, *partS;
    RbState *S;
};

// Mixed path: direction buffer k of the ring.
__device__ inline float *rb_ring(const RbArgs &a, int k) { return a.ring32 + (int64_t)k * a.nb_pad; }

// Direction buffers: mixed, ring slots (the current one, the next one);
// float64, the two buffers.
template <bool MIXED>
__device__ inline void *rb_dir(const RbArgs &a, int pcur, bool next) {
    if (MIXED) return rb_ring(a, next ? (pcur + 1) % kRing : pcur);
    return (next ? !pcur : pcur) ? a.p64b : a.p64a;
}

__device__ inline bool rb_is_pin_nb(const RbArgs &a, int64_t i) {
    for (int q = 0; q < a.nnb; ++q)
        if (i == a.nbr[q]) return true;
    return false;
}

// Off-diagonal part of a red-black row over the staged slab: the diagonal is
// entry rs, the neighbours rs+1 .. re-1.  As in row_product, the gathers of
// the 6 possible neighbours are issued together (slots past the row's end
// gather the first neighbour again and are left out of the sum), so g is
// only ever called with an off-diagonal column; a row without neighbours
// (a pinned cell) gives 0.
template <class Acc, class VT, class G>
__device__ inline Acc rb_offdiag(const int32_t *s_col, const VT *s_val, int rs, int re, G &&g) {
    Acc acc = Acc(0);
    if (re - rs < 2) return acc;
    Acc v[kMaxRowNnz - 1], w[kMaxRowNnz - 1];
#pragma unroll
    for (int k = 1; k < kMaxRowNnz; ++k) {
        const int e = rs + k < re ? rs + k : rs + 1;
        v[k - 1] = Acc(s_val[e]);
        w[k - 1] = g(s_col[e]);
    }
#pragma unroll
    for (int k = 1; k < kMaxRowNnz; ++k) {
        const Acc f = fma(v[k - 1], w[k - 1], acc);
        acc = rs + k < re ? f : acc;
    }
    return acc;
}

// Right-hand side in red-black order (projected: the consistent c) and the
// initial guess's black part; partial sums of ||b||^2.
__global__ void __launch_bounds__(kBlock) rb_rhs(RbArgs a) {
    __shared__ double red[kBlock / 64];
    double gamma = 0.0;
    if (a.y) {
        const double yay = reduce_partials(a.partG1, a.Gw, red);
        const double by = reduce_partials(a.partG2, a.Gw, red);
        gamma = by / yay;
        if (!(yay > 0.0) || !std::isfinite(gamma)) gamma = 0.0;
    }
    const double bpin = a.b[a.pin];
    double cpin = bpin;
    if (a.proj) {
        const double sb = reduce_partials(a.partS, a.Gs, red);
        cpin = -(sb - bpin) + (double)a.nnb * bpin;
    }
    double bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const double bi = a.b[i];
        double ci = bi;
        if (a.proj) ci = (i == a.pin) ? cpin : (rb_is_pin_nb(a, i) ? bi - bpin : bi);
        const int64_t p = a.perm[i];
        a.bp[p] = ci;
        bb = fma(bi, bi, bb);
        if (p >= a.nr) {
            double g = 0.0;
            if (a.y) g = (i == a.pin) ? 0.0 : gamma * a.y[i];
            else if (a.x0) g = a.x0[i];
            a.xb[p - a.nr] = g;
        }
    }
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) a.partF2[blockIdx.x] = bb;
}

// Red rows of the initial residual: y = D_r^{-1} (b_r - B x0_b) and
// yb = D_r^{-1} b_r (for the Schur right-hand side).
__global__ void __launch_bounds__(kBlock) rb_init_red(RbArgs a) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    auto none = [](int64_t) { return 0; };
    csr_stream_rows<float>(a.rp, a.col, a.v32, 0, a.nr, s_col, s_val, none, [&](int64_t p, int rs, int re, int) {
        const double acc = rb_offdiag<double>(s_col, s_val, rs, re, [&](int32_t c) { return a.xb[c - a.nr]; });
        const double bi = a.bp[p], di = (double)s_val[rs];
        a.y64[p] = (bi - acc) / di;
        a.yb[p] = bi / di;
    });
}

// Black rows: b_S = b_b - B^T yb and r = b_S - S x0 = b_b - D_b x0 - B^T y;
// partial sums of ||r||^2 (all rows, and without the pin row), r^T D_S^{-1} r;
// fresh control state.
__global__ void __launch_bounds__(kBlock) rb_init_black(RbArgs a, int64_t t) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    __shared__ double red[kBlock / 64];
    double gamma = 0.0;
    int fallback = 0;
    if (a.y) {  // the warm-start scale, as rb_rhs applied it (reduced by every thread)
        const double yay = reduce_partials(a.partG1, a.Gw, red);
        const double by = reduce_partials(a.partG2, a.Gw, red);
        gamma = by / yay;
        if (!(yay > 0.0) || !std::isfinite(gamma)) {
            gamma = 0.0;
            fallback = 1;
        }
    }
    double rr = 0.0, rp_ = 0.0, rz = 0.0;
    const int64_t pin_p = a.perm[a.pin];
    auto none = [](int64_t) { return 0; };
    csr_stream_rows<float>(a.rp, a.col, a.v32, a.nr, a.n, s_col, s_val, none, [&](int64_t p, int rs, int re, int) {
        const double sy = rb_offdiag<double>(s_col, s_val, rs, re, [&](int32_t c) { return a.y64[c]; });
        const double syb = rb_offdiag<double>(s_col, s_val, rs, re, [&](int32_t c) { return a.yb[c]; });
        const int64_t k = p - a.nr;
        const double bi = a.bp[p];
        a.bS[k] = bi - syb;
        const double ri = bi - (double)s_val[rs] * a.xb[k] - sy;
        a.r64[k] = ri;
        rr = fma(ri, ri, rr);
        if (!(a.proj && p == pin_p)) rp_ = fma(ri, ri, rp_);
        rz = fma(ri, ri / a.d64[k], rz);
    });
    rr = block_sum(rr, red);
    rp_ = block_sum(rp_, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        a.partF[blockIdx.x] = rr;
        a.partFp[blockIdx.x] = rp_;
        a.partFz[blockIdx.x] = rz;
    }
    if (lead()) {
        RbState ns{};
        ns.cg.mode = MODE_INIT;
        ns.cg.scale = 1.0;
        ns.cg.gamma = gamma;
        ns.cg.fallback = fallback;
        a.S[(t + 1) & 1] = ns;
    }
}

// Decision at the start of each red sweep (identical in every workgroup).
// Normal mode: from the vector kernel's partial sums of ||r||^2 (r = D_S z)
// and r^T z.  Restart (init or refresh): from the true residual's sums.
// Mixed precision keeps z normalised by the scale s of the last true
// residual: z_true = s z, and rho = r^T z in those units.
template <bool MIXED>
__device__ inline Decision rb_decide(const RbArgs &a, const CgState &st, double *red) {
    Decision D;
    D.stop = false;
    D.zero_x = false;
    D.fold = false;
    D.beta = 0.0;
    D.cref = 0.0;
    D.inv_s = 1.0;
    D.shift = 0.0;
    CgState ns = st;
    if (st.mode == MODE_NORMAL) {
        const double rr = reduce_partials(a.partB, a.Gv, red);
        const double rz = reduce_partials(a.partB2, a.Gv, red);
        const double nr = sqrt(rr);
        int reason = R_NONE;
        if (!std::isfinite(rr) || !std::isfinite(rz)) reason = R_NONFINITE;
        else if (nr * st.scale <= a.tolv[0] * st.bnorm) reason = R_CONVERGED;
        else if (MIXED && nr < a.ru_delta * st.rmax) reason = R_REFRESH;
        else if (st.iters >= a.max_iters) reason = R_NOCONV;
        if (reason != R_NONE) {
            ns.pending = 1;
            ns.reason = reason;
            ns.rho_new = rr;
            D.stop = true;
        } else {
            D.beta = rz / st.rho;
            ns.rho = rz;
            ns.rmax = std::max(st.rmax, nr);
        }
    } else {
        const double rr = reduce_partials(a.partF, a.Gf2, red);
        const double rrp = reduce_partials(a.partFp, a.Gf2, red);
        const double rz = reduce_partials(a.partFz, a.Gf2, red);
        if (st.mode == MODE_INIT) {
            ns.bnorm = sqrt(reduce_partials(a.partF2, a.Gv, red));
            ns.margin = a.tolv[1];
        }
        const double tr = sqrt(rr), trp = sqrt(rrp);
        const double bn = ns.bnorm;
        ns.reason = R_NONE;
        ns.alpha = 0.0;
        if (!std::isfinite(bn) || !std::isfinite(rr) || !std::isfinite(rrp) || !std::isfinite(rz)) {
            ns.done = 1;
            ns.status = CFD_ENONFINITE;
            ns.relres = NAN;
        } else if (bn == 0.0) {
            ns.done = 1;
            ns.status = CFD_OK;
            ns.relres = 0.0;
            D.zero_x = true;
        } else {
            ns.relres = trp / bn;
            if (st.mode == MODE_INIT) ns.init_relres = ns.relres;
            if (trp <= a.tolv[0] * bn) {
                ns.done = 1;
                ns.status = CFD_OK;
            } else if (st.reason == R_NOCONV || st.iters >= a.max_iters) {
                ns.done = 1;
                ns.status = CFD_ENOCONV;
            } else if (st.reason == R_BREAKDOWN) {
                ns.done = 1;
                ns.status = CFD_EBREAKDOWN;
            } else if (st.reason == R_NONFINITE) {
                ns.done = 1;
                ns.status = CFD_ENONFINITE;
            }
        }
        if (ns.done) {
            D.stop = true;
        } else if (MIXED) {
            // restart from z = r / (s D_S) with s = ||r||, keeping the old
            // direction: beta_true = rz / (s_old^2 rho_old), rescaled by
            // s_old / s into the new units
            D.inv_s = 1.0 / tr;
            D.cref = (st.mode == MODE_INIT) ? 0.0 : rz / (st.scale * st.rho * tr);
            ns.scale = tr;
            ns.rho = rz / (tr * tr);
            ns.rmax = 1.0;
        } else {
            D.beta = 0.0;  // float64: restart from z = D_S^{-1} r
            ns.rho = rz;
        }
    }
    D.ns = ns;
    return D;
}

// x in natural order when the solve ends: black cells from x_b, red cells
// x_r = D_r^{-1} (b_r - B x_b); projected formulation: shifted so that
// x_pin = b_pin.
__device__ inline double rb_x_at(const RbArgs &a, int64_t p) {
    if (p >= a.nr) return a.xb[p - a.nr];
    double acc = 0.0;
    for (int32_t e = a.rp[p] + 1; e < a.rp[p + 1]; ++e) acc = fma((double)a.v32[e], a.xb[a.col[e] - a.nr], acc);
    return (a.bp[p] - acc) / (double)a.v32[a.rp[p]];
}

__device__ inline void rb_write_x(const RbArgs &a, bool zero_x) {
    const double shift = (a.proj && !zero_x) ? a.b[a.pin] - rb_x_at(a, a.perm[a.pin]) : 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * kBlock) {
        const int64_t m = a.iperm[p];
        a.x[m] = zero_x ? 0.0 : (a.proj && m == a.pin) ? a.b[a.pin] : rb_x_at(a, p) + shift;
    }
}

// The direction at black index k: p = z + cf p_old, with z = z32/z64 in normal
// mode and z = r64 / (s d) (mixed) or r64 / d (float64) in a restart.
template <bool MIXED>
struct RbDir {
    typedef typename std::conditional<MIXED, float, double>::type VT;
    const RbArgs &a;
    const VT *pold;
    VT cf;
    double inv_s;
    bool normal, use_p;
    __device__ inline VT z(int64_t k) const {
        if (normal) return MIXED ? (VT)a.z32[k] : (VT)a.z64[k];
        return MIXED ? (VT)(a.r64[k] * inv_s / a.d64[k]) : (VT)(a.r64[k] / a.d64[k]);
    }
    __device__ inline VT w(int64_t k) const {
        const VT zk = z(k);
        return use_p ? (VT)fma(cf, pold[k], zk) : zk;
    }
};

// Red sweep: y = D_r^{-1} B p, with p = z + cf p_old formed on the fly at the
// black neighbours.  Red row p also forms and stores the new direction of
// black cell p (the two are neighbours in space: both sit near natural index
// 2p), loading that cell's z and p_old a tile ahead; those loads bring in the
// lines the row's own gathers need.  In a restart it stores the new z too.
// GENERAL = false is the normal-mode-only instance, without the restart's
// float64 gathers: only the first launch after a refresh kernel can see a
// restart, so the host launches the general instance there.
template <bool MIXED, bool GENERAL>
__global__ void __launch_bounds__(kBlock) rb_k1(RbArgs a, int64_t t) {
    typedef typename std::conditional<MIXED, float, double>::type VT;
    typedef typename std::conditional<MIXED, f32x2, f64x2>::type VT2;
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];  // exact values (small integers)
    __shared__ double red[kBlock / 64];
    const RbState st = a.S[t & 1];
    RbState *out = &a.S[(t + 1) & 1];
    if (st.cg.done || st.cg.pending) {
        if (lead()) *out = st;
        return;
    }
    if (!GENERAL && st.cg.mode != MODE_NORMAL) {  // launch order broken: end the solve
        if (lead()) {
            RbState ns = st;
            ns.cg.done = 1;
            ns.cg.status = CFD_EHIP;
            *out = ns;
        }
        return;
    }
    const Decision D = rb_decide<MIXED>(a, st.cg, red);
    if (D.stop) {
        if (GENERAL && D.ns.done) rb_write_x(a, D.zero_x);
        if (lead()) {
            RbState ns = st;
            ns.cg = D.ns;
            *out = ns;
        }
        return;
    }
    const bool normal = !GENERAL || st.cg.mode == MODE_NORMAL;
    const VT cf = (VT)(normal ? D.beta : (MIXED ? D.cref : 0.0));
    if (lead()) {
        RbState ns = st;
        ns.cg = D.ns;
        *out = ns;
    }
    const VT *pold = (const VT *)rb_dir<MIXED>(a, st.cg.pcur, false);
    VT *pnew = (VT *)rb_dir<MIXED>(a, st.cg.pcur, true);
    VT *z = MIXED ? (VT *)a.z32 : (VT *)a.z64;
    const RbDir<MIXED> dir{a, pold, cf, D.inv_s, normal, normal || (MIXED && st.cg.mode == MODE_REFRESH)};
    VT *y = MIXED ? (VT *)a.y32 : (VT *)a.y64;
    // black cell k = p: its z and p_old, a tile ahead
    auto own = [&](int64_t k) -> VT2 {
        VT2 o;
        o.x = k < a.nb ? dir.z(k) : VT(0);
        o.y = (k < a.nb && dir.use_p) ? pold[k] : VT(0);
        return o;
    };
    // float64: the tile's black directions (black cell p of red row p) go to
    // LDS with the slab; black neighbours inside the tile's range come from
    // there (the same value dir.w forms).  FP64 DIC per iteration 64^3 38.1
    // -> 26.1 us, 256^3 403.9 -> 393.3; the float32 sweep measured slower with
    // it (256^3 301.8 -> 334.8 us), so it gathers every neighbour.
    __shared__ VT s_w[MIXED ? 1 : kBlock];
    int64_t w0 = 0;
    int wn = 0;
    auto stage = [&](int64_t r0, int nr, const VT2 &o) {
        if constexpr (!MIXED) {
            w0 = r0;
            wn = (int)(a.nb - r0 < nr ? (a.nb - r0 > 0 ? a.nb - r0 : 0) : nr);
            if ((int)threadIdx.x < wn) s_w[threadIdx.x] = dir.use_p ? (VT)fma(dir.cf, o.y, o.x) : o.x;
        }
    };
    auto wl = [&](int32_t c) -> VT {
        const int64_t k = (int64_t)c - a.nr;
        if constexpr (!MIXED) {
            const uint32_t d = (uint32_t)(k - w0);
            if (d < (uint32_t)wn) return s_w[d];
        }
        return dir.w(k);
    };
    csr_stream_rows_staged<float>(a.rp, a.col, a.v32, 0, a.nr, s_col, s_val, own, stage,
                                  [&](int64_t p, int rs, int re, VT2 o) {
        const VT acc = rb_offdiag<VT>(s_col, s_val, rs, re, wl);
        y[p] = acc / (VT)s_val[rs];
        if (p < a.nb) {
            const VT wk = dir.use_p ? (VT)fma(dir.cf, o.y, o.x) : o.x;
            if (!normal) store_stream(z + p, o.x);
            // the black sweep reads it next: a plain store keeps the float32
            // direction in L2 (1-2 % faster per mixed solve at 256^3); the
            // float64 one is stored non-temporally (1.5 % faster per solve)
            if constexpr (MIXED) pnew[p] = wk;
            else store_stream(pnew + p, wk);
        }
    });
}

// Black sweep: q = D_b p - B^T y with the direction p stored by the red
// sweep; partial sums of p^T q.
template <bool MIXED>
__global__ void __launch_bounds__(kBlock) rb_k2(RbArgs a, int64_t t) {
    typedef typename std::conditional<MIXED, float, double>::type VT;
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];  // exact values (small integers)
    __shared__ double red[kBlock / 64];
    RB_STATE(t);
    RbState *out = &a.S[(t + 1) & 1];
    if (st.cg.done || st.cg.pending) {
        if (lead()) *out = st;
        return;
    }
    const VT *pnew = (const VT *)rb_dir<MIXED>(a, st.cg.pcur, true);
    VT *q = MIXED ? (VT *)a.q32 : (VT *)a.q64;
    const VT *y = MIXED ? (const VT *)a.y32 : (const VT *)a.y64;
    double pq = 0.0;
    auto own = [&](int64_t p) { return pnew[p - a.nr]; };
    csr_stream_rows<float>(a.rp, a.col, a.v32, a.nr, a.n, s_col, s_val, own, [&](int64_t p, int rs, int re, VT wk) {
        const int64_t k = p - a.nr;
        const VT acc = rb_offdiag<VT>(s_col, s_val, rs, re, [&](int32_t c) { return y[c]; });
        const VT qk = fma((VT)s_val[rs], wk, -acc);
        store_stream(q + k, qk);
        pq = fma((double)wk, (double)qk, pq);
    });
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) a.partA[blockIdx.x] = pq;
    if (lead()) {
        RbState ns = st;
        ns.cg.mode = MODE_NORMAL;
        ns.cg.iters = st.cg.iters + 1;
        ns.cg.pcur = MIXED ? (st.cg.pcur + 1) % kRing : 1 - st.cg.pcur;
        *out = ns;
    }
}

// Vector kernel: alpha = rho / p^T q; z -= alpha D_S^{-1} q; partial sums of
// ||D_S z||^2 and z^T D_S z.  x_b += s alpha p in float64: every iteration
// (float64 path), or queued and applied kDefer at a time, oldest first
// (mixed path, as in the unpreconditioned solver).
template <bool MIXED>
__global__ void __launch_bounds__(kBlock) rb_b(RbArgs a, int64_t t) {
    typedef typename std::conditional<MIXED, float, double>::type VT;
    __shared__ double red[kBlock / 64];
    RB_STATE(t);
    RbState *out = &a.S[(t + 1) & 1];
    if (st.cg.done || st.cg.pending) {
        if (lead()) *out = st;
        return;
    }
    const double pq = reduce_partials(a.partA, a.G2, red);
    const double alpha = st.cg.rho / pq;
    if (!(pq > 0.0) || !std::isfinite(alpha) || st.cg.iters == a.break_at) {
        if (lead()) {
            RbState ns = st;
            ns.cg.pending = 1;
            ns.cg.reason = R_BREAKDOWN;
            // mixed: as in cg_b, the newest queued update is the previous
            // direction, so rb_apply must count the queue back from it
            if (MIXED) ns.cg.pcur = (st.cg.pcur - 1 + kRing) % kRing;
            *out = ns;
        }
        return;
    }
    const VT *q = MIXED ? (const VT *)a.q32 : (const VT *)a.q64;
    VT *z = MIXED ? (VT *)a.z32 : (VT *)a.z64;
    const VT *d = MIXED ? (const VT *)a.d32 : (const VT *)a.d64;
    const VT av = (VT)alpha;
    const double sa = st.cg.scale * alpha;
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x, stride = (int64_t)gridDim.x * kBlock;
    if (!MIXED) {
        const double *p = (const double *)rb_dir<false>(a, st.cg.pcur, false);
        for (int64_t k = first; k < a.nb; k += stride) store_stream(a.xb + k, fma(sa, p[k], a.xb[k]));
    } else if (st.cg.npend == kDefer - 1) {
        const float *pe[kDefer];
        double se[kDefer];
#pragma unroll
        for (int e = 0; e < kDefer; ++e) {
            pe[e] = rb_ring(a, (st.cg.pcur - (kDefer - 1 - e) + kRing) % kRing);
            se[e] = e < kDefer - 1 ? st.cg.sa[e] : sa;
        }
        // four black cells per thread and step, then the scalar tail
        const int64_t nv = a.nb / 4;
        f64x2 *x2 = reinterpret_cast<f64x2 *>(a.xb);
        for (int64_t v = first; v < nv; v += stride) {
            f64x2 xa = x2[2 * v], xc = x2[2 * v + 1];
#pragma unroll
            for (int e = 0; e < kDefer; ++e) {
                const f32x4 pv = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(pe[e]) + v);
                if (se[e] != 0.0) {
                    xa.x = fma(se[e], (double)pv.x, xa.x);
                    xa.y = fma(se[e], (double)pv.y, xa.y);
                    xc.x = fma(se[e], (double)pv.z, xc.x);
                    xc.y = fma(se[e], (double)pv.w, xc.y);
                }
            }
            store_stream(x2 + 2 * v, xa);
            store_stream(x2 + 2 * v + 1, xc);
        }
        for (int64_t k = nv * 4 + first; k < a.nb; k += stride) {
            double xk = a.xb[k];
#pragma unroll
            for (int e = 0; e < kDefer; ++e)
                if (se[e] != 0.0) xk = fma(se[e], (double)pe[e][k], xk);
            store_stream(a.xb + k, xk);
        }
    }
    double rr = 0.0, rz = 0.0;
    auto upd = [&](VT dk, VT qk, VT zk0) -> VT {
        const VT zk = fma(-av, qk / dk, zk0);
        const double rk = (double)dk * (double)zk;
        rr = fma(rk, rk, rr);
        rz = fma(rk, (double)zk, rz);
        return zk;
    };
    int64_t tail = 0;
    if (MIXED) {  // four black cells per thread and step (the buffers are 256-byte aligned)
        const int64_t nv = a.nb / 4;
        const f32x4 *d4 = reinterpret_cast<const f32x4 *>(a.d32);
        const f32x4 *q4 = reinterpret_cast<const f32x4 *>(a.q32);
        f32x4 *z4 = reinterpret_cast<f32x4 *>(a.z32);
        for (int64_t v = first; v < nv; v += stride) {
            const f32x4 dv = d4[v], qv = q4[v];
            f32x4 zv = z4[v];
            zv.x = (float)upd(dv.x, qv.x, zv.x);
            zv.y = (float)upd(dv.y, qv.y, zv.y);
            zv.z = (float)upd(dv.z, qv.z, zv.z);
            zv.w = (float)upd(dv.w, qv.w, zv.w);
            store_stream(z4 + v, zv);
        }
        tail = nv * 4;
    }
    for (int64_t k = tail + first; k < a.nb; k += stride) store_stream(z + k, upd(d[k], q[k], z[k]));
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        a.partB[blockIdx.x] = rr;
        a.partB2[blockIdx.x] = rz;
    }
    if (lead()) {
        RbState ns = st;
        ns.cg.alpha = alpha;
        if (MIXED) {
            if (st.cg.npend < kDefer - 1) {
#pragma unroll
                for (int e = 0; e < kDefer - 1; ++e)
                    if (e == st.cg.npend) ns.cg.sa[e] = sa;
                ns.cg.npend = st.cg.npend + 1;
            } else {
                ns.cg.npend = 0;  // applied above
            }
        }
        *out = ns;
    }
}

// Mixed path, before each refresh: when a refresh is pending, apply the
// queued x updates (oldest first) and empty the queue, so the refresh and the
// final x read x_b itself.
__global__ void __launch_bounds__(kBlock) rb_apply(RbArgs a, int64_t t) {
    RB_STATE(t);
    RbState *out = &a.S[(t + 1) & 1];
    if (st.cg.done || !st.cg.pending || st.cg.npend == 0) {
        if (lead()) *out = st;
        return;
    }
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < a.nb; k += (int64_t)gridDim.x * kBlock) {
        double xk = a.xb[k];
        for (int e = 0; e < st.cg.npend; ++e) {
            const int slot = (st.cg.pcur - (st.cg.npend - 1 - e) + kRing) % kRing;
            if (st.cg.sa[e] != 0.0) xk = fma(st.cg.sa[e], (double)rb_ring(a, slot)[k], xk);
        }
        store_stream(a.xb + k, xk);
    }
    if (lead()) {
        RbState ns = st;
        ns.cg.npend = 0;
        *out = ns;
    }
}

// Refresh, red sweep (when a refresh is pending): y64 = D_r^{-1} B x_b.
__global__ void __launch_bounds__(kBlock) rb_f1(RbArgs a, int64_t t) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    RB_STATE(t);
    RbState *out = &a.S[(t + 1) & 1];
    if (lead()) *out = st;
    if (st.cg.done || !st.cg.pending) return;
    auto none = [](int64_t) { return 0; };
    csr_stream_rows<float>(a.rp, a.col, a.v32, 0, a.nr, s_col, s_val, none, [&](int64_t p, int rs, int re, int) {
        const double acc = rb_offdiag<double>(s_col, s_val, rs, re, [&](int32_t c) { return a.xb[c - a.nr]; });
        a.y64[p] = acc / (double)s_val[rs];
    });
}

// Refresh, black sweep: r = b_S - S x_b = b_S - D_b x_b + B^T y64 in float64;
// partial sums of ||r||^2 (all rows, and without the pin row), r^T D_S^{-1} r.
__global__ void __launch_bounds__(kBlock) rb_f2(RbArgs a, int64_t t) {
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    __shared__ double red[kBlock / 64];
    RB_STATE(t);
    RbState *out = &a.S[(t + 1) & 1];
    if (st.cg.done || !st.cg.pending) {
        if (lead()) *out = st;
        return;
    }
    const int64_t pin_p = a.perm[a.pin];
    double rr = 0.0, rp_ = 0.0, rz = 0.0;
    auto none = [](int64_t) { return 0; };
    csr_stream_rows<float>(a.rp, a.col, a.v32, a.nr, a.n, s_col, s_val, none, [&](int64_t p, int rs, int re, int) {
        const double acc = rb_offdiag<double>(s_col, s_val, rs, re, [&](int32_t c) { return a.y64[c]; });
        const int64_t k = p - a.nr;
        const double ri = a.bS[k] - (double)s_val[rs] * a.xb[k] + acc;
        a.r64[k] = ri;
        rr = fma(ri, ri, rr);
        if (!(a.proj && p == pin_p)) rp_ = fma(ri, ri, rp_);
        rz = fma(ri, ri / a.d64[k], rz);
    });
    rr = block_sum(rr, red);
    rp_ = block_sum(rp_, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        a.partF[blockIdx.x] = rr;
        a.partFp[blockIdx.x] = rp_;
        a.partFz[blockIdx.x] = rz;
    }
    if (lead()) {
        RbState ns = st;
        ns.cg.pending = 0;
        ns.cg.mode = MODE_REFRESH;
        ns.cg.updates = st.cg.updates + 1;
        *out = ns;
    }
}

// Workgroups per CU of the red sweep's normal mixed instance: measured at 256^3,
// more resident workgroups make it slower (185 us at 8 per CU against 145 us
// at 7), the gathers of the black vectors thrashing the XCD's L2.
constexpr int kRbRedPerCu = 7;
// Workgroups per CU of both float64 sweeps, measured the same way (FP64 DIC
// solve at 256^3): 372 ms at 5 per CU, 378-380 ms at 6 or 7 (8 for the
// black sweep).
constexpr int kRb64PerCu = 5;

// Host driver of the preconditioned solve (options already validated).
static int rb_solve_impl(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts &opts,
                         double *x, cfd_solve_info *info, hipStream_t s) {
    const bool mixed = opts.precision == CFD_PREC_MIXED;
    const bool proj = opts.formulation == CFD_FORM_PROJECTED;
    const int max_iters = opts.max_iters > 0 ? opts.max_iters : 100000;
    const double delta = opts.ru_delta > 0.0 ? opts.ru_delta : 0.1;
    const int K = opts.chunk > 0 ? opts.chunk : 16;
    int rc = ensure_workspace(A, false, false, opts.net != nullptr, false);
    if (rc != CFD_OK) return rc;
    Workspace *w = A->ws;
    RbMatrix *&M = w->rb[proj ? 1 : 0];
    if (!M) {
        rc = rb_build(A, proj, w->gmax, s, &M);
        if (rc != CFD_OK) return rc;
    }
    rc = rb_buffers(M, mixed);
    if (rc != CFD_OK) return rc;
    const int64_t n = A->n, nr = M->nr, nb = n - nr;

    // the natural-order helpers (warm-start scale, right-hand-side sum)
    SolveArgs g{};
    g.n = n;
    g.rp = A->rp;
    g.col = A->col;
    g.v32 = A->val32;
    g.pin = A->pin;
    g.proj = proj ? 1 : 0;
    g.nxny = (int64_t)A->nx * A->ny;
    {
        const int64_t p = A->pin, nx = A->nx, ny = A->ny, nz = A->nz;
        const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
        const int64_t cand[6] = {k > 0 ? p - nx * ny : -1, j > 0 ? p - nx : -1, i > 0 ? p - 1 : -1,
                                 i < nx - 1 ? p + 1 : -1, j < ny - 1 ? p + nx : -1, k < nz - 1 ? p + nx * ny : -1};
        for (int q = 0; q < 6; ++q)
            if (cand[q] >= 0) g.nb[g.nnb++] = cand[q];
    }
    g.b = b;
    g.Gb = grid_vec(n);
    g.Gf = grid_tiles(n, resident_per_cu(warm_gamma));
    const int64_t gm = w->gmax;
    g.partG1 = w->part + 4 * gm;
    g.partG2 = w->part + 5 * gm;
    g.partS = w->part + 8 * gm;
    g.partR = w->part + 9 * gm;
    g.partRb = w->part + 10 * gm;
    g.tolv = w->tolv;
    g.tol = tol;

    RbArgs a{};
    a.n = n;
    a.nr = nr;
    a.nb = nb;
    a.rp = M->rp;
    a.col = M->col;
    a.v32 = M->v32;
    a.d64 = M->d64;
    a.d32 = M->d32;
    a.perm = M->perm;
    a.iperm = M->iperm;
    a.tolv = w->tolv;
    a.ru_delta = delta;
    a.max_iters = max_iters;
    a.break_at = opts.debug_breakdown_at > 0 ? opts.debug_breakdown_at : -1;
    // the red sweep writes no partial sums, so its two instances get grids of their own
    static const int k1g_per_cu[2] = {resident_per_cu(rb_k1<false, true>), resident_per_cu(rb_k1<true, true>)};
    static const int k1_per_cu[2] = {resident_per_cu(rb_k1<false, false>), resident_per_cu(rb_k1<true, false>)};
    static const int k2_per_cu[2] = {resident_per_cu(rb_k2<false>), resident_per_cu(rb_k2<true>)};
    static const int f_per_cu = std::min(std::min(resident_per_cu(rb_f1), resident_per_cu(rb_f2)),
                                         std::min(resident_per_cu(rb_init_red), resident_per_cu(rb_init_black)));
    a.G1 = grid_tiles(nr, std::min(k1_per_cu[mixed], mixed ? kRbRedPerCu : kRb64PerCu));
    const int G1g = grid_tiles(nr, k1g_per_cu[mixed]);
    a.G2 = grid_tiles(nb, mixed ? k2_per_cu[mixed] : std::min(k2_per_cu[mixed], kRb64PerCu));
    a.Gf1 = grid_tiles(nr, f_per_cu);
    a.Gf2 = grid_tiles(nb, f_per_cu);
    a.Gv = grid_vec(nb);
    a.Gw = g.Gf;
    a.Gs = g.Gb;
    a.pin = A->pin;
    a.proj = proj ? 1 : 0;
    a.nnb = g.nnb;
    for (int q = 0; q < 6; ++q) a.nbr[q] = g.nb[q];
    a.b = b;
    a.x = x;
    a.x0 = x0;
    a.y = nullptr;
    a.bp = M->bp;
    a.bS = M->bS;
    a.xb = M->xb;
    a.r64 = M->r64;
    a.y64 = M->y64;
    a.yb = M->yb;
    a.z64 = M->z64;
    a.p64a = M->p64[0];
    a.p64b = M->p64[1];
    a.q64 = M->q64;
    a.z32 = M->z32;
    a.ring32 = M->ring32;
    a.nb_pad = M->nb_pad;
    a.q32 = M->q32;
    a.y32 = M->y32;
    a.partA = M->part;
    a.partB = M->part + gm;
    a.partB2 = M->part + 2 * gm;
    a.partF = M->part + 3 * gm;
    a.partFp = M->part + 4 * gm;
    a.partFz = M->part + 5 * gm;
    a.partF2 = M->part + 6 * gm;
    a.partG1 = g.partG1;
    a.partG2 = g.partG2;
    a.partS = g.partS;
    a.S = M->S;

    CFD_HIP(hipEventRecord(w->ev0, s));
    launch_stop_tol(g, opts, mixed, s);
    if (opts.net) {
        cfd_grid gr{A->nx, A->ny, A->nz, A->h};
        rc = net_predict(opts.net, &gr, b, w->y, s);
        if (rc != CFD_OK) return rc;
        g.y = w->y;
        a.y = w->y;
        hipLaunchKernelGGL(warm_gamma, dim3(g.Gf), dim3(kBlock), 0, s, g);
    }
    if (proj) hipLaunchKernelGGL(rhs_sum, dim3(g.Gb), dim3(kBlock), 0, s, g);
    hipLaunchKernelGGL(rb_rhs, dim3(a.Gv), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(rb_init_red, dim3(a.Gf1), dim3(kBlock), 0, s, a);
    int64_t t = 0;
    hipLaunchKernelGGL(rb_init_black, dim3(a.Gf2), dim3(kBlock), 0, s, a, t);
    ++t;
    CFD_HIP(hipGetLastError());

    const int pool = opts.timing ? 256 : 0;
    while ((int)w->ta.size() < pool) {
        hipEvent_t e0, e1;
        CFD_HIP(hipEventCreate(&e0));
        CFD_HIP(hipEventCreate(&e1));
        w->ta.push_back(e0);
        w->tb.push_back(e1);
    }
    std::vector<char> sampled, live;
    const int64_t cap = (int64_t)max_iters + 64;
    int64_t c = 0;
    RbState final_state{};
    for (;; ++c) {
        if (c > cap) return fail(CFD_EHIP, "cfd_solve: solver control did not terminate");
        bool smp = false;
        for (int i = 0; i < K; ++i) {
            const bool time_it = (i == 1 || K == 1) && c < pool;
            smp = smp || time_it;
            // one product with S: the red sweep and the black sweep
            if (mixed) {
                if (i == 0)
                    hipLaunchKernelGGL((rb_k1<true, true>), dim3(G1g), dim3(kBlock), 0, s, a, t);
                else if (time_it)
                    hipExtLaunchKernelGGL((rb_k1<true, false>), dim3(a.G1), dim3(kBlock), 0, s, w->ta[c], nullptr, 0, a, t);
                else
                    hipLaunchKernelGGL((rb_k1<true, false>), dim3(a.G1), dim3(kBlock), 0, s, a, t);
                ++t;
                if (time_it)
                    hipExtLaunchKernelGGL(rb_k2<true>, dim3(a.G2), dim3(kBlock), 0, s, nullptr, w->tb[c], 0, a, t);
                else
                    hipLaunchKernelGGL(rb_k2<true>, dim3(a.G2), dim3(kBlock), 0, s, a, t);
                ++t;
                hipLaunchKernelGGL(rb_b<true>, dim3(a.Gv), dim3(kBlock), 0, s, a, t);
            } else {
                if (i == 0)
                    hipLaunchKernelGGL((rb_k1<false, true>), dim3(G1g), dim3(kBlock), 0, s, a, t);
                else if (time_it)
                    hipExtLaunchKernelGGL((rb_k1<false, false>), dim3(a.G1), dim3(kBlock), 0, s, w->ta[c], nullptr, 0, a, t);
                else
                    hipLaunchKernelGGL((rb_k1<false, false>), dim3(a.G1), dim3(kBlock), 0, s, a, t);
                ++t;
                if (time_it)
                    hipExtLaunchKernelGGL(rb_k2<false>, dim3(a.G2), dim3(kBlock), 0, s, nullptr, w->tb[c], 0, a, t);
                else
                    hipLaunchKernelGGL(rb_k2<false>, dim3(a.G2), dim3(kBlock), 0, s, a, t);
                ++t;
                hipLaunchKernelGGL(rb_b<false>, dim3(a.Gv), dim3(kBlock), 0, s, a, t);
            }
            ++t;
        }
        if (mixed) {
            hipLaunchKernelGGL(rb_apply, dim3(a.Gv), dim3(kBlock), 0, s, a, t);
            ++t;
        }
        hipLaunchKernelGGL(rb_f1, dim3(a.Gf1), dim3(kBlock), 0, s, a, t);
        ++t;
        hipLaunchKernelGGL(rb_f2, dim3(a.Gf2), dim3(kBlock), 0, s, a, t);
        ++t;
        CFD_HIP(hipGetLastError());
        sampled.push_back(smp);
        live.push_back(0);
        const int slot = (int)(c & 1);
        CFD_HIP(hipMemcpyAsync(&M->host[slot], &M->S[t & 1], sizeof(RbState), hipMemcpyDeviceToHost, s));
        CFD_HIP(hipEventRecord(w->evc[slot], s));
        if (c >= 1) {
            const int prev = (int)((c - 1) & 1);
            CFD_HIP(hipEventSynchronize(w->evc[prev]));
            const RbState ps = M->host[prev];
            live[c - 1] = !ps.cg.done;
            if (ps.cg.done) break;
        }
    }
    CFD_HIP(hipEventSynchronize(w->evc[c & 1]));
    final_state = M->host[c & 1];
    live[c] = !final_state.cg.done;
    CFD_HIP(hipEventRecord(w->ev1, s));
    CFD_HIP(hipEventSynchronize(w->ev1));
    float ms = 0.0f;
    CFD_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));

    const CgState &fs = final_state.cg;
    cfd_solve_info inf{};
    inf.iters = fs.iters;
    inf.updates = fs.updates;
    inf.status = fs.done ? fs.status : CFD_EHIP;
    inf.used_fallback = fs.fallback;
    inf.rel_residual = fs.relres;
    inf.init_residual = fs.init_relres;
    inf.gamma = fs.gamma;
    inf.stop_margin = fs.margin;
    inf.seconds = ms * 1e-3;
    double tot = 0.0;
    int ns = 0;
    for (int64_t i = 0; i < (int64_t)sampled.size() && i < pool; ++i) {
        if (!sampled[i] || !live[i]) continue;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, w->ta[i], w->tb[i]) == hipSuccess) {
            tot += e;
            ++ns;
        }
    }
    inf.spmv_ms = ns ? tot / ns : 0.0;
    inf.spmv_samples = ns;
    if (info) *info = inf;
    if (!fs.done) return fail(CFD_EHIP, "cfd_solve: solver did not finish");
    if (inf.status != CFD_OK) {
        const char *what = inf.status == CFD_ENOCONV ? "max_iters reached"
                         : inf.status == CFD_EBREAKDOWN ? "breakdown: p^T S p <= 0"
                         : inf.status == CFD_ENONFINITE ? "non-finite value in the solve"
                                                        : "solver error";
        return fail(inf.status, std::string("cfd_solve: ") + what);
    }
    return CFD_OK;
}

int solve_internal(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts *o,
                   double *x, cfd_solve_info *info, hipStream_t s) {
    return solve_impl(A, b, x0, tol, o, x, info, s);
}

}  // namespace cfd

extern "C" int cfd_solve(cfd_csr_t A, const double *b, const double *x0, double tol, const cfd_solve_opts *opts,
                         double *x, cfd_solve_info *info, void *stream) {
    if (!A || !b || !x) return cfd::fail(CFD_EINVAL, "cfd_solve: null argument");
    return cfd::solve_impl(A, b, x0, tol, opts, x, info, (hipStream_t)stream);
}
