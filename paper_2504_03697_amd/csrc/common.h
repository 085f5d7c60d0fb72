// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <type_traits>

#include "cfdmi.h"

namespace cfd {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define CFD_HIP(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return ::cfd::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- launch shape

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kTileRows = 256;   // CSR rows per SpMV tile: one row per thread
constexpr int kMaxRowNnz = 7;    // the 7-point stencil
constexpr int kXcd = 8;          // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kSlab = kTileRows * kMaxRowNnz + 4;  // entries a slab may span (+ alignment slack)
// The same for a tile of B rows (SpMV-shaped kernels of B threads, one row each).
template <int B>
constexpr int slab_entries() { return B * kMaxRowNnz + 4; }
constexpr int kPad = 8;          // extra CSR entries allocated past nnz (vector over-read)

struct Device {
    int id = 0;
    int cus = 256;
};
int device_info(Device *d);

// Grid sizes for the solver's kernels on this device (fixed per device so
// reductions, which depend on the number of partial sums, are reproducible).
int grid_spmv(int64_t n, bool fp64_vectors);  // the standalone SpMV
int grid_tiles(int64_t n, int per_cu, int tile_rows = kTileRows);  // SpMV-shaped grid, per_cu workgroups per CU
int grid_vec(int64_t n);

// ---------------------------------------------------------------- matrix handle

struct Workspace;

}  // namespace cfd

struct cfd_csr {
    int32_t nx, ny, nz;
    double h;
    int64_t n, nnz, pin;
    int device;
    int32_t *rp = nullptr;    // n+1
    int32_t *col = nullptr;   // nnz + kPad
    float *val32 = nullptr;   // nnz + kPad; the values are small integers, exact in float32,
                              // so the float64 kernels read them too (exact conversion)
    cfd::Workspace *ws = nullptr;
    void *step_ws = nullptr;  // time-step buffers (step.hip)
    void *sym = nullptr;      // symmetric storage (csr.hip), built on first use
};

namespace cfd {

void workspace_free(Workspace *ws);
void step_ws_free(void *ws);

// ---------------------------------------------------------------- device helpers

// XCD-aware tile schedule.  Workgroup b is dispatched to XCD b % 8; give each
// XCD one contiguous range of tiles so the +-nx*ny plane reuse of the SpMV
// gathers stays inside that XCD's L2.  Falls back to a plain grid-stride loop
// when the grid is not a multiple of 8.
struct TileRange {
    int64_t first, step, end;
};

__device__ inline TileRange tile_range(int64_t ntiles) {
    TileRange t;
    const int G = gridDim.x, b = blockIdx.x;
    if (G >= kXcd && (G % kXcd) == 0) {
        const int x = b % kXcd, lb = b / kXcd, bpx = G / kXcd;
        const int64_t lo = ntiles * x / kXcd, hi = ntiles * (x + 1) / kXcd;
        t.first = lo + lb;
        t.step = bpx;
        t.end = hi;
    } else {
        t.first = b;
        t.step = G;
        t.end = ntiles;
    }
    return t;
}

// Sum over the 64 lanes of a wavefront; every lane receives the same bits.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup of B threads in a fixed order; every thread
// receives the same bits.  `red` must be __shared__ double[B / 64].
template <int B = kBlock>
__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Reduce count partial sums written by the previous kernel, in a fixed order
// (thread t sums entries t, t+B, ... serially, then block_sum).  Every
// block of the calling kernel obtains the same bits.
template <int B = kBlock>
__device__ inline double reduce_partials(const double *part, int count, double *red) {
    // eight loads in flight, then the adds in the same order as one at a time
    // (every kernel starts with this reduction: 0.6 % off the mixed SpMV kernel)
    double s = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * B < count; i += 8 * B) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[i + k * B];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; i < count; i += B) s += part[i];
    return block_sum<B>(s, red);
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Store with the non-temporal hint, for vectors far larger than the L2 that
// the next kernel re-reads from HBM anyway: their lines then do not displace
// the gathered neighbour planes the current sweep reuses from L2.
template <class T>
__device__ inline void store_stream(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Software-pipelined CSR slab loader.  A tile is B consecutive rows (B the
// workgroup size);
// its slab is the contiguous range [ea, e1) of the column and value arrays
// (ea = row_ptr[r0] rounded down to a multiple of 4, so every load is a
// 16-byte vector load).  fetch() issues the loads of a tile into registers;
// commit() stores them to LDS.  The sweep below fetches tile t+1 while the
// rows of tile t gather their vector entries, which keeps HBM requests in
// flight across the whole tile loop.
template <class VT, int B = kBlock>
struct SlabPipe {
    typedef typename std::conditional<sizeof(VT) == 8, f64x2, f32x4>::type VV;
    static constexpr int kPerV = sizeof(VV) / sizeof(VT);  // values per vector load
    static constexpr int kS = slab_entries<B>();
    static constexpr int kVecC = (kS + 4 * B - 1) / (4 * B);
    static constexpr int kVecV = (kS + kPerV * B - 1) / (kPerV * B);
    i32x4 rc[kVecC];
    VV rv[kVecV];
    int64_t r0 = 0;
    int nr = 0, ea = 0, cnt = 0, rs = 0, re = 0;

    __device__ inline void fetch(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const VT *__restrict__ val, int64_t n, int64_t tile) {
        const int tid = threadIdx.x;
        r0 = tile * B;
        nr = (int)(n - r0 < B ? n - r0 : B);
        const int32_t e0 = rp[r0], e1 = rp[r0 + nr];
        ea = e0 & ~3;
        cnt = e1 - ea;
        const i32x4 *c4 = reinterpret_cast<const i32x4 *>(col + ea);
        const VV *v4 = reinterpret_cast<const VV *>(val + ea);
#pragma unroll
        for (int v = 0; v < kVecC; ++v)
            if ((tid + v * B) * 4 < cnt) rc[v] = __builtin_nontemporal_load(c4 + tid + v * B);
#pragma unroll
        for (int v = 0; v < kVecV; ++v)
            if ((tid + v * B) * kPerV < cnt) rv[v] = __builtin_nontemporal_load(v4 + tid + v * B);
        if (tid < nr) {
            rs = rp[r0 + tid] - ea;
            re = rp[r0 + tid + 1] - ea;
        } else {
            rs = re = 0;
        }
    }

    // As fetch(), for the nr_ rows starting at row r0_ (a tile of a row range).
    __device__ inline void fetch_range(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                       const VT *__restrict__ val, int64_t r0_, int nr_) {
        const int tid = threadIdx.x;
        r0 = r0_;
        nr = nr_;
        const int32_t e0 = rp[r0], e1 = rp[r0 + nr];
        ea = e0 & ~3;
        cnt = e1 - ea;
        const i32x4 *c4 = reinterpret_cast<const i32x4 *>(col + ea);
        const VV *v4 = reinterpret_cast<const VV *>(val + ea);
#pragma unroll
        for (int v = 0; v < kVecC; ++v)
            if ((tid + v * B) * 4 < cnt) rc[v] = __builtin_nontemporal_load(c4 + tid + v * B);
#pragma unroll
        for (int v = 0; v < kVecV; ++v)
            if ((tid + v * B) * kPerV < cnt) rv[v] = __builtin_nontemporal_load(v4 + tid + v * B);
        if (tid < nr) {
            rs = rp[r0 + tid] - ea;
            re = rp[r0 + tid + 1] - ea;
        } else {
            rs = re = 0;
        }
    }

    __device__ inline void commit(int32_t *s_col, VT *s_val) const {
        const int tid = threadIdx.x;
#pragma unroll
        for (int v = 0; v < kVecC; ++v)
            if ((tid + v * B) * 4 < cnt) reinterpret_cast<i32x4 *>(s_col)[tid + v * B] = rc[v];
#pragma unroll
        for (int v = 0; v < kVecV; ++v)
            if ((tid + v * B) * kPerV < cnt) reinterpret_cast<VV *>(s_val)[tid + v * B] = rv[v];
    }
};

// LDS entries reserved per slab: commit() stores whole vectors only below cnt
// (at most kSlab + 3 entries).
constexpr int kSlabLds = kSlab + 4;
template <int B>
constexpr int slab_lds() { return slab_entries<B>() + 4; }

// Sweep the tiles assigned to this workgroup (XCD-aware schedule).  For each
// tile, once its slab is in LDS, body(i, rs, re) runs for every row i of the
// tile owned by this thread (one row per thread), with [rs, re) the row's
// entries in s_col/s_val.  The call is workgroup-uniform.
template <class VT, int B = kBlock, class Body>
__device__ inline void csr_sweep(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const VT *__restrict__ val, int64_t n, int32_t *s_col, VT *s_val, Body &&body) {
    const int64_t ntiles = (n + B - 1) / B;
    const TileRange tr = tile_range(ntiles);
    SlabPipe<VT, B> P;
    if (tr.first < tr.end) P.fetch(rp, col, val, n, tr.first);
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t r0 = P.r0;
        const int nr = P.nr, rs = P.rs, re = P.re;
        P.commit(s_col, s_val);
        __syncthreads();
        if (t + tr.step < tr.end) P.fetch(rp, col, val, n, t + tr.step);
        if ((int)threadIdx.x < nr) body(r0 + threadIdx.x, rs, re);
        __syncthreads();
    }
}

// csr_sweep with per-row operands fetched one tile ahead as well: pre(i)
// loads what the body needs from row i's own vector entries, for the next
// tile while the current one computes; body(i, rs, re, v) gets the value.
template <class VT, int B = kBlock, class Pre, class Body>
__device__ inline void csr_sweep_pre(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                     const VT *__restrict__ val, int64_t n, int32_t *s_col, VT *s_val, Pre &&pre,
                                     Body &&body) {
    using T = decltype(pre(int64_t(0)));
    const int64_t ntiles = (n + B - 1) / B;
    const TileRange tr = tile_range(ntiles);
    SlabPipe<VT, B> P;
    T next{};
    if (tr.first < tr.end) {
        P.fetch(rp, col, val, n, tr.first);
        if ((int)threadIdx.x < P.nr) next = pre(P.r0 + threadIdx.x);
    }
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t r0 = P.r0;
        const int nr = P.nr, rs = P.rs, re = P.re;
        const T cur = next;
        P.commit(s_col, s_val);
        __syncthreads();
        if (t + tr.step < tr.end) {
            P.fetch(rp, col, val, n, t + tr.step);
            if ((int)threadIdx.x < P.nr) next = pre(P.r0 + threadIdx.x);
        }
        if ((int)threadIdx.x < nr) body(r0 + threadIdx.x, rs, re, cur);
        __syncthreads();
    }
}

// Row product over the staged slab: sum_e val[e] * g(col[e]) in ascending
// column order.  Rows of the 7-point matrix hold at most 7 entries.
template <class Acc, class VT, class G>
__device__ inline Acc row_product(const int32_t *s_col, const VT *s_val, int rs, int re, G &&g) {
    Acc acc = Acc(0);
#pragma unroll
    for (int k = 0; k < kMaxRowNnz; ++k) {
        const int e = rs + k;
        if (e < re) acc = fma(Acc(s_val[e]), g(s_col[e]), acc);
    }
    return acc;
}

// Slab loader of the streamed sweep below: the same tiles and slabs as
// SlabPipe, with fewer waits.  A wave's memory counter drains in issue order,
// so a wait for any load also waits for every older one.  fetch() therefore
// takes the tile's entry bounds as arguments (loaded with the previous tile,
// lanes 0 and 1 of bv) instead of loading them and waiting; every load it
// issues is unconditional (indexes clamped into the tile); and the row
// pointers it loads stay raw until the commit that consumes the slab.  So
// nothing between a fetch and that commit waits for the slab, and the
// row gathers of the current tile overlap it.  It costs registers: the
// float32 SpMV, the red-black sweeps and the float64 CG kernel gain from it
// (3-4 % at 256^3); the mixed CG kernel (at its 64-register limit) and the
// float64 SpMV do not, and keep SlabPipe.
template <class VT, int B = kBlock>
struct SlabStream {
    typedef typename std::conditional<sizeof(VT) == 8, f64x2, f32x4>::type VV;
    static constexpr int kPerV = sizeof(VV) / sizeof(VT);  // values per vector load
    static constexpr int kS = slab_entries<B>();
    static constexpr int kVecC = (kS + 4 * B - 1) / (4 * B);
    static constexpr int kVecV = (kS + kPerV * B - 1) / (kPerV * B);
    i32x4 rc[kVecC];
    VV rv[kVecV];
    int64_t r0 = 0;
    int nr = 0, ea = 0, cnt = 0, e0 = 0;
    int rsr = 0, rer = 0;  // row_ptr of this thread's row (clamped into the tile) and the next
    int bv = 0;            // lane 0: row_ptr at the start of the tile after; lane 1: at its end

    // Load the nr_ rows from r0_, whose entries are [b0, b1), and the entry
    // bounds of the nq rows from q0 (the tile fetched next).  b1 > b0.
    __device__ inline void fetch(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const VT *__restrict__ val, int64_t r0_, int nr_, int b0, int b1, int64_t q0,
                                 int nq) {
        const int tid = threadIdx.x;
        r0 = r0_;
        nr = nr_;
        e0 = b0;
        ea = b0 & ~3;
        cnt = b1 - ea;
        const int lastc = (cnt - 1) >> 2, lastv = (cnt - 1) / kPerV;
        const i32x4 *c4 = reinterpret_cast<const i32x4 *>(col + ea);
        const VV *v4 = reinterpret_cast<const VV *>(val + ea);
#pragma unroll
        for (int v = 0; v < kVecC; ++v) rc[v] = __builtin_nontemporal_load(c4 + min(tid + v * B, lastc));
#pragma unroll
        for (int v = 0; v < kVecV; ++v) rv[v] = __builtin_nontemporal_load(v4 + min(tid + v * B, lastv));
        const int64_t rr = r0 + min(tid, nr - 1);
        rsr = rp[rr];
        rer = rp[rr + 1];
        bv = rp[q0 + ((tid & 63) == 1 ? nq : 0)];
    }

    // Entry bounds of the tile after the fetched one (uniform).
    __device__ inline void bounds(int &b0, int &b1) const {
        b0 = __builtin_amdgcn_readfirstlane(bv);
        b1 = __builtin_amdgcn_readlane(bv, 1);
    }

    __device__ inline void commit(int32_t *s_col, VT *s_val) const {
        const int tid = threadIdx.x;
#pragma unroll
        for (int v = 0; v < kVecC; ++v)
            if ((tid + v * B) * 4 < cnt) reinterpret_cast<i32x4 *>(s_col)[tid + v * B] = rc[v];
#pragma unroll
        for (int v = 0; v < kVecV; ++v)
            if ((tid + v * B) * kPerV < cnt) reinterpret_cast<VV *>(s_val)[tid + v * B] = rv[v];
    }
};

// Sweep the rows [row_begin, row_end) in tiles of B rows counted from
// row_begin, the tiles assigned to this workgroup by the XCD-aware schedule.
// pre(i) loads what the body needs from row i's own vector entries; it runs
// for the next tile while the current one computes (it must accept any row
// of the range: rows past a tile's end are clamped to its last row).  Once a
// tile's slab is in LDS, body(i, rs, re, v) runs for every row i of the tile
// owned by this thread (one row per thread), with [rs, re) the row's entries
// in s_col/s_val and v = pre(i).  The call is workgroup-uniform; every row
// holds at least one entry.  stage(r0, nr, v) runs in every thread as each
// tile's slab goes to LDS, before the barrier that publishes it (v = pre of
// the thread's row of that tile; rows past its end see the last row's), so
// values it stores in LDS are there for the tile's bodies.
template <class VT, int B = kBlock, class Pre, class Stage, class Body>
__device__ inline void csr_stream_rows_staged(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                             const VT *__restrict__ val, int64_t row_begin, int64_t row_end,
                                             int32_t *s_col, VT *s_val, Pre &&pre, Stage &&stage, Body &&body) {
    using T = decltype(pre(int64_t(0)));
    const int64_t rows = row_end - row_begin;
    const int64_t ntiles = (rows + B - 1) / B;
    const TileRange tr = tile_range(ntiles);
    if (tr.first >= tr.end) return;
    auto tile_r0 = [&](int64_t t) -> int64_t { return row_begin + t * B; };
    auto tile_nr = [&](int64_t t) -> int {
        return (int)(rows - t * B < B ? rows - t * B : B);
    };
    const int tid = threadIdx.x;
    SlabStream<VT, B> P;
    {
        const int64_t t = tr.first, tq = t + tr.step < tr.end ? t + tr.step : t;
        const int64_t r0 = tile_r0(t);
        const int nr = tile_nr(t);
        P.fetch(rp, col, val, r0, nr, rp[r0], rp[r0 + nr], tile_r0(tq), tile_nr(tq));
    }
    T next = pre(P.r0 + min(tid, P.nr - 1));
    for (int64_t t = tr.first; t < tr.end; t += tr.step) {
        const int64_t r0 = P.r0;
        const int nr = P.nr, e0 = P.e0;
        const int rs = P.rsr - P.ea, re = P.rer - P.ea;
        const T cur = next;
        int b0, b1;
        P.bounds(b0, b1);
        P.commit(s_col, s_val);
        stage(r0, nr, cur);
        __syncthreads();
        // After the last tile the fetch re-reads the current tile's first
        // vector, so every iteration issues the same loads.
        const int64_t tn = t + tr.step;
        const bool more = tn < tr.end;
        const int64_t tq = tn + tr.step < tr.end ? tn + tr.step : tn;
        P.fetch(rp, col, val, more ? tile_r0(tn) : r0, more ? tile_nr(tn) : nr, more ? b0 : e0,
                more ? b1 : e0 + 1, more ? tile_r0(tq) : r0, more ? tile_nr(tq) : nr);
        next = pre(P.r0 + min(tid, P.nr - 1));
        if (tid < nr) body(r0 + tid, rs, re, cur);
        __syncthreads();
    }
}

template <class VT, int B = kBlock, class Pre, class Body>
__device__ inline void csr_stream_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                      const VT *__restrict__ val, int64_t row_begin, int64_t row_end,
                                      int32_t *s_col, VT *s_val, Pre &&pre, Body &&body) {
    csr_stream_rows_staged<VT, B>(rp, col, val, row_begin, row_end, s_col, s_val, pre,
                                  [](int64_t, int, const auto &) {}, body);
}

// row_product with all gathers issued before the first multiply-add: the
// slots past the row's end gather the row's first entry again and are left
// out of the sum by a select, which adds the same terms in the same order as
// row_product (bit-identical results).  The row holds at least one entry.
template <class Acc, class VT, class G>
__device__ inline Acc row_product_all(const int32_t *s_col, const VT *s_val, int rs, int re, G &&g) {
    Acc v[kMaxRowNnz], w[kMaxRowNnz];
#pragma unroll
    for (int k = 0; k < kMaxRowNnz; ++k) {
        const int e = rs + k < re ? rs + k : rs;
        v[k] = Acc(s_val[e]);
        w[k] = g(s_col[e]);
    }
    Acc acc = Acc(0);
#pragma unroll
    for (int k = 0; k < kMaxRowNnz; ++k) {
        const Acc f = fma(v[k], w[k], acc);
        acc = rs + k < re ? f : acc;
    }
    return acc;
}

}  // namespace cfd
