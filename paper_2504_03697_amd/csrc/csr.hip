// Matrix handle: assembly on the device, export, plain SpMV, right-hand-side
// preparation, and the library's error reporting.
#include "common.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

namespace cfd {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CFD_ENOMEM : CFD_EHIP;
}

int device_info(Device *d) {
    CFD_HIP(hipGetDevice(&d->id));
    int cus = 0;
    CFD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->id));
    d->cus = cus > 0 ? cus : 1;
    return CFD_OK;
}

static int g_cus = 0;

static int cus() {
    if (g_cus == 0) {
        Device d;
        if (device_info(&d) == CFD_OK) g_cus = d.cus;
        else g_cus = 256;
    }
    return g_cus;
}

static int round_grid(int64_t want, int64_t cap) {
    int64_t g = std::min(want, cap);
    if (g >= kXcd) g -= g % kXcd;
    return (int)std::max<int64_t>(g, 1);
}

// Workgroups per CU of the standalone SpMV with float64 vectors: measured at
// 256^3, 245 / 240 / 236 us per product at 6 / 7 / 8.
constexpr int kSpmv64PerCu = 8;

// The float32 SpMV sweeps tiles of kSpmv32Rows rows with workgroups of as
// many threads, kSpmv32PerCu per CU.  HBM streams a workgroup's slab faster
// when it spans more contiguous bytes: at the same registers and bytes in
// flight per CU, 512-thread workgroups reading 16 KB per array per tile
// measured 0.86 of 8 TB/s in a plain read, 256-thread ones reading 8 KB 0.79.
constexpr int kSpmv32Rows = 512;
constexpr int kSpmv32PerCu = 4;

// Workgroups for the SpMV-shaped kernels: 8 resident workgroups (32 waves)
// per CU measured best on MI355X at 256^3; at most one per tile.  The grid is
// the same for every SpMV-shaped kernel of the solver so that their partial
// sums line up.
int grid_spmv(int64_t n, bool fp64_vectors) {
    return grid_tiles(n, fp64_vectors ? kSpmv64PerCu : 8);
}

int grid_tiles(int64_t n, int per_cu, int tile_rows) {
    const int64_t tiles = (n + tile_rows - 1) / tile_rows;
    return round_grid(tiles, (int64_t)cus() * per_cu);
}

// Workgroups for the streaming vector kernels (4 wave64 each).
int grid_vec(int64_t n) {
    const int64_t chunks = (n + 4 * kBlock - 1) / (4 * kBlock);
    return round_grid(chunks, (int64_t)cus() * 4);
}

// ---------------------------------------------------------------- assembly

// Entries of the unpinned row (i,j,k): 1 + number of in-domain neighbours.
__host__ __device__ inline int64_t cnt1(int64_t a, int64_t n) {  // neighbours along one axis
    return (a > 0) + (a < n - 1);
}
// sum_{a' < a} cnt1(a', n)
__host__ __device__ inline int64_t pre1(int64_t a, int64_t n) {
    return (a > 1 ? a - 1 : 0) + (a < n - 1 ? a : n - 1);
}

// Start of row (i,j,k) in the unpinned matrix, in closed form: rows are
// ordered x fastest, so the start is the sum of the lengths of all complete
// z-planes, y-lines and cells before it.
__host__ __device__ inline int64_t row_start_unpinned(int64_t i, int64_t j, int64_t k, int64_t nx,
                                                      int64_t ny, int64_t nz) {
    const int64_t sx = pre1(nx, nx), sy = pre1(ny, ny);  // 2(n-1) for n >= 1
    const int64_t cz = cnt1(k, nz), cy = cnt1(j, ny);
    const int64_t planes = k * (ny * (nx + sx) + nx * sy) + nx * ny * pre1(k, nz);
    const int64_t lines = j * (nx * (1 + cz) + sx) + nx * pre1(j, ny);
    const int64_t cells = i * (1 + cy + cz) + pre1(i, nx);
    return planes + lines + cells;
}

struct PinInfo {
    int64_t pin;          // -1: none
    int64_t nb[6];        // in-domain neighbours of the pin, ascending
    int nnb;
    int64_t pin_len;      // unpinned length of the pin row
};

__host__ __device__ inline int64_t row_start(int64_t row, int64_t i, int64_t j, int64_t k,
                                             int64_t nx, int64_t ny, int64_t nz, const PinInfo &P) {
    int64_t s = row_start_unpinned(i, j, k, nx, ny, nz);
    if (P.pin >= 0) {
        if (row > P.pin) s -= P.pin_len - 1;           // the pin row keeps one entry
        for (int q = 0; q < P.nnb; ++q) s -= (P.nb[q] < row);  // each neighbour loses one
    }
    return s;
}

__global__ void __launch_bounds__(kBlock) assemble_kernel(int64_t nx, int64_t ny, int64_t nz,
                                                          PinInfo P, int32_t *__restrict__ rp,
                                                          int32_t *__restrict__ col,
                                                          float *__restrict__ v32) {
    const int64_t n = nx * ny * nz;
    for (int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x; row <= n;
         row += (int64_t)gridDim.x * kBlock) {
        if (row == n) {
            rp[n] = (int32_t)row_start(n, 0, 0, nz, nx, ny, nz, P);  // one past the last plane
            continue;
        }
        const int64_t i = row % nx, j = (row / nx) % ny, k = row / (nx * ny);
        int64_t e = row_start(row, i, j, k, nx, ny, nz, P);
        rp[row] = (int32_t)e;
        if (row == P.pin) {
            col[e] = (int32_t)row;
            v32[e] = 1.0f;
            continue;
        }
        const int64_t deg = cnt1(i, nx) + cnt1(j, ny) + cnt1(k, nz);
        const int64_t cand[7] = {k > 0 ? row - nx * ny : -1, j > 0 ? row - nx : -1,
                                 i > 0 ? row - 1 : -1,       row,
                                 i < nx - 1 ? row + 1 : -1,  j < ny - 1 ? row + nx : -1,
                                 k < nz - 1 ? row + nx * ny : -1};
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const int64_t c = cand[q];
            if (c < 0 || c == P.pin) continue;
            col[e] = (int32_t)c;
            v32[e] = (c == row) ? (float)deg : -1.0f;
            ++e;
        }
    }
}

// Zero the vector over-read padding past nnz so it never holds NaN bits.
__global__ void pad_kernel(int64_t nnz, int32_t *col, float *v32) {
    const int t = threadIdx.x;
    if (t < kPad) {
        col[nnz + t] = 0;
        v32[nnz + t] = 0.0f;
    }
}

// val = the values in float64 (an exact conversion).
__global__ void __launch_bounds__(kBlock) widen_kernel(int64_t nnz, const float *__restrict__ v32,
                                                       double *__restrict__ val) {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock)
        val[e] = (double)v32[e];
}

}  // namespace cfd

using namespace cfd;

extern "C" int cfd_assemble(const cfd_grid *grid, int64_t pin, void *stream, cfd_csr_t *out) {
    if (!grid || !out) return fail(CFD_EINVAL, "cfd_assemble: null argument");
    *out = nullptr;
    const int64_t nx = grid->nx, ny = grid->ny, nz = grid->nz;
    if (nx < 1 || ny < 1 || nz < 1) return fail(CFD_EINVAL, "cfd_assemble: grid dimensions must be >= 1");
    if (!(grid->h > 0.0)) return fail(CFD_EINVAL, "cfd_assemble: h must be > 0");
    const int64_t n = nx * ny * nz;
    if (pin >= n) return fail(CFD_EINVAL, "cfd_assemble: pin index out of range");
    if (pin < 0) pin = -1;
    PinInfo P{};
    P.pin = pin;
    P.nnb = 0;
    P.pin_len = 0;
    if (pin >= 0) {
        const int64_t i = pin % nx, j = (pin / nx) % ny, k = pin / (nx * ny);
        const int64_t cand[6] = {k > 0 ? pin - nx * ny : -1, j > 0 ? pin - nx : -1,
                                 i > 0 ? pin - 1 : -1,       i < nx - 1 ? pin + 1 : -1,
                                 j < ny - 1 ? pin + nx : -1, k < nz - 1 ? pin + nx * ny : -1};
        for (int q = 0; q < 6; ++q)
            if (cand[q] >= 0) P.nb[P.nnb++] = cand[q];
        P.pin_len = 1 + P.nnb;
    }
    const int64_t nnz = row_start(n, 0, 0, nz, nx, ny, nz, P);
    if (n + 1 > INT32_MAX || nnz + kPad > INT32_MAX)
        return fail(CFD_EINVAL, "cfd_assemble: matrix too large for 32-bit CSR indices");

    cfd_csr *A = new cfd_csr();
    A->nx = (int32_t)nx;
    A->ny = (int32_t)ny;
    A->nz = (int32_t)nz;
    A->h = grid->h;
    A->n = n;
    A->nnz = nnz;
    A->pin = pin;
    int rc = CFD_OK;
    hipError_t e = hipGetDevice(&A->device);
    if (e == hipSuccess) e = hipMalloc(&A->rp, sizeof(int32_t) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&A->col, sizeof(int32_t) * (nnz + kPad));
    if (e == hipSuccess) e = hipMalloc(&A->val32, sizeof(float) * (nnz + kPad));
    if (e != hipSuccess) {
        rc = hip_fail(e, "cfd_assemble: hipMalloc");
        cfd_csr_destroy(A);
        return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t blocks = std::min<int64_t>((n + 1 + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, nx, ny, nz, P,
                       A->rp, A->col, A->val32);
    hipLaunchKernelGGL(pad_kernel, dim3(1), dim3(64), 0, s, nnz, A->col, A->val32);
    e = hipGetLastError();
    if (e != hipSuccess) {
        rc = hip_fail(e, "cfd_assemble: launch");
        cfd_csr_destroy(A);
        return rc;
    }
    *out = A;
    return CFD_OK;
}

extern "C" int cfd_csr_info(cfd_csr_t A, int64_t *n, int64_t *nnz) {
    if (!A) return fail(CFD_EINVAL, "cfd_csr_info: null handle");
    if (n) *n = A->n;
    if (nnz) *nnz = A->nnz;
    return CFD_OK;
}

extern "C" int cfd_csr_export(cfd_csr_t A, int32_t *row_ptr, int32_t *col, double *val, void *stream) {
    if (!A) return fail(CFD_EINVAL, "cfd_csr_export: null handle");
    hipStream_t s = (hipStream_t)stream;
    if (row_ptr)
        CFD_HIP(hipMemcpyAsync(row_ptr, A->rp, sizeof(int32_t) * (A->n + 1), hipMemcpyDeviceToDevice, s));
    if (col) CFD_HIP(hipMemcpyAsync(col, A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, s));
    if (val && A->nnz > 0) {
        const int64_t blocks = std::min<int64_t>((A->nnz + kBlock - 1) / kBlock, 65536);
        hipLaunchKernelGGL(widen_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, A->nnz,
                           (const float *)A->val32, val);
        CFD_HIP(hipGetLastError());
    }
    return CFD_OK;
}

namespace cfd {
static void sym_free(void *p);
}

extern "C" void cfd_csr_destroy(cfd_csr_t A) {
    if (!A) return;
    if (A->ws) workspace_free(A->ws);
    if (A->step_ws) step_ws_free(A->step_ws);
    if (A->sym) sym_free(A->sym);
    if (A->rp) (void)hipFree(A->rp);
    if (A->col) (void)hipFree(A->col);
    if (A->val32) (void)hipFree(A->val32);
    delete A;
}

// ---------------------------------------------------------------- plain SpMV

namespace cfd {

// y = A x with vectors of type VT; the values are the exact float32 array in
// both precisions (a float64 product of a converted value is exact).
template <class VT, int B>
__global__ void __launch_bounds__(B) spmv_kernel(const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const float *__restrict__ val, int64_t n,
                                                 const VT *__restrict__ x, VT *__restrict__ y) {
    __shared__ __align__(16) int32_t s_col[slab_lds<B>()];
    __shared__ __align__(16) float s_val[slab_lds<B>()];
    auto xg = [&](int j) { return x[j]; };
    if constexpr (sizeof(VT) == 4) {
        csr_stream_rows<float, B>(rp, col, val, 0, n, s_col, s_val, [](int64_t) { return 0; },
                               [&](int64_t i, int rs, int re, int) {
                                   store_stream(y + i, row_product_all<float>(s_col, s_val, rs, re, xg));
                               });
    } else {
        csr_sweep<float, B>(rp, col, val, n, s_col, s_val, [&](int64_t i, int rs, int re) {
            store_stream(y + i, row_product<double>(s_col, s_val, rs, re, xg));
        });
    }
}

// ---------------------------------------------------------------- plane-marching sweep
//
// For grids whose x-rows are one workgroup long (nx = B, x fastest).
// Workgroup (row j, planes k0 .. k0 + KZ - 1) walks up its z range one
// x-row (B consecutive CSR rows) at a time.  The row's slab goes through the
// register pipeline of csr_stream_rows (SlabStream), and the vector values
// the 7-point rows read sit in LDS, staged a step ahead: row j at planes
// k - 1, k, k + 1 (a 3-slot ring, each row staged once, as plane k + 2) and
// rows j - 1, j + 1 at plane k.  Workgroups b with b mod 8 = c (one XCD)
// take the rows j of one contiguous range, so the rows j +- 1 a workgroup
// stages are ones its neighbours on that XCD have just brought into L2.
constexpr int kZmarchB = 256;                  // x-row length (= workgroup size)
constexpr int kZmarchKz = 8;                   // planes per workgroup
constexpr int64_t kZmarchMinRows = 1 << 22;    // below: too few workgroups

// Workgroups (row j, z range) of the plane-marching kernels for an
// nx x ny x nz grid of n cells, 0 when they do not apply.
inline int zmarch_grid(int nx, int ny, int nz, int64_t n) {
    if (nx != kZmarchB || n < kZmarchMinRows) return 0;
    return kXcd * ((ny + kXcd - 1) / kXcd) * ((nz + kZmarchKz - 1) / kZmarchKz);
}

// The LDS a plane-marching sweep stages its values in.
template <int B>
struct ZStage {
    float zr[3][B];  // row j, planes k - 1, k, k + 1 (slot = plane mod 3)
    float yr[2][B];  // rows j - 1, j + 1 at plane k
};

// Value staged for the neighbour at offset d = column - row of the cell in
// lane tid, or false if d is no 7-point offset.  The z offsets are tested
// first: with ny = 1 the z offset equals B.
template <int B>
__device__ inline bool zmarch_value(const ZStage<B> &S, int k, int tid, int64_t d, int64_t nxny, float &v) {
    if (d == -nxny) v = S.zr[(k + 2) % 3][tid];
    else if (d == nxny) v = S.zr[(k + 1) % 3][tid];
    else if (d == -B) v = S.yr[0][tid];
    else if (d == B) v = S.yr[1][tid];
    else if (d >= -1 && d <= 1) v = S.zr[k % 3][tid + (int)d];  // i +- 1 stays in the row (walls have no entry)
    else return false;
    return true;
}

// The sweep.  stage(idx) gives the value to stage for grid cell idx (it is
// called with indexes clamped into the grid; values of cells outside it are
// never read).  body(r, rs, re, k) runs for the row r = (k ny + j) B + tid of
// every step, with its entries [rs, re) in s_col/s_val and the staged
// values readable through zmarch_value(S, k, tid, ...).  The call is
// workgroup-uniform; the workgroup returns at once if it has no rows.
template <int B, int KZ, class Stage, class Body>
__device__ inline void zmarch_sweep(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                    const float *__restrict__ val, int ny, int nz, int32_t *s_col, float *s_val,
                                    ZStage<B> &S, Stage &&stage, Body &&body) {
    const int tid = threadIdx.x;
    const int jper = (ny + kXcd - 1) / kXcd;
    const int b = blockIdx.x, l = b / kXcd;
    const int j = (b % kXcd) * jper + l % jper;
    const int k0 = (l / jper) * KZ;
    if (j >= ny || k0 >= nz) return;
    const int k1 = min(nz, k0 + KZ);
    auto cell = [&](int jj, int kk) -> float {
        jj = min(max(jj, 0), ny - 1);
        kk = min(max(kk, 0), nz - 1);
        return stage(((int64_t)kk * ny + jj) * B + tid);
    };
    auto tile_r0 = [&](int kk) -> int64_t { return ((int64_t)kk * ny + j) * B; };
    SlabStream<float, B> P;
    {
        const int64_t r0 = tile_r0(k0);
        const int kq = k0 + 1 < k1 ? k0 + 1 : k0;
        P.fetch(rp, col, val, r0, B, rp[r0], rp[r0 + B], tile_r0(kq), B);
    }
    S.zr[(k0 + 2) % 3][tid] = cell(j, k0 - 1);
    S.zr[k0 % 3][tid] = cell(j, k0);
    S.zr[(k0 + 1) % 3][tid] = cell(j, k0 + 1);
    S.yr[0][tid] = cell(j - 1, k0);
    S.yr[1][tid] = cell(j + 1, k0);
    for (int k = k0; k < k1; ++k) {
        const int64_t r0 = tile_r0(k);
        const int e0 = P.e0, ea = P.ea;
        const int rs = P.rsr - ea, re = P.rer - ea;
        int b0, b1;
        P.bounds(b0, b1);
        P.commit(s_col, s_val);
        __syncthreads();
        // the next step's slab and rows (after the last step a dummy
        // re-read, so every step issues the same loads)
        const bool more = k + 1 < k1;
        const int kn = more ? k + 1 : k;
        const int kq = kn + 1 < k1 ? kn + 1 : kn;
        P.fetch(rp, col, val, tile_r0(kn), B, more ? b0 : e0, more ? b1 : e0 + 1, tile_r0(kq), B);
        const float nym = cell(j - 1, k + 1), nyp = cell(j + 1, k + 1), nzp = cell(j, k + 2);
        body(r0 + tid, rs, re, k);
        __syncthreads();
        S.yr[0][tid] = nym;
        S.yr[1][tid] = nyp;
        S.zr[(k + 2) % 3][tid] = nzp;  // plane k + 2 takes the slot of plane k - 1
    }
}

// Plane-marching float32 SpMV (zmarch_sweep above) for grids with
// 256-cell x-rows: the row products read x from LDS, in the CSR's entry
// order, so y has the tile kernel's bits; an entry whose column is no
// 7-point neighbour reads x from memory.  Measured at 256^3: 202.2 against
// 204.8 us per product back to back (0.703 against 0.694 of 8 TB/s).
__global__ void __launch_bounds__(kZmarchB) spmv_zmarch(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const float *__restrict__ val, int ny, int nz,
                                                        const float *__restrict__ x, float *__restrict__ y) {
    constexpr int B = kZmarchB;
    __shared__ __align__(16) int32_t s_col[slab_lds<B>()];
    __shared__ __align__(16) float s_val[slab_lds<B>()];
    __shared__ ZStage<B> S;
    const int64_t nxny = (int64_t)B * ny;
    const int tid = threadIdx.x;
    zmarch_sweep<B, kZmarchKz>(rp, col, val, ny, nz, s_col, s_val, S, [&](int64_t idx) { return x[idx]; },
                               [&](int64_t r, int rs, int re, int k) {
                                   float acc = 0.0f;
#pragma unroll
                                   for (int q = 0; q < kMaxRowNnz; ++q) {
                                       const int e = rs + q < re ? rs + q : rs;
                                       float xv;
                                       if (!zmarch_value(S, k, tid, (int64_t)s_col[e] - r, nxny, xv)) xv = x[s_col[e]];
                                       const float f = fmaf(s_val[e], xv, acc);
                                       acc = rs + q < re ? f : acc;
                                   }
                                   store_stream(y + r, acc);
                               });
}

// Partial sums of b for the mean.
__global__ void __launch_bounds__(kBlock) sum_kernel(const double *__restrict__ b, int64_t n,
                                                     double *__restrict__ part) {
    __shared__ double red[kBlock / 64];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = chunk * blockIdx.x, hi = std::min(n, lo + chunk);
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) s += b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) center_kernel(double *__restrict__ b, int64_t n, int64_t pin,
                                                        const double *__restrict__ part, int count) {
    __shared__ double red[kBlock / 64];
    const double mean = reduce_partials(part, count, red) / (double)n;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        b[i] = (i == pin) ? 0.0 : b[i] - mean;
}

}  // namespace cfd

extern "C" int cfd_spmv(cfd_csr_t A, int32_t precision, const void *x, void *y, void *stream) {
    if (!A || !x || !y) return fail(CFD_EINVAL, "cfd_spmv: null argument");
    if (precision != CFD_PREC_FP64 && precision != CFD_PREC_MIXED)
        return fail(CFD_EINVAL, "cfd_spmv: precision must be 0 (float64) or 1 (float32)");
    hipStream_t s = (hipStream_t)stream;
    if (precision == CFD_PREC_FP64)
        hipLaunchKernelGGL((spmv_kernel<double, kBlock>), dim3(grid_spmv(A->n, true)), dim3(kBlock), 0, s, A->rp,
                           A->col, A->val32, A->n, (const double *)x, (double *)y);
    else if (const int G = zmarch_grid(A->nx, A->ny, A->nz, A->n))
        hipLaunchKernelGGL(spmv_zmarch, dim3(G), dim3(kZmarchB), 0, s, A->rp, A->col, A->val32, A->ny, A->nz,
                           (const float *)x, (float *)y);
    else
        hipLaunchKernelGGL((spmv_kernel<float, kSpmv32Rows>), dim3(grid_tiles(A->n, kSpmv32PerCu, kSpmv32Rows)),
                           dim3(kSpmv32Rows), 0, s, A->rp, A->col, A->val32, A->n, (const float *)x, (float *)y);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

// ---------------------------------------------------------------- symmetric storage

namespace cfd {

// The matrix in the layout of Sec. 3.3: the diagonal and the upper triangle
// as a CSR with values (diagonal first in each row), and the lower triangle
// as a column pattern only.  n + 1 row pointers each; kPad zeroed entries
// past the ends of the slab-loaded arrays.
struct SymStorage {
    int64_t nnz_u = 0, nnz_l = 0;
    int32_t *rp_u = nullptr, *col_u = nullptr, *rp_l = nullptr, *col_l = nullptr;
    float *val_u = nullptr;
};

static void sym_free(void *p) {
    SymStorage *S = (SymStorage *)p;
    void *pp[] = {S->rp_u, S->col_u, S->rp_l, S->col_l, S->val_u};
    for (void *q : pp) if (q) (void)hipFree(q);
    delete S;
}

// Entries of row i left of the diagonal (the columns ascend in a row).
__global__ void __launch_bounds__(kBlock) sym_count(int64_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, int32_t *__restrict__ cl) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        int32_t e = rp[i];
        while (e < rp[i + 1] && col[e] < i) ++e;
        cl[i] = e - rp[i];
    }
}

// Split each row: its lower columns go to col_l at rp_l[i], its diagonal and
// upper entries to col_u/val_u at rp_u[i] = rp[i] - rp_l[i].
__global__ void __launch_bounds__(kBlock) sym_fill(int64_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, const float *__restrict__ val,
                                                   const int32_t *__restrict__ rp_l, int32_t *__restrict__ rp_u,
                                                   int32_t *__restrict__ col_u, float *__restrict__ val_u,
                                                   int32_t *__restrict__ col_l) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t l = rp_l[i], u = rp[i] - l;
        rp_u[i] = u;
        if (i == n) continue;
        int32_t k = u;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < i) {
                col_l[l + (e - rp[i])] = col[e];
            } else {
                col_u[k] = col[e];
                val_u[k] = val[e];
                ++k;
            }
        }
    }
}

static int sym_build(cfd_csr_t A, hipStream_t s) {
    if (A->sym) return CFD_OK;
    const int64_t n = A->n;
    SymStorage *S = new SymStorage();
    std::vector<int32_t> cl(n), rpl(n + 1);
    int32_t *d_cl = nullptr;
    hipError_t h = hipMalloc(&d_cl, sizeof(int32_t) * std::max<int64_t>(n, 1));
    const unsigned g = (unsigned)std::min<int64_t>((n + 1 + kBlock - 1) / kBlock, 65536);
    if (h == hipSuccess) {
        hipLaunchKernelGGL(sym_count, dim3(g), dim3(kBlock), 0, s, n, (const int32_t *)A->rp,
                           (const int32_t *)A->col, d_cl);
        h = hipGetLastError();
    }
    if (h == hipSuccess) h = hipMemcpyAsync(cl.data(), d_cl, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    if (d_cl) (void)hipFree(d_cl);
    if (h != hipSuccess) {
        sym_free(S);
        return hip_fail(h, "cfd_spmv_sym: row counts");
    }
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        rpl[i] = (int32_t)acc;
        acc += cl[i];
    }
    rpl[n] = (int32_t)acc;
    S->nnz_l = acc;
    S->nnz_u = A->nnz - acc;
    if (h == hipSuccess) h = hipMalloc(&S->rp_l, sizeof(int32_t) * (n + 1));
    if (h == hipSuccess) h = hipMalloc(&S->rp_u, sizeof(int32_t) * (n + 1));
    if (h == hipSuccess) h = hipMalloc(&S->col_u, sizeof(int32_t) * (S->nnz_u + kPad));
    if (h == hipSuccess) h = hipMalloc(&S->val_u, sizeof(float) * (S->nnz_u + kPad));
    if (h == hipSuccess) h = hipMalloc(&S->col_l, sizeof(int32_t) * std::max<int64_t>(S->nnz_l, 1));
    if (h == hipSuccess) h = hipMemcpyAsync(S->rp_l, rpl.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s);
    if (h == hipSuccess) h = hipMemsetAsync(S->col_u + S->nnz_u, 0, sizeof(int32_t) * kPad, s);
    if (h == hipSuccess) h = hipMemsetAsync(S->val_u + S->nnz_u, 0, sizeof(float) * kPad, s);
    if (h == hipSuccess) {
        hipLaunchKernelGGL(sym_fill, dim3(g), dim3(kBlock), 0, s, n, (const int32_t *)A->rp, (const int32_t *)A->col,
                           (const float *)A->val32, (const int32_t *)S->rp_l, S->rp_u, S->col_u, S->val_u, S->col_l);
        h = hipGetLastError();
    }
    // the host copy of the row pointers must outlive the transfer
    if (h == hipSuccess) h = hipStreamSynchronize(s);
    if (h != hipSuccess) {
        sym_free(S);
        return hip_fail(h, "cfd_spmv_sym: build");
    }
    A->sym = S;
    return CFD_OK;
}

// y = A x from the symmetric storage.  Per row: the lower terms first, each
// value found as entry (j, i) among row j's upper entries (after its
// diagonal; symmetry guarantees it is there, the bound keeps the search in
// the row otherwise), then the diagonal and upper terms from the staged
// slab, all in ascending column order with one fused multiply-add each,
// as the full-CSR product does.
template <class VT>
__global__ void __launch_bounds__(kBlock) spmv_sym_kernel(const int32_t *__restrict__ rp_u,
                                                          const int32_t *__restrict__ col_u,
                                                          const float *__restrict__ val_u,
                                                          const int32_t *__restrict__ rp_l,
                                                          const int32_t *__restrict__ col_l, int64_t n,
                                                          const VT *__restrict__ x, VT *__restrict__ y) {
    typedef typename std::conditional<sizeof(VT) == 4, float, double>::type Acc;
    __shared__ __align__(16) int32_t s_col[kSlabLds];
    __shared__ __align__(16) float s_val[kSlabLds];
    csr_sweep<float>(rp_u, col_u, val_u, n, s_col, s_val, [&](int64_t i, int rs, int re) {
        Acc acc = Acc(0);
        for (int32_t e = rp_l[i]; e < rp_l[i + 1]; ++e) {
            const int32_t j = col_l[e];
            int32_t k = rp_u[j] + 1;
            const int32_t kend = rp_u[j + 1];
            while (k < kend && col_u[k] != (int32_t)i) ++k;
            if (k < kend) acc = fma(Acc(val_u[k]), Acc(x[j]), acc);
        }
        for (int e = rs; e < re; ++e) acc = fma(Acc(s_val[e]), Acc(x[s_col[e]]), acc);
        store_stream(y + i, (VT)acc);
    });
}

}  // namespace cfd

extern "C" int cfd_spmv_sym(cfd_csr_t A, int32_t precision, const void *x, void *y, void *stream) {
    if (!A || !x || !y) return fail(CFD_EINVAL, "cfd_spmv_sym: null argument");
    if (precision != CFD_PREC_FP64 && precision != CFD_PREC_MIXED)
        return fail(CFD_EINVAL, "cfd_spmv_sym: precision must be 0 (float64) or 1 (float32)");
    hipStream_t s = (hipStream_t)stream;
    int rc = sym_build(A, s);
    if (rc != CFD_OK) return rc;
    const SymStorage *S = (const SymStorage *)A->sym;
    const int G = grid_spmv(A->n, precision == CFD_PREC_FP64);
    if (precision == CFD_PREC_FP64)
        hipLaunchKernelGGL(spmv_sym_kernel<double>, dim3(G), dim3(kBlock), 0, s, (const int32_t *)S->rp_u,
                           (const int32_t *)S->col_u, (const float *)S->val_u, (const int32_t *)S->rp_l,
                           (const int32_t *)S->col_l, A->n, (const double *)x, (double *)y);
    else
        hipLaunchKernelGGL(spmv_sym_kernel<float>, dim3(G), dim3(kBlock), 0, s, (const int32_t *)S->rp_u,
                           (const int32_t *)S->col_u, (const float *)S->val_u, (const int32_t *)S->rp_l,
                           (const int32_t *)S->col_l, A->n, (const float *)x, (float *)y);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

namespace cfd {
double *scratch_partials(cfd_csr_t A);  // defined with the solver workspace
}

extern "C" int cfd_rhs_prepare(cfd_csr_t A, double *b, void *stream) {
    if (!A || !b) return fail(CFD_EINVAL, "cfd_rhs_prepare: null argument");
    double *part = scratch_partials(A);
    if (!part) return CFD_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const int G = grid_vec(A->n);
    hipLaunchKernelGGL(sum_kernel, dim3(G), dim3(kBlock), 0, s, (const double *)b, A->n, part);
    hipLaunchKernelGGL(center_kernel, dim3(G), dim3(kBlock), 0, s, b, A->n, A->pin, (const double *)part, G);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

// ---------------------------------------------------------------- allocation-free variant

namespace cfd {

// Partial sums of cfd_rhs_prepare_noalloc: a fixed device array instead of
// the matrix handle's workspace.  Every GPU the library runs on holds its own
// copy until the process ends; calls on one GPU share it (the last call's
// partial sums stay there), so calls that overlap on one GPU race.
constexpr int kNoAllocParts = 1024;  // 8 KiB
static __device__ __align__(256) double scratch[kNoAllocParts];

constexpr int kMaxDevices = 64;
static double *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device, looked up once per
// device (host code must not pass the symbol itself to a kernel).
static int scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(CFD_EINVAL, "cfd_rhs_prepare_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                     "cfd_rhs_prepare_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return CFD_OK;
}

}  // namespace cfd

extern "C" int cfd_rhs_prepare_noalloc(cfd_csr_t A, double *b, void *stream) {
    if (!A || !b) return fail(CFD_EINVAL, "cfd_rhs_prepare_noalloc: null argument");
    int dev = -1;
    CFD_HIP(hipGetDevice(&dev));
    if (dev != A->device)
        return fail(CFD_EINVAL, "cfd_rhs_prepare_noalloc: call with the matrix's device current");
    // the same grid, kernels and summation order as cfd_rhs_prepare
    const int G = grid_vec(A->n);
    if (G > kNoAllocParts)
        return fail(CFD_EINVAL, "cfd_rhs_prepare_noalloc: needs " + std::to_string(G) +
                                    " partial sums, more than the fixed scratch holds (" +
                                    std::to_string(kNoAllocParts) + ")");
    double *part = nullptr;
    int rc = scratch_address(dev, &part);
    if (rc != CFD_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(sum_kernel, dim3(G), dim3(kBlock), 0, s, (const double *)b, A->n, part);
    hipLaunchKernelGGL(center_kernel, dim3(G), dim3(kBlock), 0, s, b, A->n, A->pin, (const double *)part, G);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

extern "C" const char *cfd_last_error(void) { return cfd::g_err.c_str(); }
