// Learned warm start: a small 3-D convolutional network whose forward and
// backward passes run on the gfx950 matrix cores (bfloat16 operands, float32
// accumulation).
//
// Network: layers l = 0..L-1 of 3x3x3 convolutions with replicate padding
// and no bias, channels 1 -> 16 -> ... -> 16 -> 1, ReLU after all but the
// last.  Weights of a layer: W[t][ci][co], t = (dz+1)*9 + (dy+1)*3 + (dx+1).
// Activations are stored voxel-major with 16 channels contiguous (32 bytes
// per voxel, bfloat16).
//
// Forward (implicit GEMM): for 16 output voxels at a time one wave computes
// D[co][v] = sum_k A[co][k] B[k][v] with v_mfma_f32_16x16x32_bf16, where
// k enumerates (tap, input channel) pairs, two taps per 32-wide K step (14
// steps for 16 input channels, 1 step for the single-channel input layer),
// A = the layer's weights (pre-packed per lane), and B = the input values at
// the clamped neighbour of each voxel (a 16-byte read per lane from the
// input planes the workgroup stages in LDS as it marches along z).  The 16x16 accumulator holds four
// consecutive channels of one voxel per lane, so the output is written as one
// 8-byte (bf16) or 16-byte (float) store.
//
// Backward data: replicate padding is X_pad[v'] = X[clamp(v')] on the padded
// grid [-1, n]^3.  Its adjoint is computed in two steps: the same MFMA kernel
// in "full" mode produces dX_pad[v'] = sum_t dY[v' - d_t] W[t]^T (dY zero
// outside the grid) over the padded grid, then a fold kernel sums the padded
// cells that clamp to each voxel.
//
// Backward weights: dW[t][ci][co] = sum_v X[clamp(v + d_t)][ci] dY[v][co] is
// a GEMM with K = voxels; each workgroup marches its columns along z with
// X's halo planes and dY's plane in LDS, its waves accumulate a share of the
// 27 taps on the matrix cores, and it writes one partial sum, which two
// more kernels reduce in a fixed order (deterministic, no atomics).
#include "common.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace cfd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16;  // hidden channels (the matrix-core tile width)

__device__ inline uint16_t f2bf(float f) {
    const __bf16 h = (__bf16)f;  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

struct Geo {
    int nx, ny, nz;
    int64_t n;
};

__device__ inline int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

enum ConvMode { FWD = 0, FULL = 1 };

// Source voxel of output o (coordinates i, j, k of the output grid) through
// tap t, or -1 when it lies outside the input grid (full mode only).
template <int MODE>
__device__ inline int64_t conv_src(const Geo &g, int i, int j, int k, int t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    if (MODE == FWD) {
        const int a = clampi(i + dx, 0, g.nx - 1), b = clampi(j + dy, 0, g.ny - 1), c = clampi(k + dz, 0, g.nz - 1);
        return (int64_t)a + (int64_t)g.nx * ((int64_t)b + (int64_t)g.ny * c);
    } else {
        // output grid is the padded grid: cell (i, j, k) is v' = (i-1, j-1, k-1)
        const int a = i - 1 - dx, b = j - 1 - dy, c = k - 1 - dz;
        if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) return -1;
        return (int64_t)a + (int64_t)g.nx * ((int64_t)b + (int64_t)g.ny * c);
    }
}

// One convolution on the matrix cores.  CIN/COUT are the channel counts of
// this convolution (1 or 16); frag holds the packed weights (STEPS x 64 lanes
// x 8 bfloat16).  Output: float or bfloat16 (with optional ReLU), COUT
// channels per voxel of the output grid (the input grid, or the padded grid
// in full mode).
template <int CIN, int COUT, int MODE, bool OUT_BF16>
__global__ void __launch_bounds__(kBlock) conv_mfma(Geo g, const uint16_t *__restrict__ in,
                                                    const u16x8 *__restrict__ frag, void *__restrict__ out,
                                                    int relu) {
    constexpr int STEPS = CIN == 16 ? 14 : 1;
    const int lane = threadIdx.x & 63;
    const int nl = lane & 15, grp = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / 64);
    bf16x8 A[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) A[s] = __builtin_bit_cast(bf16x8, frag[s * 64 + lane]);
    const int ox = g.nx + (MODE == FULL ? 2 : 0), oy = g.ny + (MODE == FULL ? 2 : 0),
              oz = g.nz + (MODE == FULL ? 2 : 0);
    const int64_t nout = (int64_t)ox * oy * oz;
    const int64_t ntiles = (nout + 15) / 16;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        const int64_t o = tile * 16 + nl;
        const bool valid = o < nout;
        const int i = (int)(o % ox), j = (int)((o / ox) % oy), k = (int)(o / ((int64_t)ox * oy));
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
            if constexpr (CIN == 16) {
                const int t = 2 * s + (grp >> 1);
                const int64_t src = (valid && t < 27) ? conv_src<MODE>(g, i, j, k, t) : -1;
                if (src >= 0) b = *reinterpret_cast<const u16x8 *>(in + src * 16 + 8 * (grp & 1));
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int t = 8 * grp + e;
                    const int64_t src = (valid && t < 27) ? conv_src<MODE>(g, i, j, k, t) : -1;
                    if (src >= 0) b[e] = in[src];
                }
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s], __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
        }
        if (!valid) continue;
        if (relu) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = acc[q] > 0.f ? acc[q] : 0.f;
        }
        if constexpr (COUT == 16) {
            if constexpr (OUT_BF16) {
                u16x4 v = {f2bf(acc[0]), f2bf(acc[1]), f2bf(acc[2]), f2bf(acc[3])};
                *reinterpret_cast<u16x4 *>((uint16_t *)out + o * 16 + 4 * grp) = v;
            } else {
                *reinterpret_cast<f32x4 *>((float *)out + o * 16 + 4 * grp) = acc;
            }
        } else {
            if (grp == 0) {
                if constexpr (OUT_BF16) ((uint16_t *)out)[o] = f2bf(acc[0]);
                else ((float *)out)[o] = acc[0];
            }
        }
    }
}

// Forward convolution marching along z.  A work item is a column of
// kTX x kTY output voxels (one 16-voxel MFMA tile per y row, 4 rows per
// wave) over zc consecutive z planes.  The input planes z-1, z and z+1 of the
// column's halo ((kTX+2) x (kTY+2) voxels, replicate padding applied while
// loading) sit in a 3-slot LDS ring; plane z+2 is loaded into registers while
// plane z computes and is committed into the slot of plane z-1 afterwards.
// Each input plane is thus read once per column, plus the column's halo ring
// (18 x 18 / 16 x 16) and two boundary planes per z range, and every tap's B
// operand is a 16-byte LDS read, issued four steps ahead of its matrix
// instruction.  At 16 input channels those reads (1 KB per 16x16x32 step)
// bound the kernel: LDS delivers 128 bytes per clock per CU, half of what the
// matrix cores would consume at their full rate.  Work items run in XCD-contiguous
// ranges so neighbouring columns share their halo in one L2.
constexpr int kTX = 16, kTY = 16;
constexpr int kPX = kTX + 2, kPY = kTY + 2, kPlane = kPX * kPY;

template <int CIN>
struct PlaneRegs {
    // CIN = 16: a plane is kPlane * 2 16-byte chunks; CIN = 1: kPlane values
    static constexpr int kN = CIN == 16 ? (kPlane * 2 + kBlock - 1) / kBlock : (kPlane + kBlock - 1) / kBlock;
    typedef typename std::conditional<CIN == 16, u16x8, uint16_t>::type T;
    T v[kN];
};

template <int CIN, int COUT, bool OUT_BF16>
__global__ void __launch_bounds__(kBlock) conv_fwd_z(Geo g, int zc, const uint16_t *__restrict__ in,
                                                     const u16x8 *__restrict__ frag, void *__restrict__ out,
                                                     int relu) {
    constexpr int STEPS = CIN == 16 ? 14 : 1;
    __shared__ __align__(16) uint16_t s_in[3 * kPlane * CIN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nl = lane & 15, grp = lane >> 4;
    bf16x8 A[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) A[s] = __builtin_bit_cast(bf16x8, frag[s * 64 + lane]);
    const int ntx = (g.nx + kTX - 1) / kTX, nty = (g.ny + kTY - 1) / kTY, nzc = (g.nz + zc - 1) / zc;
    const TileRange tr = tile_range((int64_t)ntx * nty * nzc);
    for (int64_t item = tr.first; item < tr.end; item += tr.step) {
        const int x0 = (int)(item % ntx) * kTX, y0 = (int)((item / ntx) % nty) * kTY;
        const int z0 = (int)(item / ((int64_t)ntx * nty)) * zc;
        const int z1 = min(z0 + zc, g.nz);
        // halo plane p (clamped into the grid) into registers / into its slot
        auto load = [&](int p, PlaneRegs<CIN> &R) {
            const int64_t zoff = (int64_t)g.nx * g.ny * clampi(p, 0, g.nz - 1);
#pragma unroll
            for (int q = 0; q < PlaneRegs<CIN>::kN; ++q) {
                const int c = threadIdx.x + q * kBlock;
                const int h = CIN == 16 ? (c >> 1) : c;
                const int hh = min(h, kPlane - 1);
                const int hx = hh % kPX, hy = hh / kPX;
                const int64_t src = zoff + clampi(x0 + hx - 1, 0, g.nx - 1) +
                                    (int64_t)g.nx * clampi(y0 + hy - 1, 0, g.ny - 1);
                if constexpr (CIN == 16) R.v[q] = *reinterpret_cast<const u16x8 *>(in + src * 16 + 8 * (c & 1));
                else R.v[q] = in[src];
            }
        };
        auto commit = [&](int p, const PlaneRegs<CIN> &R) {
            const int slot = (p + 3) % 3;
#pragma unroll
            for (int q = 0; q < PlaneRegs<CIN>::kN; ++q) {
                const int c = threadIdx.x + q * kBlock;
                if constexpr (CIN == 16) {
                    if (c < kPlane * 2) reinterpret_cast<u16x8 *>(s_in)[slot * kPlane * 2 + c] = R.v[q];
                } else {
                    if (c < kPlane) s_in[slot * kPlane + c] = R.v[q];
                }
            }
        };
        PlaneRegs<CIN> R;
        for (int p = z0 - 1; p <= z0 + 1; ++p) {
            load(p, R);
            commit(p, R);
        }
        load(z0 + 2, R);
        __syncthreads();
        for (int z = z0; z < z1; ++z) {
            // 16 tiles (rows of 16 voxels along x), 4 per wave
            for (int ty = wave; ty < kTY; ty += kBlock / 64) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                u16x8 bb[STEPS];
                if constexpr (CIN == 16) {
#pragma unroll
                    for (int s = 0; s < STEPS; ++s) {
                        // tap 27 (the padding half of the last step) reads tap 26's
                        // operand; its weights are zero
                        const int t = min(2 * s + (grp >> 1), 26);
                        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                        const int slot = (z + dz + 3) % 3;
                        const int h = (nl + 1 + dx) + kPX * (ty + 1 + dy);
                        bb[s] = reinterpret_cast<const u16x8 *>(s_in)[(slot * kPlane + h) * 2 + (grp & 1)];
                    }
                }
#pragma unroll
                for (int s = 0; s < STEPS; ++s) {
                    u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
                    if constexpr (CIN == 16) {
                        b = bb[s];
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int t = 8 * grp + e;
                            if (t < 27) {
                                const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                                const int slot = (z + dz + 3) % 3;
                                b[e] = s_in[slot * kPlane + (nl + 1 + dx) + kPX * (ty + 1 + dy)];
                            }
                        }
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s], __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
                }
                if constexpr (CIN == 16) {
                    // keep 4 operand reads in flight ahead of the matrix ops
                    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
                    for (int s = 0; s < STEPS - 4; ++s) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
                }
                const int x = x0 + nl, y = y0 + ty;
                if (x >= g.nx || y >= g.ny) continue;
                const int64_t o = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
                if (relu) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] = acc[q] > 0.f ? acc[q] : 0.f;
                }
                if constexpr (COUT == 16) {
                    if constexpr (OUT_BF16) {
                        u16x4 v = {f2bf(acc[0]), f2bf(acc[1]), f2bf(acc[2]), f2bf(acc[3])};
                        *reinterpret_cast<u16x4 *>((uint16_t *)out + o * 16 + 4 * grp) = v;
                    } else {
                        *reinterpret_cast<f32x4 *>((float *)out + o * 16 + 4 * grp) = acc;
                    }
                } else if (grp == 0) {
                    if constexpr (OUT_BF16) ((uint16_t *)out)[o] = f2bf(acc[0]);
                    else ((float *)out)[o] = acc[0];
                }
            }
            __syncthreads();  // every wave is done with the slot of plane z-1
            if (z + 1 < z1) {
                commit(z + 2, R);
                load(z + 3, R);
            }
            __syncthreads();
        }
    }
}

// Pack a layer's float32 weights W[t][cin_f][cout_f] into per-lane MFMA
// fragments for a convolution with CIN_C input and COUT_C output channels.
// trans = 0: forward (CIN_C = cin_f); trans = 1: backward data (the
// convolution maps cout_f channels to cin_f channels).
template <int CIN_C>
__global__ void pack_weights(const float *__restrict__ W, int cin_f, int cout_f, int trans, uint16_t *__restrict__ frag) {
    constexpr int STEPS = CIN_C == 16 ? 14 : 1;
    const int cin_c = trans ? cout_f : cin_f, cout_c = trans ? cin_f : cout_f;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < STEPS * 64 * 8; id += gridDim.x * blockDim.x) {
        const int e = id & 7, lane = (id >> 3) & 63, s = id >> 9;
        const int grp = lane >> 4, co = lane & 15;
        int t, ci;
        if (CIN_C == 16) {
            t = 2 * s + (grp >> 1);
            ci = 8 * (grp & 1) + e;
        } else {
            t = 8 * grp + e;
            ci = 0;
        }
        float w = 0.f;
        if (t < 27 && ci < cin_c && co < cout_c)
            w = trans ? W[((int64_t)t * cin_f + co) * cout_f + ci] : W[((int64_t)t * cin_f + ci) * cout_f + co];
        frag[id] = f2bf(w);
    }
}

// dX[v][c] = sum of dX_pad over the padded cells that clamp to v; optional
// ReLU mask (act > 0) of the layer input; float or bfloat16 output.
template <int C, bool MASK, bool OUT_BF16>
__global__ void __launch_bounds__(kBlock) fold_kernel(Geo g, const float *__restrict__ dxp,
                                                      const uint16_t *__restrict__ act, void *__restrict__ out) {
    const int px = g.nx + 2, py = g.ny + 2;
    for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < g.n * C; id += (int64_t)gridDim.x * kBlock) {
        const int64_t v = id / C;
        const int c = (int)(id % C);
        const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((int64_t)g.nx * g.ny));
        // padded coordinates (+1) that clamp to i: i itself, the low halo if
        // i == 0, the high halo if i == nx-1
        int xs[3], ys[3], zs[3], nxs = 0, nys = 0, nzs = 0;
        xs[nxs++] = i + 1;
        if (i == 0) xs[nxs++] = 0;
        if (i == g.nx - 1) xs[nxs++] = g.nx + 1;
        ys[nys++] = j + 1;
        if (j == 0) ys[nys++] = 0;
        if (j == g.ny - 1) ys[nys++] = g.ny + 1;
        zs[nzs++] = k + 1;
        if (k == 0) zs[nzs++] = 0;
        if (k == g.nz - 1) zs[nzs++] = g.nz + 1;
        float s = 0.f;
        for (int c3 = 0; c3 < nzs; ++c3)
            for (int b3 = 0; b3 < nys; ++b3)
                for (int a3 = 0; a3 < nxs; ++a3)
                    s += dxp[((int64_t)xs[a3] + (int64_t)px * ((int64_t)ys[b3] + (int64_t)py * zs[c3])) * C + c];
        if (MASK && !(bf2f(act[id]) > 0.f)) s = 0.f;
        if (OUT_BF16) ((uint16_t *)out)[id] = f2bf(s);
        else ((float *)out)[id] = s;
    }
}

// Weight gradient marching along z (the columns and z ranges of
// conv_fwd_z).  dW[t][ci][co] = sum_v X[clamp(v + d_t)][ci] dY[v][co] is an
// MFMA product with K = voxels: a 32-voxel block is two rows of the 16 x 16
// tile, and lane (m, grp) holds its voxels 8 grp .. 8 grp + 7.  The halo
// planes of X sit in a 3-slot LDS ring (the next one loaded into registers
// while a plane computes), dY's plane in LDS (zero outside the grid); both
// operands are read from LDS.  Wave w owns the taps w, w + 4, ... and
// accumulates them over its workgroup's items; each workgroup writes one
// partial dW, which wgrad_reduce_* sum in a fixed order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(kBlock) wgrad_z(Geo g, int zc, const uint16_t *__restrict__ in,
                                                  const uint16_t *__restrict__ dy, float *__restrict__ part) {
    constexpr int kTaps = 7;  // taps per wave: wave + 4 j < 27
    __shared__ __align__(16) uint16_t s_in[3 * kPlane * CIN];
    __shared__ __align__(16) uint16_t s_dy[kTX * kTY * COUT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ml = lane & 15, grp = lane >> 4;
    f32x4 acc[kTaps];
#pragma unroll
    for (int j = 0; j < kTaps; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ntx = (g.nx + kTX - 1) / kTX, nty = (g.ny + kTY - 1) / kTY, nzc = (g.nz + zc - 1) / zc;
    const TileRange tr = tile_range((int64_t)ntx * nty * nzc);
    for (int64_t item = tr.first; item < tr.end; item += tr.step) {
        const int x0 = (int)(item % ntx) * kTX, y0 = (int)((item / ntx) % nty) * kTY;
        const int z0 = (int)(item / ((int64_t)ntx * nty)) * zc;
        const int z1 = min(z0 + zc, g.nz);
        auto load = [&](int p, PlaneRegs<CIN> &R) {
            const int64_t zoff = (int64_t)g.nx * g.ny * clampi(p, 0, g.nz - 1);
#pragma unroll
            for (int q = 0; q < PlaneRegs<CIN>::kN; ++q) {
                const int c = threadIdx.x + q * kBlock;
                const int h = CIN == 16 ? (c >> 1) : c;
                const int hh = min(h, kPlane - 1);
                const int hx = hh % kPX, hy = hh / kPX;
                const int64_t src = zoff + clampi(x0 + hx - 1, 0, g.nx - 1) +
                                    (int64_t)g.nx * clampi(y0 + hy - 1, 0, g.ny - 1);
                if constexpr (CIN == 16) R.v[q] = *reinterpret_cast<const u16x8 *>(in + src * 16 + 8 * (c & 1));
                else R.v[q] = in[src];
            }
        };
        auto commit = [&](int p, const PlaneRegs<CIN> &R) {
            const int slot = (p + 3) % 3;
#pragma unroll
            for (int q = 0; q < PlaneRegs<CIN>::kN; ++q) {
                const int c = threadIdx.x + q * kBlock;
                if constexpr (CIN == 16) {
                    if (c < kPlane * 2) reinterpret_cast<u16x8 *>(s_in)[slot * kPlane * 2 + c] = R.v[q];
                } else {
                    if (c < kPlane) s_in[slot * kPlane + c] = R.v[q];
                }
            }
        };
        PlaneRegs<CIN> R;
        for (int p = z0 - 1; p <= z0 + 1; ++p) {
            load(p, R);
            commit(p, R);
        }
        load(z0 + 2, R);
        for (int z = z0; z < z1; ++z) {
            // dY of the tile's plane z, zero outside the grid
            if constexpr (COUT == 16) {
                for (int c = threadIdx.x; c < kTX * kTY * 2; c += kBlock) {
                    const int v = c >> 1, x = x0 + v % kTX, y = y0 + v / kTX;
                    u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
                    if (x < g.nx && y < g.ny)
                        val = *reinterpret_cast<const u16x8 *>(
                            dy + ((int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z)) * 16 + 8 * (c & 1));
                    reinterpret_cast<u16x8 *>(s_dy)[c] = val;
                }
            } else {
                for (int v = threadIdx.x; v < kTX * kTY; v += kBlock) {
                    const int x = x0 + v % kTX, y = y0 + v / kTX;
                    s_dy[v] = (x < g.nx && y < g.ny)
                                  ? dy[(int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z)]
                                  : (uint16_t)0;
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int kb = 0; kb < kTX * kTY / 32; ++kb) {
                u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int v = 32 * kb + 8 * grp + e;  // voxel of the tile, x fastest
                    if (ml < COUT) b[e] = s_dy[v * COUT + ml];
                }
                const bf16x8 B = __builtin_bit_cast(bf16x8, b);
#pragma unroll
                for (int j = 0; j < kTaps; ++j) {
                    const int t = wave + 4 * j;
                    if (t < 27) {
                        const int dx = t % 3 - 1, dyy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                        const int slot = (z + dz + 3) % 3;
                        u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int v = 32 * kb + 8 * grp + e;
                            const int h = (v % kTX + 1 + dx) + kPX * (v / kTX + 1 + dyy);
                            if (ml < CIN) a[e] = s_in[(slot * kPlane + h) * CIN + ml];
                        }
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), B, acc[j], 0,
                                                                         0, 0);
                    }
                }
            }
            __syncthreads();  // every wave is done with the slot of plane z-1 and with s_dy
            if (z + 1 < z1) {
                commit(z + 2, R);
                load(z + 3, R);
            }
            __syncthreads();
        }
    }
    // lane holds D[ci = 4 grp + q][co = ml] of each of its taps
    float *dst = part + (int64_t)blockIdx.x * (27 * CIN * COUT);
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
        const int t = wave + 4 * j;
        if (t >= 27) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ci = 4 * grp + q, co = ml;
            if (ci < CIN && co < COUT) dst[((int64_t)t * CIN + ci) * COUT + co] = acc[j][q];
        }
    }
}

// grad[i] (+)= sum over waves of part[w][i], in a fixed order: the waves in
// kWgradSeg contiguous segments, each summed in wave order by one thread per
// weight (consecutive weights in consecutive lanes, so the loads coalesce),
// then the segment sums in segment order.
constexpr int kWgradSeg = 64;
__global__ void wgrad_reduce_seg(const float *__restrict__ part, int64_t nwaves, int count,
                                 double *__restrict__ seg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t w0 = nwaves * blockIdx.y / kWgradSeg, w1 = nwaves * (blockIdx.y + 1) / kWgradSeg;
    double s = 0.0;
    for (int64_t w = w0; w < w1; ++w) s += part[w * count + i];
    seg[(int64_t)blockIdx.y * count + i] = s;
}

__global__ void wgrad_reduce(const double *__restrict__ seg, int count, float *__restrict__ grad, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s = 0.0;
    for (int k = 0; k < kWgradSeg; ++k) s += seg[(int64_t)k * count + i];
    grad[i] = accumulate ? grad[i] + (float)s : (float)s;
}

// Partial sums of squares of a float64 vector (for rms normalisation).
__global__ void __launch_bounds__(kBlock) sumsq_kernel(const double *__restrict__ b, int64_t n, double *__restrict__ part) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s = fma(b[i], b[i], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// act0 = bf16(b / s), s = rms(b) (0 input when b = 0).
__global__ void __launch_bounds__(kBlock) net_input_kernel(const double *__restrict__ b, int64_t n,
                                                           const double *__restrict__ part, int count,
                                                           uint16_t *__restrict__ act0) {
    __shared__ double red[kBlock / 64];
    const double s = sqrt(reduce_partials(part, count, red) / (double)n);
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        act0[i] = f2bf((float)(b[i] * inv));
}

// y = s * y32.
__global__ void __launch_bounds__(kBlock) net_output_kernel(const float *__restrict__ y32, int64_t n,
                                                            const double *__restrict__ part, int count,
                                                            double *__restrict__ y) {
    __shared__ double red[kBlock / 64];
    const double s = sqrt(reduce_partials(part, count, red) / (double)n);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = s * (double)y32[i];
}

__global__ void __launch_bounds__(kBlock) to_bf16_kernel(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ o) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        o[i] = f2bf(x[i]);
}

__global__ void __launch_bounds__(kBlock) from_bf16_kernel(const uint16_t *__restrict__ x, int64_t n, float *__restrict__ o) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        o[i] = bf2f(x[i]);
}

// dY = bf16(scale * (y - target)); partial sums of (y - target)^2.
__global__ void __launch_bounds__(kBlock) loss_grad_kernel(const float *__restrict__ y, const float *__restrict__ tgt,
                                                           int64_t n, float scale, uint16_t *__restrict__ dy,
                                                           double *__restrict__ part) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float d = y[i] - tgt[i];
        dy[i] = f2bf(scale * d);
        s = fma((double)d, (double)d, s);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void sum_partials_kernel(const double *__restrict__ part, int count, double *__restrict__ out, int accumulate) {
    __shared__ double red[kBlock / 64];
    const double s = reduce_partials(part, count, red);
    if (threadIdx.x == 0) *out = accumulate ? *out + s : s;
}

// Training pairs (input = b / rms(b), target = (p - mean p) / rms(p - mean p)):
// partial sums of b^2 and of p (first pass), of (p - mean p)^2 (second pass).
__global__ void __launch_bounds__(kBlock) pair_sums_kernel(const double *__restrict__ b, const double *__restrict__ p,
                                                           int64_t n, double *__restrict__ part_bb,
                                                           double *__restrict__ part_p) {
    __shared__ double red[kBlock / 64];
    double bb = 0.0, sp = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        bb = fma(b[i], b[i], bb);
        sp += p[i];
    }
    bb = block_sum(bb, red);
    sp = block_sum(sp, red);
    if (threadIdx.x == 0) {
        part_bb[blockIdx.x] = bb;
        part_p[blockIdx.x] = sp;
    }
}

__global__ void __launch_bounds__(kBlock) pair_var_kernel(const double *__restrict__ p, int64_t n,
                                                          const double *__restrict__ part_p, int count,
                                                          double *__restrict__ part_pp) {
    __shared__ double red[kBlock / 64];
    const double mean = reduce_partials(part_p, count, red) / (double)n;
    double pp = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double d = p[i] - mean;
        pp = fma(d, d, pp);
    }
    pp = block_sum(pp, red);
    if (threadIdx.x == 0) part_pp[blockIdx.x] = pp;
}

__global__ void __launch_bounds__(kBlock) pair_write_kernel(const double *__restrict__ b, const double *__restrict__ p,
                                                            int64_t n, const double *__restrict__ part, int count,
                                                            float *__restrict__ input, float *__restrict__ target) {
    __shared__ double red[kBlock / 64];
    const double sb = sqrt(reduce_partials(part, count, red) / (double)n);
    const double mean = reduce_partials(part + count, count, red) / (double)n;
    const double sp = sqrt(reduce_partials(part + 2 * count, count, red) / (double)n);
    const double ib = sb > 0.0 ? 1.0 / sb : 0.0, ip = sp > 0.0 ? 1.0 / sp : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        input[i] = (float)(b[i] * ib);
        target[i] = (float)((p[i] - mean) * ip);
    }
}

// Adam (Kingma & Ba 2015) on float32 master weights.
__global__ void adam_kernel(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ gr, int count, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float g = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ---------------------------------------------------------------- host side

// Work items and grid of the z-marching kernels (conv_fwd_z, wgrad_z): z
// ranges sized so the items about fill the resident workgroups.
struct ZGrid {
    int zc, blocks;
};
template <class K>
static ZGrid zgrid(const Geo &g, K kernel) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    Device d;
    if (device_info(&d) != CFD_OK) d.cus = 256;
    const int64_t resident = (int64_t)per_cu * d.cus;
    const int64_t ncol = (int64_t)((g.nx + kTX - 1) / kTX) * ((g.ny + kTY - 1) / kTY);
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(g.nz, (resident + ncol - 1) / ncol));
    ZGrid z;
    z.zc = (int)((g.nz + want - 1) / want);
    const int64_t items = ncol * ((g.nz + z.zc - 1) / z.zc);
    z.blocks = (int)std::min<int64_t>(items, resident);
    if (z.blocks > kXcd) z.blocks -= z.blocks % kXcd;
    return z;
}

static int grid_waves(int64_t work_items_per_wave_units) {
    Device d;
    if (device_info(&d) != CFD_OK) d.cus = 256;
    const int64_t want = (work_items_per_wave_units + 3) / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)d.cus * 8));
}

template <int CIN, int COUT, int MODE, bool OUT_BF16>
static void launch_conv(const Geo &g, const uint16_t *in, const uint16_t *frag, void *out, int relu, hipStream_t s) {
    if constexpr (MODE == FWD) {
        const ZGrid z = zgrid(g, conv_fwd_z<CIN, COUT, OUT_BF16>);
        hipLaunchKernelGGL((conv_fwd_z<CIN, COUT, OUT_BF16>), dim3(z.blocks), dim3(kBlock), 0, s, g, z.zc, in,
                           (const u16x8 *)frag, out, relu);
        return;
    }
    const int64_t nout = (int64_t)(g.nx + (MODE == FULL ? 2 : 0)) * (g.ny + (MODE == FULL ? 2 : 0)) *
                         (g.nz + (MODE == FULL ? 2 : 0));
    const int blocks = grid_waves((nout + 15) / 16);
    hipLaunchKernelGGL((conv_mfma<CIN, COUT, MODE, OUT_BF16>), dim3(blocks), dim3(kBlock), 0, s, g, in,
                       (const u16x8 *)frag, out, relu);
}

static void launch_pack(const float *W, int cin_f, int cout_f, int trans, uint16_t *frag, hipStream_t s) {
    const int cin_c = trans ? cout_f : cin_f;
    if (cin_c == 16) hipLaunchKernelGGL(pack_weights<16>, dim3(28), dim3(256), 0, s, W, cin_f, cout_f, trans, frag);
    else hipLaunchKernelGGL(pack_weights<1>, dim3(2), dim3(256), 0, s, W, cin_f, cout_f, trans, frag);
}

// Partial weight gradients: at most this many (one per workgroup of wgrad_z).
static int64_t wgrad_parts(int64_t) {
    Device d;
    if (device_info(&d) != CFD_OK) d.cus = 256;
    return (int64_t)d.cus * 8;
}

// Floats of the partial-sum buffer launch_wgrad needs for `count` weights:
// one partial per workgroup, then kWgradSeg segment sums (doubles).
static int64_t wgrad_part_floats(int64_t n, int count) {
    return wgrad_parts(n) * count + 2 * (int64_t)kWgradSeg * count + 2;
}

template <int CIN, int COUT>
static void launch_wgrad(const Geo &g, const uint16_t *x, const uint16_t *dy, float *part, float *grad, int accumulate,
                         hipStream_t s) {
    const ZGrid z = zgrid(g, wgrad_z<CIN, COUT>);
    const int64_t nparts = std::min<int64_t>(z.blocks, wgrad_parts(g.n));
    hipLaunchKernelGGL((wgrad_z<CIN, COUT>), dim3(nparts), dim3(kBlock), 0, s, g, z.zc, x, dy, part);
    const int count = 27 * CIN * COUT;
    // segment sums after the partials, 8-byte aligned
    double *seg = reinterpret_cast<double *>(part + ((nparts * count + 1) & ~(int64_t)1));
    hipLaunchKernelGGL(wgrad_reduce_seg, dim3((count + 255) / 256, kWgradSeg), dim3(256), 0, s, (const float *)part,
                       nparts, count, seg);
    hipLaunchKernelGGL(wgrad_reduce, dim3((count + 255) / 256), dim3(256), 0, s, (const double *)seg, count, grad,
                       accumulate);
}

static int frag_elems(int cin_c) { return (cin_c == 16 ? 14 : 1) * 64 * 8; }

}  // namespace cfd

struct cfd_net {
    int C = 16, L = 4;
    int64_t count = 0;
    std::vector<int> cin, cout;
    std::vector<int64_t> off;        // parameter offset per layer
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *ffrag = nullptr, *bfrag = nullptr;  // forward / backward-data fragments, 14*64*8 per layer
    bool dirty = true;
    int64_t t = 0;                   // Adam step
    // activation buffers (sized for n)
    int64_t n = 0, npad = 0;
    uint16_t *act0 = nullptr;
    std::vector<uint16_t *> h;       // h[l] = output of layer l (l = 0..L-2), n*16 bf16
    float *y32 = nullptr;
    uint16_t *dy = nullptr;          // n bf16
    uint16_t *dh[2] = {nullptr, nullptr};
    float *dxp = nullptr;            // padded * 16 float
    float *wpart = nullptr;
    int64_t wpart_elems = 0;
    double *part = nullptr;          // reductions
    double *loss = nullptr;          // device scalar
    int gpart = 0;
};

namespace cfd {

static void net_free_acts(cfd_net *N) {
    if (N->act0) (void)hipFree(N->act0);
    for (auto p : N->h) if (p) (void)hipFree(p);
    N->h.clear();
    if (N->y32) (void)hipFree(N->y32);
    if (N->dy) (void)hipFree(N->dy);
    for (int i = 0; i < 2; ++i) if (N->dh[i]) (void)hipFree(N->dh[i]);
    if (N->dxp) (void)hipFree(N->dxp);
    if (N->wpart) (void)hipFree(N->wpart);
    N->act0 = nullptr;
    N->y32 = nullptr;
    N->dy = nullptr;
    N->dh[0] = N->dh[1] = nullptr;
    N->dxp = nullptr;
    N->wpart = nullptr;
    N->n = 0;
}

static int net_ensure(cfd_net *N, const Geo &g, bool train) {
    const int64_t npad = (int64_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    const bool need_train = train && !N->dxp;
    if (N->n == g.n && N->npad == npad && !need_train) return CFD_OK;
    const bool keep_train = train || (N->dxp != nullptr);
    net_free_acts(N);
    N->n = g.n;
    N->npad = npad;
    CFD_HIP(hipMalloc(&N->act0, sizeof(uint16_t) * g.n));
    N->h.assign(N->L - 1, nullptr);
    for (int l = 0; l < N->L - 1; ++l) CFD_HIP(hipMalloc(&N->h[l], sizeof(uint16_t) * g.n * kC));
    CFD_HIP(hipMalloc(&N->y32, sizeof(float) * g.n));
    if (keep_train) {
        CFD_HIP(hipMalloc(&N->dy, sizeof(uint16_t) * g.n));
        for (int i = 0; i < 2; ++i) CFD_HIP(hipMalloc(&N->dh[i], sizeof(uint16_t) * g.n * kC));
        CFD_HIP(hipMalloc(&N->dxp, sizeof(float) * npad * kC));
        N->wpart_elems = wgrad_part_floats(g.n, 27 * kC * kC);
        CFD_HIP(hipMalloc(&N->wpart, sizeof(float) * N->wpart_elems));
    }
    return CFD_OK;
}

static void net_pack(cfd_net *N, hipStream_t s) {
    if (!N->dirty) return;
    for (int l = 0; l < N->L; ++l) {
        launch_pack(N->theta + N->off[l], N->cin[l], N->cout[l], 0, N->ffrag + (int64_t)l * 14 * 64 * 8, s);
        launch_pack(N->theta + N->off[l], N->cin[l], N->cout[l], 1, N->bfrag + (int64_t)l * 14 * 64 * 8, s);
    }
    N->dirty = false;
}

// Forward pass from the bf16 input act0; layer outputs in h[], final float
// output in y32.
static void net_forward_acts(cfd_net *N, const Geo &g, hipStream_t s) {
    const uint16_t *in = N->act0;
    for (int l = 0; l < N->L; ++l) {
        const uint16_t *fr = N->ffrag + (int64_t)l * 14 * 64 * 8;
        const bool last = l == N->L - 1;
        if (l == 0) {
            launch_conv<1, 16, FWD, true>(g, in, fr, N->h[0], 1, s);
        } else if (!last) {
            launch_conv<16, 16, FWD, true>(g, in, fr, N->h[l], 1, s);
        } else {
            launch_conv<16, 1, FWD, false>(g, in, fr, N->y32, 0, s);
        }
        if (!last) in = N->h[l];
    }
}

static int grid1(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
}

// Backward pass for one sample whose forward activations are in place and
// whose output gradient (bf16) is in dy; adds the weight gradients to grad.
static void net_backward(cfd_net *N, const Geo &g, hipStream_t s) {
    const uint16_t *gout = N->dy;  // gradient w.r.t. the output of layer l
    int cur = 0;
    const int gb = grid1(g.n * kC);
    for (int l = N->L - 1; l >= 0; --l) {
        const uint16_t *xin = l == 0 ? N->act0 : N->h[l - 1];
        float *gw = N->grad + N->off[l];
        const int cin = N->cin[l], cout = N->cout[l];
        if (cin == 16 && cout == 1) launch_wgrad<16, 1>(g, xin, gout, N->wpart, gw, 1, s);
        else if (cin == 16) launch_wgrad<16, 16>(g, xin, gout, N->wpart, gw, 1, s);
        else launch_wgrad<1, 16>(g, xin, gout, N->wpart, gw, 1, s);
        if (l == 0) break;
        // dX_pad over the padded grid, then fold with the ReLU mask of h[l-1]
        const uint16_t *bf = N->bfrag + (int64_t)l * 14 * 64 * 8;
        if (cout == 1) launch_conv<1, 16, FULL, false>(g, gout, bf, N->dxp, 0, s);
        else launch_conv<16, 16, FULL, false>(g, gout, bf, N->dxp, 0, s);
        hipLaunchKernelGGL((fold_kernel<16, true, true>), dim3(gb), dim3(kBlock), 0, s, g, (const float *)N->dxp,
                           (const uint16_t *)N->h[l - 1], (void *)N->dh[cur]);
        gout = N->dh[cur];
        cur ^= 1;
    }
}

int net_predict(cfd_net_t N, const cfd_grid *grid, const double *b, double *y, hipStream_t s) {
    const Geo g{grid->nx, grid->ny, grid->nz, (int64_t)grid->nx * grid->ny * grid->nz};
    int rc = net_ensure(N, g, false);
    if (rc != CFD_OK) return rc;
    net_pack(N, s);
    const int G = grid1(g.n);
    hipLaunchKernelGGL(sumsq_kernel, dim3(G), dim3(kBlock), 0, s, b, g.n, N->part);
    hipLaunchKernelGGL(net_input_kernel, dim3(G), dim3(kBlock), 0, s, b, g.n, (const double *)N->part, G, N->act0);
    net_forward_acts(N, g, s);
    hipLaunchKernelGGL(net_output_kernel, dim3(G), dim3(kBlock), 0, s, (const float *)N->y32, g.n,
                       (const double *)N->part, G, y);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

static int net_grad_impl(cfd_net_t N, const cfd_grid *grid, int32_t batch, const float *input, const float *target,
                         float *loss_out, hipStream_t s) {
    if (!N || !grid || !input || !target || batch < 1) return fail(CFD_EINVAL, "cfd_net: bad argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(CFD_EINVAL, "cfd_net: bad grid");
    const Geo g{grid->nx, grid->ny, grid->nz, (int64_t)grid->nx * grid->ny * grid->nz};
    int rc = net_ensure(N, g, true);
    if (rc != CFD_OK) return rc;
    net_pack(N, s);
    CFD_HIP(hipMemsetAsync(N->grad, 0, sizeof(float) * N->count, s));
    const int G = grid1(g.n);
    const float scale = 2.0f / (float)((double)batch * (double)g.n);
    for (int bi = 0; bi < batch; ++bi) {
        hipLaunchKernelGGL(to_bf16_kernel, dim3(G), dim3(kBlock), 0, s, input + (int64_t)bi * g.n, g.n, N->act0);
        net_forward_acts(N, g, s);
        hipLaunchKernelGGL(loss_grad_kernel, dim3(G), dim3(kBlock), 0, s, (const float *)N->y32,
                           target + (int64_t)bi * g.n, g.n, scale, N->dy, N->part);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, (const double *)N->part, G, N->loss,
                           bi > 0 ? 1 : 0);
        net_backward(N, g, s);
    }
    CFD_HIP(hipGetLastError());
    double l = 0.0;
    CFD_HIP(hipMemcpyAsync(&l, N->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    CFD_HIP(hipStreamSynchronize(s));
    if (loss_out) *loss_out = (float)(l / ((double)batch * (double)g.n));
    return CFD_OK;
}

}  // namespace cfd

using namespace cfd;

extern "C" int64_t cfd_net_param_count(int32_t channels, int32_t layers) {
    if (channels < 1 || layers < 2) return 0;
    return 27LL * ((int64_t)channels * 2 + (int64_t)(layers - 2) * channels * channels);
}

extern "C" int cfd_net_create(int32_t channels, int32_t layers, const float *init, cfd_net_t *out) {
    if (!out) return fail(CFD_EINVAL, "cfd_net_create: null output");
    *out = nullptr;
    if (channels != kC) return fail(CFD_EINVAL, "cfd_net_create: only 16 channels are supported");
    if (layers < 2 || layers > 16) return fail(CFD_EINVAL, "cfd_net_create: layers must be in [2, 16]");
    cfd_net *N = new cfd_net();
    N->C = channels;
    N->L = layers;
    int64_t off = 0;
    for (int l = 0; l < layers; ++l) {
        const int ci = l == 0 ? 1 : kC, co = l == layers - 1 ? 1 : kC;
        N->cin.push_back(ci);
        N->cout.push_back(co);
        N->off.push_back(off);
        off += 27LL * ci * co;
    }
    N->count = off;
    hipError_t e = hipMalloc(&N->theta, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&N->m, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&N->v, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&N->grad, sizeof(float) * off);
    if (e == hipSuccess) e = hipMalloc(&N->ffrag, sizeof(uint16_t) * 14 * 64 * 8 * layers);
    if (e == hipSuccess) e = hipMalloc(&N->bfrag, sizeof(uint16_t) * 14 * 64 * 8 * layers);
    if (e == hipSuccess) e = hipMalloc(&N->part, sizeof(double) * 4096);
    if (e == hipSuccess) e = hipMalloc(&N->loss, sizeof(double));
    if (e == hipSuccess) e = hipMemset(N->m, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipMemset(N->v, 0, sizeof(float) * off);
    if (e == hipSuccess) e = init ? hipMemcpy(N->theta, init, sizeof(float) * off, hipMemcpyHostToDevice)
                                  : hipMemset(N->theta, 0, sizeof(float) * off);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "cfd_net_create");
        cfd_net_destroy(N);
        return rc;
    }
    *out = N;
    return CFD_OK;
}

extern "C" void cfd_net_destroy(cfd_net_t N) {
    if (!N) return;
    net_free_acts(N);
    float *ff[] = {N->theta, N->m, N->v, N->grad};
    for (float *p : ff) if (p) (void)hipFree(p);
    if (N->ffrag) (void)hipFree(N->ffrag);
    if (N->bfrag) (void)hipFree(N->bfrag);
    if (N->part) (void)hipFree(N->part);
    if (N->loss) (void)hipFree(N->loss);
    delete N;
}

extern "C" int cfd_net_forward(cfd_net_t N, const cfd_grid *grid, const double *b, double *y, void *stream) {
    if (!N || !grid || !b || !y) return fail(CFD_EINVAL, "cfd_net_forward: null argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(CFD_EINVAL, "cfd_net_forward: bad grid");
    return net_predict(N, grid, b, y, (hipStream_t)stream);
}

extern "C" int cfd_net_gradient(cfd_net_t N, const cfd_grid *grid, int32_t batch, const float *input,
                                const float *target, float *grad_host, float *loss, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    int rc = net_grad_impl(N, grid, batch, input, target, loss, s);
    if (rc != CFD_OK) return rc;
    if (grad_host) CFD_HIP(hipMemcpy(grad_host, N->grad, sizeof(float) * N->count, hipMemcpyDeviceToHost));
    return CFD_OK;
}

extern "C" int cfd_net_train_step(cfd_net_t N, const cfd_grid *grid, int32_t batch, const float *input,
                                  const float *target, float lr, float *loss, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    int rc = net_grad_impl(N, grid, batch, input, target, loss, s);
    if (rc != CFD_OK) return rc;
    N->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)N->t)), c2 = (float)(1.0 - std::pow(b2, (double)N->t));
    hipLaunchKernelGGL(adam_kernel, dim3((N->count + 255) / 256), dim3(256), 0, s, N->theta, N->m, N->v,
                       (const float *)N->grad, (int)N->count, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    CFD_HIP(hipGetLastError());
    N->dirty = true;
    CFD_HIP(hipStreamSynchronize(s));
    return CFD_OK;
}

extern "C" int cfd_net_training_pair(cfd_net_t N, const cfd_grid *grid, const double *b, const double *p,
                                     float *input, float *target, void *stream) {
    if (!N || !grid || !b || !p || !input || !target) return fail(CFD_EINVAL, "cfd_net_training_pair: null argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(CFD_EINVAL, "cfd_net_training_pair: empty grid");
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    hipStream_t s = (hipStream_t)stream;
    const int G = std::min(grid1(n), 1024);  // three partial-sum arrays in the 4096-entry scratch
    double *part = N->part;
    hipLaunchKernelGGL(pair_sums_kernel, dim3(G), dim3(kBlock), 0, s, b, p, n, part, part + G);
    hipLaunchKernelGGL(pair_var_kernel, dim3(G), dim3(kBlock), 0, s, p, n, (const double *)(part + G), G, part + 2 * G);
    hipLaunchKernelGGL(pair_write_kernel, dim3(G), dim3(kBlock), 0, s, b, p, n, (const double *)part, G, input, target);
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

extern "C" int cfd_net_get_params(cfd_net_t N, float *host_buf, int64_t count) {
    if (!N || !host_buf || count != N->count) return fail(CFD_EINVAL, "cfd_net_get_params: bad argument");
    CFD_HIP(hipDeviceSynchronize());
    CFD_HIP(hipMemcpy(host_buf, N->theta, sizeof(float) * count, hipMemcpyDeviceToHost));
    return CFD_OK;
}

extern "C" int cfd_net_set_params(cfd_net_t N, const float *host_buf, int64_t count) {
    if (!N || !host_buf || count != N->count) return fail(CFD_EINVAL, "cfd_net_set_params: bad argument");
    CFD_HIP(hipDeviceSynchronize());
    CFD_HIP(hipMemcpy(N->theta, host_buf, sizeof(float) * count, hipMemcpyHostToDevice));
    N->dirty = true;
    return CFD_OK;
}

// ---------------------------------------------------------------- kernel-level entry points

static int conv_args(const cfd_grid *grid, int32_t cin, int32_t cout, Geo *g) {
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(CFD_EINVAL, "conv3d: bad grid");
    if ((cin != 1 && cin != 16) || (cout != 1 && cout != 16) || (cin == 1 && cout == 1))
        return fail(CFD_EINVAL, "conv3d: channels must be 1 or 16 (not both 1)");
    *g = Geo{grid->nx, grid->ny, grid->nz, (int64_t)grid->nx * grid->ny * grid->nz};
    return CFD_OK;
}

// float32 copy of bf16 weights + packed fragments in one stream-ordered
// allocation.
static int conv_weights(const uint16_t *w, int cin, int cout, int trans, hipStream_t s, void **mem, uint16_t **frag) {
    const int64_t cnt = 27LL * cin * cout;
    const size_t fbytes = sizeof(uint16_t) * frag_elems(16);
    CFD_HIP(hipMallocAsync(mem, sizeof(float) * cnt + fbytes, s));
    float *wf = (float *)*mem;
    *frag = (uint16_t *)((char *)*mem + sizeof(float) * cnt);
    hipLaunchKernelGGL(from_bf16_kernel, dim3(grid1(cnt)), dim3(kBlock), 0, s, w, cnt, wf);
    launch_pack(wf, cin, cout, trans, *frag, s);
    return CFD_OK;
}

extern "C" int cfd_conv3d_forward(const cfd_grid *grid, int32_t cin, int32_t cout, const uint16_t *x,
                                  const uint16_t *w, float *y, int32_t relu, void *stream) {
    Geo g;
    int rc = conv_args(grid, cin, cout, &g);
    if (rc != CFD_OK) return rc;
    if (!x || !w || !y) return fail(CFD_EINVAL, "conv3d: null pointer");
    hipStream_t s = (hipStream_t)stream;
    void *mem;
    uint16_t *frag;
    rc = conv_weights(w, cin, cout, 0, s, &mem, &frag);
    if (rc != CFD_OK) return rc;
    if (cin == 1) launch_conv<1, 16, FWD, false>(g, x, frag, y, relu, s);
    else if (cout == 16) launch_conv<16, 16, FWD, false>(g, x, frag, y, relu, s);
    else launch_conv<16, 1, FWD, false>(g, x, frag, y, relu, s);
    CFD_HIP(hipFreeAsync(mem, s));
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

extern "C" int cfd_conv3d_backward_data(const cfd_grid *grid, int32_t cin, int32_t cout, const uint16_t *dy,
                                        const uint16_t *w, float *dx, void *stream) {
    Geo g;
    int rc = conv_args(grid, cin, cout, &g);
    if (rc != CFD_OK) return rc;
    if (!dy || !w || !dx) return fail(CFD_EINVAL, "conv3d: null pointer");
    hipStream_t s = (hipStream_t)stream;
    void *mem;
    uint16_t *frag;
    rc = conv_weights(w, cin, cout, 1, s, &mem, &frag);
    if (rc != CFD_OK) return rc;
    const int64_t npad = (int64_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
    float *dxp;
    CFD_HIP(hipMallocAsync((void **)&dxp, sizeof(float) * npad * cin, s));
    // this convolution maps cout channels to cin channels
    if (cout == 1) launch_conv<1, 16, FULL, false>(g, dy, frag, dxp, 0, s);
    else if (cin == 16) launch_conv<16, 16, FULL, false>(g, dy, frag, dxp, 0, s);
    else launch_conv<16, 1, FULL, false>(g, dy, frag, dxp, 0, s);
    const int gb = grid1(g.n * cin);
    if (cin == 16)
        hipLaunchKernelGGL((fold_kernel<16, false, false>), dim3(gb), dim3(kBlock), 0, s, g, (const float *)dxp,
                           (const uint16_t *)nullptr, (void *)dx);
    else
        hipLaunchKernelGGL((fold_kernel<1, false, false>), dim3(gb), dim3(kBlock), 0, s, g, (const float *)dxp,
                           (const uint16_t *)nullptr, (void *)dx);
    CFD_HIP(hipFreeAsync(dxp, s));
    CFD_HIP(hipFreeAsync(mem, s));
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}

extern "C" int cfd_conv3d_backward_weight(const cfd_grid *grid, int32_t cin, int32_t cout, const uint16_t *x,
                                          const uint16_t *dy, float *dw, void *stream) {
    Geo g;
    int rc = conv_args(grid, cin, cout, &g);
    if (rc != CFD_OK) return rc;
    if (!x || !dy || !dw) return fail(CFD_EINVAL, "conv3d: null pointer");
    hipStream_t s = (hipStream_t)stream;
    float *part;
    CFD_HIP(hipMallocAsync((void **)&part, sizeof(float) * wgrad_part_floats(g.n, 27 * cin * cout), s));
    if (cin == 1) launch_wgrad<1, 16>(g, x, dy, part, dw, 0, s);
    else if (cout == 16) launch_wgrad<16, 16>(g, x, dy, part, dw, 0, s);
    else launch_wgrad<16, 1>(g, x, dy, part, dw, 0, s);
    CFD_HIP(hipFreeAsync(part, s));
    CFD_HIP(hipGetLastError());
    return CFD_OK;
}
