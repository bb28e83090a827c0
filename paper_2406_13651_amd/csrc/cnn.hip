// Learned prior agent: a residual 3D CNN denoiser with BF16 MFMA kernels.
//
// Network: 8 convolutions of 3x3x3 taps with biases and zero padding,
// channels 1 -> 32 -> ... -> 32 -> 1, ReLU after the first seven, output
// H(x) = x + N(x).  Applied to a volume w of any scale it runs on w / m with
// m = mean(w) and returns w + m N(w / m).
//
// Storage: activations and gradients are channels-last bfloat16, [voxel][C]
// with C = 8 for one-channel tensors (channel 0 used) and 32 otherwise.
// Every convolution is an implicit GEMM on the 32x32x8 bf16 MFMA with fp32
// accumulation: a wave owns 32 consecutive voxels along x and 32 output
// channels, and walks K = 27 taps x (C / 8) input-channel groups, loading the
// A fragment (4 channels of one shifted voxel per lane) and the B fragment
// (4 input channels of one output channel per lane) as 8-byte loads.  The
// backward data pass is the same kernel with tap-flipped, channel-swapped
// weights; the weight gradient is a per-tap GEMM over voxel chunks with
// per-chunk partial sums reduced in a fixed order.
//
// MFMA 32x32x8 bf16 lane layout (64 lanes, l = lane): A[m][k] in lane
// m + 32 (k / 4), element k % 4; B[k][n] in lane n + 32 (k / 4), element
// k % 4; D[m][n] in lane n + 32 ((m / 4) % 2), register (m / 8) 4 + m % 4.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cnn.h"

namespace clampk {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kCnnBlock = 256;

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two floats as packed bf16 (lo in bits 0..15), round to nearest even: one
// hardware conversion instruction on gfx950.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const v2bf v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// Mask of a dword of two bf16 ReLU outputs: each half is all ones when that
// value is > 0 (sign clear, not zero), else zero.
__device__ __forceinline__ uint32_t relu_keep2(uint32_t k) {
    const uint32_t lo = ((k & 0x8000u) == 0u && (k & 0x7fffu) != 0u) ? 0x0000ffffu : 0u;
    const uint32_t hi = ((k & 0x80000000u) == 0u && (k & 0x7fff0000u) != 0u) ? 0xffff0000u : 0u;
    return lo | hi;
}

__device__ __forceinline__ void tap_offset(int t, int& dz, int& dy, int& dx) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// Row index of the MFMA output register i of lane l (the column is l % 32).
__device__ __forceinline__ int d_row(int l, int i) { return (l / 32) * 4 + (i / 4) * 8 + (i % 4); }

// ---------------------------------------------------------------------------
// Convolution (forward or backward-data), tiled implicit GEMM on the
// 32x32x16 bf16 MFMA.
//
// A block of 4 waves owns an output tile of 16 rows x 32 x-voxels and walks a
// chunk of range slices.  Input slices (tile plus a one-voxel halo: 18 rows x
// 34 voxels, zero outside the volume) live in two LDS slots: output slice z
// takes its dz = -1 and dz = 0 taps from the slots holding input z - 1 and z,
// then input z + 1 (fetched into registers during the previous step) replaces
// input z - 1 and the dz = +1 taps follow, while input z + 2 is fetched.
// Every weight fragment of the layer stays in LDS for the whole block, so the
// MFMA loop reads only LDS.  Wave w computes rows 4w..4w+3; for each (dz, dy)
// tap pair and K fragment q it reads the six input rows its four output rows
// need once and applies each to up to three output rows (the dy taps).  K
// fragments: for 32 input channels q = (dx, channel half), 6 per (dz, dy); for
// 8 input channels q pairs two dx taps (q = 0: dx = -1 in k 0..7 and dx = 0 in
// k 8..15; q = 1: dx = +1 and zeros).
//
// LDS layouts.  Input slot: 16-byte chunks; for 32 channels the chunk j of
// voxel (row ys, column xs) sits at (ys * 34 + xs) * 4 + (j ^ ((xs >> 2) & 3)),
// so that the 16 lanes of one 128-bit LDS access phase (16 consecutive voxels,
// one chunk each) hit 16 distinct 16-byte bank groups of the 256-byte bank
// window.  Weights: wq[g = 3 dz + dy][q][h][n][8] (see k_prep_q), 16 lanes of
// one phase reading 16 consecutive fragments rows.  Output staging: each wave
// writes two output rows (32 voxels x 32 bf16 channels) into a private area,
// voxel v at record v ^ (((v >> 2) & 1) << 1) so that the two voxels of one
// MFMA register (v and v + 4) fall into different bank windows, and reads it
// back in 16-byte chunks for coalesced global stores (and, for the
// backward-data pass, coalesced ReLU-mask loads).
constexpr int kTileRows = 16;
constexpr int kTileCols = 32;
constexpr int kRingRows = kTileRows + 2;
constexpr int kRingCols = kTileCols + 2;

template <int CIN>
struct TileGeo {
    static constexpr int kChunks = CIN / 8;                              // 16-byte chunks per voxel
    static constexpr int kSlice = kRingRows * kRingCols * kChunks;      // chunks per input slot
    static constexpr int kQ = CIN == 32 ? 6 : 2;                         // K fragments per (dz, dy)
    static constexpr int kW = 9 * kQ * 64;                               // weight chunks (16 bytes)
    static constexpr int kFill = (kSlice + kCnnBlock - 1) / kCnnBlock;  // chunks per thread per slice
};

template <int CIN>
__device__ __forceinline__ int ring_pos(int ys, int xs, int j) {
    if constexpr (CIN == 32) return (ys * kRingCols + xs) * 4 + (j ^ ((xs >> 2) & 3));
    else return ys * kRingCols + xs;
}

template <int CIN>
__device__ __forceinline__ void tile_fetch(const ConvArgs& a, const uint16_t* in, int zin, int y0, int x0,
                                           uint4 (&pre)[TileGeo<CIN>::kFill]) {
    using G = TileGeo<CIN>;
#pragma unroll
    for (int i = 0; i < G::kFill; ++i) {
        const int e = threadIdx.x + i * kCnnBlock;
        const int j = e % G::kChunks, vox = e / G::kChunks;
        const int xs = vox % kRingCols, ys = vox / kRingCols;
        const int y = y0 - 1 + ys, x = x0 - 1 + xs;
        const bool ok = e < G::kSlice && zin >= 0 && zin < a.nz && y >= 0 && y < a.ny && x >= 0 && x < a.nx;
        // out-of-volume chunks read voxel 0 and are zeroed (no divergent branch around the load)
        const long off = ok ? (((long)zin * a.ny + y) * a.nx + x) * CIN + j * 8 : 0;
        const uint4 v = *reinterpret_cast<const uint4*>(in + off);
        pre[i] = ok ? v : make_uint4(0u, 0u, 0u, 0u);
    }
}

template <int CIN>
__device__ __forceinline__ void tile_store(uint4* slot, const uint4 (&pre)[TileGeo<CIN>::kFill]) {
    using G = TileGeo<CIN>;
#pragma unroll
    for (int i = 0; i < G::kFill; ++i) {
        const int e = threadIdx.x + i * kCnnBlock;
        if (e < G::kSlice) {
            const int j = e % G::kChunks, vox = e / G::kChunks;
            slot[ring_pos<CIN>(vox / kRingCols, vox % kRingCols, j)] = pre[i];
        }
    }
}

// acc[r] += the taps of range offset dz (index 0..2) from the input slot.
template <int CIN>
__device__ __forceinline__ void conv_dz(const uint4* slot, const uint4* wsh, int dz, int wave, int m, int h,
                                        v16f (&acc)[4]) {
    using G = TileGeo<CIN>;
#pragma unroll
    for (int q = 0; q < G::kQ; ++q) {
        int xs, j;
        if constexpr (CIN == 32) {
            xs = m + (q >> 1);
            j = 2 * (q & 1) + h;
        } else {
            xs = m + (q == 0 ? h : 2);
            j = 0;
        }
        v8bf A[6];
#pragma unroll
        for (int rr = 0; rr < 6; ++rr) A[rr] = __builtin_bit_cast(v8bf, slot[ring_pos<CIN>(4 * wave + rr, xs, j)]);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const v8bf B = __builtin_bit_cast(v8bf, wsh[(((dz * 3 + dy) * G::kQ + q) * 2 + h) * 32 + m]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[r + dy], B, acc[r], 0, 0, 0);
        }
    }
}

template <int CIN, int EPI>
__global__ __launch_bounds__(kCnnBlock, 1) void k_conv(ConvArgs a) {
    using G = TileGeo<CIN>;
    __shared__ uint4 ring[2][G::kSlice];
    __shared__ uint4 wsh[G::kW];
    __shared__ uint32_t stage[4 * 2 * 32 * 16];  // per wave: 2 rows x 32 voxels x 16 dwords
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    int b = blockIdx.x;
    const int xt = b % a.tiles_x;
    b /= a.tiles_x;
    const int yt = b % a.tiles_y;
    b /= a.tiles_y;
    const int zc = b % a.zchunks;
    const int vol = b / a.zchunks;
    const int x0 = xt * kTileCols, y0 = yt * kTileRows;
    const int z0 = zc * a.zc;
    const int z1 = z0 + a.zc < a.nz ? z0 + a.zc : a.nz;
    const long vol_off = (long)vol * a.nz * a.ny * a.nx;
    const uint16_t* in = a.in + vol_off * CIN;

    for (int i = threadIdx.x; i < G::kW; i += kCnnBlock) wsh[i] = reinterpret_cast<const uint4*>(a.wq)[i];
    uint4 pre[G::kFill];
    tile_fetch<CIN>(a, in, z0 - 1, y0, x0, pre);
    tile_store<CIN>(ring[0], pre);
    tile_fetch<CIN>(a, in, z0, y0, x0, pre);
    tile_store<CIN>(ring[1], pre);
    tile_fetch<CIN>(a, in, z0 + 1, y0, x0, pre);
    __syncthreads();

    float bias_n = 0.f, scale = 1.f;
    if constexpr (EPI == EPI_RELU) bias_n = a.bias[m];
    if constexpr (EPI == EPI_FINAL) {
        bias_n = a.bias[0];
        if (a.scale != nullptr) scale = *a.scale;
    }

    int old = 0;  // slot of input z - 1; the other slot holds input z
    for (int z = z0; z < z1; ++z) {
        v16f acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = v16f{};
        conv_dz<CIN>(ring[old], wsh, 0, wave, m, h, acc);
        conv_dz<CIN>(ring[old ^ 1], wsh, 1, wave, m, h, acc);
        __syncthreads();  // every wave is done with input z - 1
        tile_store<CIN>(ring[old], pre);
        __syncthreads();
        if (z + 1 < z1) tile_fetch<CIN>(a, in, z + 2, y0, x0, pre);
        conv_dz<CIN>(ring[old], wsh, 2, wave, m, h, acc);
        old ^= 1;

        // epilogue: lane holds output channel m for 16 voxels of each of its 4 rows
        if constexpr (EPI == EPI_FINAL) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = y0 + 4 * wave + r;
                if (y >= a.ny || m != 0) continue;
                const long row0 = vol_off + ((long)z * a.ny + y) * a.nx + x0;
                float xv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) xv[i] = a.xin[row0 + d_row(lane, i)];
#pragma unroll
                for (int i = 0; i < 16; ++i) a.out_f32[row0 + d_row(lane, i)] = xv[i] + scale * (acc[r][i] + bias_n);
            }
        } else {
            uint32_t* st = stage + wave * (2 * 32 * 16);
            const uint4* st4 = reinterpret_cast<const uint4*>(st);
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
                for (int rp = 0; rp < 2; ++rp)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        float val = acc[2 * pass + rp][i];
                        if constexpr (EPI == EPI_RELU) val = fmaxf(val + bias_n, 0.f);
                        // channel m + 1 from the neighbouring lane (quad permutation 1, 0, 3, 2)
                        const float other = __builtin_bit_cast(
                            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, val), 0xB1, 0xF, 0xF, false));
                        const int vox = d_row(lane, i);
                        if ((m & 1) == 0)
                            st[(rp * 32 + (vox ^ (((vox >> 2) & 1) << 1))) * 16 + (m >> 1)] = pack_bf16x2(val, other);
                    }
                __syncthreads();
#pragma unroll
                for (int it = 0; it < 4; ++it) {
                    const int e = it * 64 + lane;
                    const int rp = e >> 7, vox = (e >> 2) & 31, c = e & 3;
                    const int y = y0 + 4 * wave + 2 * pass + rp;
                    if (y < a.ny) {
                        uint4 q = st4[(rp * 32 + (vox ^ (((vox >> 2) & 1) << 1))) * 4 + c];
                        const long v = vol_off + ((long)z * a.ny + y) * a.nx + x0 + vox;
                        if constexpr (EPI == EPI_DGRAD) {  // multiply by the ReLU mask of the layer input
                            const uint4 k = *reinterpret_cast<const uint4*>(a.relu_src + v * 32 + c * 8);
                            q.x &= relu_keep2(k.x);
                            q.y &= relu_keep2(k.y);
                            q.z &= relu_keep2(k.z);
                            q.w &= relu_keep2(k.w);
                        }
                        *reinterpret_cast<uint4*>(a.out + v * 32 + c * 8) = q;
                    }
                }
                __syncthreads();
            }
        }
    }
}

// x8[v] = (bf16(x[v] / m), 0, ..., 0) with m = *scale (1 when scale is NULL).
__global__ __launch_bounds__(kCnnBlock) void k_pack(const float* x, const float* scale, long nvox, uint16_t* x8) {
    const float inv = scale != nullptr ? 1.f / *scale : 1.f;
    for (long v = (long)blockIdx.x * kCnnBlock + threadIdx.x; v < nvox; v += (long)gridDim.x * kCnnBlock) {
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        q.x = f2bf(x[v] * inv);
        reinterpret_cast<uint4*>(x8)[v] = q;
    }
}

// Block sums of K doubles into part[block * K + k].
template <int K>
__device__ __forceinline__ void cnn_block_sum(double (&v)[K], double* out) {
    __shared__ double red[K][kCnnBlock / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < kCnnBlock / 64; ++w) s += red[k][w];
            out[k] = s;
        }
}

// Mean of x over nvox voxels into *mean (two passes: block partials, then sum).
__global__ __launch_bounds__(kCnnBlock) void k_sum_partial(const float* x, long nvox, double* part) {
    double s = 0.0;
    for (long v = (long)blockIdx.x * kCnnBlock + threadIdx.x; v < nvox; v += (long)gridDim.x * kCnnBlock) s += x[v];
    double a[1] = {s};
    cnn_block_sum<1>(a, part + blockIdx.x);
}
__global__ __launch_bounds__(kCnnBlock) void k_mean_final(const double* part, int nblocks, long nvox, float* mean) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kCnnBlock) s += part[i];
    double a[1] = {s};
    __shared__ double tot[1];
    cnn_block_sum<1>(a, tot);
    if (threadIdx.x == 0) *mean = (float)(tot[0] / (double)nvox);
}

// Squared error partials and the output gradient 2 (out - t) / nvox.
__global__ __launch_bounds__(kCnnBlock) void k_loss(const float* out, const float* target, long nvox, uint16_t* g8,
                                                    double* part) {
    const float c = (float)(2.0 / (double)nvox);
    double s = 0.0;
    for (long v = (long)blockIdx.x * kCnnBlock + threadIdx.x; v < nvox; v += (long)gridDim.x * kCnnBlock) {
        const float r = out[v] - target[v];
        s += (double)r * r;
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        q.x = f2bf(c * r);
        reinterpret_cast<uint4*>(g8)[v] = q;
    }
    double a[1] = {s};
    cnn_block_sum<1>(a, part + blockIdx.x);
}
__global__ __launch_bounds__(kCnnBlock) void k_loss_final(const double* part, int nblocks, long nvox, double* loss) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kCnnBlock) s += part[i];
    double a[1] = {s};
    __shared__ double tot[1];
    cnn_block_sum<1>(a, tot);
    if (threadIdx.x == 0) *loss = tot[0] / (double)nvox;
}

// Weight gradient of one layer: D[co][ci] = sum_v g[v][co] act[v + off(t)][ci]
// for the tap t of each wave, over chunk `blockIdx.x / 7` of the voxels
// (K-steps of 8 consecutive voxels along x); partials to part[chunk][t][co][ci].
template <int CA, int CG>
__global__ __launch_bounds__(kCnnBlock) void k_wgrad(WgradArgs a) {
    const int lane = threadIdx.x & 63;
    const int chunk = blockIdx.x / 7;
    const int t = (blockIdx.x % 7) * 4 + (threadIdx.x >> 6);
    if (t >= 27) return;  // no barriers in this kernel
    int dz, dy, dx;
    tap_offset(t, dz, dy, dx);
    const long steps = a.nvox / 8;
    const long s0 = (long)chunk * a.chunk_steps;
    const long s1 = s0 + a.chunk_steps < steps ? s0 + a.chunk_steps : steps;
    const int ch = lane & 31;
    const int kh = (lane >> 5) * 4;
    v16f acc = {};
    for (long s = s0; s < s1; ++s) {
        const long v0 = s * 8 + kh;  // this lane half's 4 voxels: v0 .. v0 + 3 (same x run)
        const int x0 = (int)(v0 % a.nx);
        long r = v0 / a.nx;
        const int y = (int)(r % a.ny);
        r /= a.ny;
        const int z = (int)(r % a.nz);
        const long n = r / a.nz;
        const int zz = z + dz, yy = y + dy;
        const bool row_ok = zz >= 0 && zz < a.nz && yy >= 0 && yy < a.ny;
        const long arow = ((n * a.nz + (row_ok ? zz : 0)) * a.ny + (row_ok ? yy : 0)) * a.nx;
        v4s av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            av[j] = ch < CG ? (short)a.g[(v0 + j) * CG + ch] : (short)0;
            const int xx = x0 + j + dx;
            const bool ok = row_ok && xx >= 0 && xx < a.nx && ch < CA;
            bv[j] = ok ? (short)a.act[(arow + xx) * CA + ch] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    float* dst = a.part + ((long)chunk * 27 + t) * 1024;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[d_row(lane, i) * 32 + ch] = acc[i];
}

// grad[W + (t * cin + ci) * cout + co] = sum over chunks of part[c][t][co][ci]:
// a block covers 16 consecutive positions p = t * 1024 + co * 32 + ci; thread
// (p, l) sums chunks l, l + 16, ... in order, then the 16 partial sums are
// added in order (a fixed summation order, so runs are bitwise repeatable).
__global__ __launch_bounds__(kCnnBlock) void k_wgrad_reduce(const float* part, int chunks, int cin, int cout,
                                                            float* gw) {
    __shared__ double red[16][16];
    const int pl = threadIdx.x & 15, l = threadIdx.x >> 4;
    const int p = blockIdx.x * 16 + pl;
    double s = 0.0;
    if (p < 27 * 1024)
        for (int c = l; c < chunks; c += 16) s += part[(long)c * 27 * 1024 + p];
    red[l][pl] = s;
    __syncthreads();
    if (l == 0 && p < 27 * 1024) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k][pl];
        const int ci = p & 31, co = (p >> 5) & 31, tap = p >> 10;
        if (ci < cin && co < cout) gw[(tap * cin + ci) * cout + co] = (float)t;
    }
}

// Bias gradient partials: part[block][co] = sum over the block's voxels of g[v][co].
template <int CG>
__global__ __launch_bounds__(kCnnBlock) void k_bias_partial(const uint16_t* g, long nvox, float* part) {
    __shared__ float red[kCnnBlock];
    const int co = threadIdx.x % 32, lane_v = threadIdx.x / 32;
    float s = 0.f;
    if (co < CG)
        for (long v = (long)blockIdx.x * 8 + lane_v; v < nvox; v += (long)gridDim.x * 8) s += bf2f(g[v * CG + co]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
        for (int k = 0; k < 8; ++k) t += red[k * 32 + threadIdx.x];
        part[(long)blockIdx.x * 32 + threadIdx.x] = t;
    }
}
// Block co: thread l sums partials l, l + 256, ... in order; thread 0 adds
// the 256 sums in order.
__global__ __launch_bounds__(kCnnBlock) void k_bias_reduce(const float* part, int nblocks, int cout, float* gb) {
    __shared__ double red[kCnnBlock];
    const int co = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kCnnBlock) s += part[(long)b * 32 + co];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kCnnBlock; ++k) t += red[k];
        if (co < cout) gb[co] = (float)t;
    }
}

// Adam with bias correction on the flat parameter vector.
__global__ __launch_bounds__(kCnnBlock) void k_adam(float* p, float* m, float* v, const float* g, int n, float lr,
                                                    float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * kCnnBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Zero-padded fp32 copy of a layer's bias.
__global__ void k_prep_bias(const float* b, int cout, float* bias32) {
    const int e = threadIdx.x;
    if (e < 32) bias32[e] = e < cout ? b[e] : 0.f;
}

// Weight fragments of the tiled convolution: wq[g = 3 dz + dy][q][h][n][8]
// (bf16) holds k = 8 h .. 8 h + 7 of K fragment q for output channel n, for
// the input-channel count CINP (8 or 32), from the fp32 W[t][cin][cout].
// Forward: the effective weight is W[t][ci][co]; backward data (flip):
// W[26 - t][co][ci] with the channel roles swapped.  Entries beyond the real
// channel counts and the zero half of the last 8-channel fragment are zero.
__global__ __launch_bounds__(kCnnBlock) void k_prep_q(const float* W, int cin, int cout, int flip, int cinp,
                                                     uint16_t* wq) {
    const int nq = cinp == 32 ? 6 : 2;
    const int e = blockIdx.x * kCnnBlock + threadIdx.x;
    if (e >= 9 * nq * 32 * 16) return;
    const int k8 = e % 8, n = (e / 8) % 32, hh = (e / 256) % 2, q = (e / 512) % nq, g = e / (512 * nq);
    const int kk = 8 * hh + k8;
    const int dz = g / 3, dy = g % 3;
    int dxi, ci;
    bool zero = false;
    if (cinp == 32) {
        dxi = q >> 1;
        ci = 16 * (q & 1) + kk;
    } else {
        ci = k8;
        dxi = q == 0 ? hh : 2;
        zero = q == 1 && hh == 1;
    }
    const int t = 9 * dz + 3 * dy + dxi;
    const int ein = flip ? cout : cin, eout = flip ? cin : cout;
    float w = 0.f;
    if (!zero && ci < ein && n < eout)
        w = flip ? W[((26 - t) * cin + n) * cout + ci] : W[(t * cin + ci) * cout + n];
    wq[e] = f2bf(w);
}

// ---------------------------------------------------------------------------
// Launchers
static int grid_for(long work, int per_block, int cap) {
    long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

hipError_t cnn_conv(int cin, int epi, ConvArgs a, hipStream_t st) {
    a.tiles_x = a.nx / kTileCols;
    a.tiles_y = (a.ny + kTileRows - 1) / kTileRows;
    // range slices per block: fewer when the volume gives too few tiles to fill the chip
    const long tiles = (long)a.nvol * a.tiles_x * a.tiles_y;
    a.zc = 8;
    while (a.zc > 2 && tiles * ((a.nz + a.zc - 1) / a.zc) < 1024) a.zc /= 2;
    a.zchunks = (a.nz + a.zc - 1) / a.zc;
    const dim3 grid((unsigned)(tiles * a.zchunks));
#define LAUNCH(CI, EP) hipLaunchKernelGGL((k_conv<CI, EP>), grid, dim3(kCnnBlock), 0, st, a)
    if (cin == 8 && epi == EPI_RELU) LAUNCH(8, EPI_RELU);
    else if (cin == 32 && epi == EPI_RELU) LAUNCH(32, EPI_RELU);
    else if (cin == 32 && epi == EPI_FINAL) LAUNCH(32, EPI_FINAL);
    else if (cin == 8 && epi == EPI_DGRAD) LAUNCH(8, EPI_DGRAD);
    else if (cin == 32 && epi == EPI_DGRAD) LAUNCH(32, EPI_DGRAD);
    else return hipErrorInvalidValue;
#undef LAUNCH
    return hipGetLastError();
}

size_t cnn_wq_elems(int cinp) { return (size_t)9 * (cinp == 32 ? 6 : 2) * 32 * 16; }

hipError_t cnn_prep_q(const float* W, int cin, int cout, int flip, int cinp, uint16_t* wq, hipStream_t st) {
    const int n = (int)cnn_wq_elems(cinp);
    hipLaunchKernelGGL(k_prep_q, dim3((n + kCnnBlock - 1) / kCnnBlock), dim3(kCnnBlock), 0, st, W, cin, cout, flip,
                       cinp, wq);
    return hipGetLastError();
}

hipError_t cnn_pack(const float* x, const float* scale, long nvox, uint16_t* x8, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nvox, kCnnBlock, 8192)), dim3(kCnnBlock), 0, st, x, scale, nvox, x8);
    return hipGetLastError();
}

int cnn_reduce_blocks(long nvox) { return grid_for(nvox, kCnnBlock, 1024); }

hipError_t cnn_mean(const float* x, long nvox, double* part, float* mean, hipStream_t st) {
    const int nb = cnn_reduce_blocks(nvox);
    hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(kCnnBlock), 0, st, x, nvox, part);
    hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(kCnnBlock), 0, st, part, nb, nvox, mean);
    return hipGetLastError();
}

hipError_t cnn_loss(const float* out, const float* target, long nvox, uint16_t* g8, double* part, double* loss,
                    hipStream_t st) {
    const int nb = cnn_reduce_blocks(nvox);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(kCnnBlock), 0, st, out, target, nvox, g8, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kCnnBlock), 0, st, part, nb, nvox, loss);
    return hipGetLastError();
}

int cnn_wgrad_chunks(long nvox, long chunk_steps) { return (int)((nvox / 8 + chunk_steps - 1) / chunk_steps); }

hipError_t cnn_wgrad(int ca, int cg, const WgradArgs& a, int cin, int cout, float* gw, float* gb, float* bias_part,
                     hipStream_t st) {
    const int chunks = cnn_wgrad_chunks(a.nvox, a.chunk_steps);
    const dim3 grid((unsigned)chunks * 7);
#define LAUNCH(A, G) hipLaunchKernelGGL((k_wgrad<A, G>), grid, dim3(kCnnBlock), 0, st, a)
    if (ca == 8 && cg == 32) LAUNCH(8, 32);
    else if (ca == 32 && cg == 32) LAUNCH(32, 32);
    else if (ca == 32 && cg == 8) LAUNCH(32, 8);
    else return hipErrorInvalidValue;
#undef LAUNCH
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(27 * 1024 / 16), dim3(kCnnBlock), 0, st,
                       a.part, chunks, cin, cout, gw);
    const int nb = grid_for(a.nvox, 8, 2048);
    if (cg == 8)
        hipLaunchKernelGGL(k_bias_partial<8>, dim3(nb), dim3(kCnnBlock), 0, st, a.g, a.nvox, bias_part);
    else
        hipLaunchKernelGGL(k_bias_partial<32>, dim3(nb), dim3(kCnnBlock), 0, st, a.g, a.nvox, bias_part);
    hipLaunchKernelGGL(k_bias_reduce, dim3(cout), dim3(kCnnBlock), 0, st, bias_part, nb, cout, gb);
    return hipGetLastError();
}

int cnn_bias_blocks(long nvox) { return grid_for(nvox, 8, 2048); }

hipError_t cnn_adam(float* p, float* m, float* v, const float* g, int n, float lr, int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
    hipLaunchKernelGGL(k_adam, dim3((n + kCnnBlock - 1) / kCnnBlock), dim3(kCnnBlock), 0, st, p, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t cnn_prep(const float* W, const float* b, int cin, int cout, int cinp, int coutp, uint16_t* wq,
                    uint16_t* wqd, float* bias32, hipStream_t st) {
    hipError_t e = cnn_prep_q(W, cin, cout, 0, cinp, wq, st);
    if (e == hipSuccess && wqd != nullptr) e = cnn_prep_q(W, cin, cout, 1, coutp, wqd, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prep_bias, dim3(1), dim3(32), 0, st, b, cout, bias32);
    return hipGetLastError();
}

}  // namespace clampk
