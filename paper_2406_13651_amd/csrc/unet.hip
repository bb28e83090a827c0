// U-Net prior kernels: 2x2x2 max pooling, the 2x2x2 stride-2 transposed
// convolution (on gfx950's 32x32x16 bf16 MFMA) with bias and skip addition,
// and the evaluation-mode batch normalisation fold.
//
// Tensors are channels-last bf16 [voxel][32] as for the CNN kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "unet.h"

namespace clampk {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
// raw buffer resource word 3 and an offset outside every buffer addressed
// here (one row of at most 2^31 bytes): stores there are dropped, loads read 0
constexpr int kWord3 = 0x00020000;
constexpr uint32_t kOutside = 0x80000000u;

__device__ __forceinline__ float bf_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const v2bf v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// elementwise max of 8 bf16 values (the inputs are exact bf16, so is the max)
__device__ __forceinline__ uint32_t max2(uint32_t a, uint32_t b) {
    const uint32_t lo = bf_lo(a) >= bf_lo(b) ? (a & 0xffffu) : (b & 0xffffu);
    const uint32_t hi = bf_hi(a) >= bf_hi(b) ? (a & 0xffff0000u) : (b & 0xffff0000u);
    return lo | hi;
}

__global__ __launch_bounds__(kBlock) void k_pool2(const uint16_t* in, uint16_t* out, int nvol, int nz, int ny,
                                                  int nx) {
    // a volume holds fewer than 2^31 voxels (checked by the caller): 32-bit
    // index arithmetic
    const unsigned cz = nz / 2, cy = ny / 2, cx = nx / 2;
    const unsigned total = (unsigned)nvol * cz * cy * cx * 4u;
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const unsigned j = i & 3u;
        unsigned v = i >> 2;
        const unsigned x = v % cx;
        v /= cx;
        const unsigned y = v % cy;
        v /= cy;
        const unsigned z = v % cz;
        const unsigned vol = v / cz;
        uint4 m;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const long f = (((long)vol * nz + 2 * z + (s >> 2)) * ny + 2 * y + ((s >> 1) & 1)) * nx + 2 * x + (s & 1);
            const uint4 q = *reinterpret_cast<const uint4*>(in + f * 32 + j * 8);
            if (s == 0) {
                m = q;
            } else {
                m.x = max2(m.x, q.x);
                m.y = max2(m.y, q.y);
                m.z = max2(m.z, q.z);
                m.w = max2(m.w, q.w);
            }
        }
        *reinterpret_cast<uint4*>(out + (long)(i >> 2) * 32 + j * 8) = m;
    }
}

// One wave per run of 32 coarse voxels along x (lane m = voxel x0 + m, half
// h).  D[co][voxel] = W_s^T X^T for each sub-position s on the MFMA (K = 32
// input channels as two halves): lane (m, h) gets channels 8 g + 4 h + 0..3
// (g = 0..3) of output voxel (2z + a, 2y + b, 2(x0 + m) + c); with the bias
// added, a swap between the lane halves gives it 8 consecutive channels 16 p +
// 8 h + 0..7 (p = 0, 1) in fp32, to which the skip is added before rounding.
__global__ __launch_bounds__(kBlock) void k_upconv(UpArgs a) {
    // the wave index read from the first lane: the run, the row bases and the
    // buffer descriptors derived from it are then scalar (no per-lane loop
    // around each buffer access)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int m = lane & 31, h = lane >> 5;
    const int runs = (a.nx + 31) / 32;
    const long total = (long)a.nvol * a.nz * a.ny * runs;
    const long run = (long)blockIdx.x * 4 + wave;
    if (run >= total) return;  // whole waves only; no block barrier below
    const int xr = (int)(run % runs);
    long r = run / runs;
    const int y = (int)(r % a.ny);
    r /= a.ny;
    const int z = (int)(r % a.nz);
    const long vol = r / a.nz;
    const int x = xr * 32 + m;
    const bool xok = x < a.nx;

    const __amdgpu_buffer_rsrc_t in_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(a.in) + ((vol * a.nz + z) * a.ny + y) * (long)a.nx * 32, 0, (uint32_t)a.nx * 64u, kWord3);
    const int NZ = 2 * a.nz, NY = 2 * a.ny, NX = 2 * a.nx;
    // every load of the run first (input, the 16 weight fragments, the 16
    // skip runs), so that their latencies overlap; then products and stores
    v8bf xb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
        xb[e] = __builtin_bit_cast(
            v8bf, __builtin_amdgcn_raw_buffer_load_b128(in_rs, xok ? (uint32_t)(x * 64 + 32 * e + 16 * h) : kOutside, 0, 0));
    v8bf w[8][2];
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int e = 0; e < 2; ++e)
            w[s][e] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.wf + ((s * 2 + e) * 64 + lane) * 8));
    auto row_of = [&](int s) { return ((vol * NZ + 2 * z + (s >> 2)) * NY + 2 * y + ((s >> 1) & 1)) * (long)NX; };
    auto off_of = [&](int s, int p) {
        return xok ? (uint32_t)((2 * x + (s & 1)) * 64 + 32 * p + 16 * h) : kOutside;
    };
    v4u sk[8][2];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const __amdgpu_buffer_rsrc_t skip_rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(a.skip) + row_of(s) * 32, 0, (uint32_t)NX * 64u, kWord3);
#pragma unroll
        for (int p = 0; p < 2; ++p) sk[s][p] = __builtin_amdgcn_raw_buffer_load_b128(skip_rs, off_of(s, p), 0, 0);
    }
    float bias_r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) bias_r[i] = a.bias[(i >> 2) * 8 + 4 * h + (i & 3)];

#pragma unroll
    for (int s = 0; s < 8; ++s) {
        v16f d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[s][0], xb[0], v16f{}, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[s][1], xb[1], d, 0, 0, 0);
        const __amdgpu_buffer_rsrc_t out_rs =
            __builtin_amdgcn_make_buffer_rsrc(a.out + row_of(s) * 32, 0, (uint32_t)NX * 64u, kWord3);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float lo[4], hi[4];  // channels 16 p + 8 h + (0..3, 4..7) after the swap
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i0 = 4 * (2 * p) + c, i1 = 4 * (2 * p + 1) + c;
                const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[i0] + bias_r[i0]),
                                                                 __float_as_uint(d[i1] + bias_r[i1]), false, false);
                lo[c] = __uint_as_float(sw[0]);
                hi[c] = __uint_as_float(sw[1]);
            }
            const v4u k = sk[s][p];
            v4u q;
            q[0] = pack2(lo[0] + bf_lo(k[0]), lo[1] + bf_hi(k[0]));
            q[1] = pack2(lo[2] + bf_lo(k[1]), lo[3] + bf_hi(k[1]));
            q[2] = pack2(hi[0] + bf_lo(k[2]), hi[1] + bf_hi(k[2]));
            q[3] = pack2(hi[2] + bf_lo(k[3]), hi[3] + bf_hi(k[3]));
            __builtin_amdgcn_raw_buffer_store_b128(q, out_rs, off_of(s, p), 0, 0);
        }
    }
}

// Fragment e = ((s 2 + kh) 64 + l) 8 + k8 holds, for the forward product, the
// A operand W^T of sub-position s: W[s][ci = 16 kh + 8 (l / 32) + k8][co = l % 32];
// for the backward-data product (transposed), the A operand W:
// W[s][ci = l % 32][co = 16 kh + 8 (l / 32) + k8].
__global__ __launch_bounds__(kBlock) void k_prep_up(const float* W, int transposed, uint16_t* wf) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= 8 * 2 * 64 * 8) return;
    const int k8 = e % 8, l = (e / 8) % 64, kh = (e / 512) % 2, s = e / 1024;
    const int k = 16 * kh + 8 * (l / 32) + k8, n = l % 32;
    const int ci = transposed ? n : k, co = transposed ? k : n;
    const __bf16 b = (__bf16)W[(s * 32 + ci) * 32 + co];
    wf[e] = __builtin_bit_cast(uint16_t, b);
}

__global__ __launch_bounds__(kBlock) void k_fold_bn(const float* W, const float* gamma, const float* beta,
                                                    const float* mean, const float* var, int cin, float* wout,
                                                    float* bout) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    const int nw = 27 * cin * 32;
    if (e < nw) {
        const int co = e % 32;
        wout[e] = W[e] * (gamma[co] / sqrtf(var[co] + kBnEps));
    } else if (e < nw + 32) {
        const int co = e - nw;
        const float s = gamma[co] / sqrtf(var[co] + kBnEps);
        bout[co] = beta[co] - mean[co] * s;
    }
}

// ---------------------------------------------------------------------------
// Training kernels

__device__ __forceinline__ void unpack8(uint4 q, float (&f)[8]) {
    f[0] = bf_lo(q.x); f[1] = bf_hi(q.x); f[2] = bf_lo(q.y); f[3] = bf_hi(q.y);
    f[4] = bf_lo(q.z); f[5] = bf_hi(q.z); f[6] = bf_lo(q.w); f[7] = bf_hi(q.w);
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
    return make_uint4(pack2(f[0], f[1]), pack2(f[2], f[3]), pack2(f[4], f[5]), pack2(f[6], f[7]));
}

// Per-channel sums over a bf16 [nvox][32] tensor, in float64, one partial per
// block in part[block][32][2] (fixed order: each thread walks its voxels in
// order, then a tree over the block's 64 voxel lanes).  MODE 0: (sum x, sum
// x^2) of X; MODE 1: (sum dy, sum dy xhat) with dy = X and xhat = (Y - mean)
// rstd per channel.  At most 256 blocks: k_chan_finalize reads every partial
// from one block, and 256 x 512 bytes keep that read short (with 2048 blocks
// a U-Net training step took 5.00 ms, with 256 blocks 4.73 ms).
constexpr int kChanBlocks = 256;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_chan_sums(const uint16_t* X, const uint16_t* Y, const float* mean,
                                                      const float* rstd, long nvox, double* part) {
    __shared__ double red[kBlock][17];
    const int t = threadIdx.x, j = t & 3, vl = t >> 2;
    double s1[8], s2[8];
    float mu[8], rs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        s1[c] = 0.0;
        s2[c] = 0.0;
        mu[c] = MODE == 1 ? mean[8 * j + c] : 0.f;
        rs[c] = MODE == 1 ? rstd[8 * j + c] : 0.f;
    }
    auto add = [&](uint4 xq, uint4 yq) {
        float x[8];
        unpack8(xq, x);
        if constexpr (MODE == 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                s1[c] += x[c];
                s2[c] += (double)x[c] * x[c];
            }
        } else {
            float z[8];
            unpack8(yq, z);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                s1[c] += x[c];
                s2[c] += (double)x[c] * ((z[c] - mu[c]) * rs[c]);
            }
        }
    };
    // voxels v, v + stride, ... in order; four loads in flight per step
    const long stride = (long)gridDim.x * 64;
    long v = (long)blockIdx.x * 64 + vl;
    for (; v + 3 * stride < nvox; v += 4 * stride) {
        uint4 xq[4], yq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xq[u] = *reinterpret_cast<const uint4*>(X + (v + u * stride) * 32 + 8 * j);
            yq[u] = MODE == 1 ? *reinterpret_cast<const uint4*>(Y + (v + u * stride) * 32 + 8 * j) : xq[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) add(xq[u], yq[u]);
    }
    for (; v < nvox; v += stride) {
        const uint4 xq = *reinterpret_cast<const uint4*>(X + v * 32 + 8 * j);
        add(xq, MODE == 1 ? *reinterpret_cast<const uint4*>(Y + v * 32 + 8 * j) : xq);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        red[t][c] = s1[c];
        red[t][8 + c] = s2[c];
    }
    __syncthreads();
    for (int w = 32; w >= 1; w /= 2) {
        if (vl < w)
#pragma unroll
            for (int k = 0; k < 16; ++k) red[t][k] += red[t + 4 * w][k];
        __syncthreads();
    }
    if (vl == 0)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            part[((long)blockIdx.x * 32 + 8 * j + c) * 2 + 0] = red[t][c];
            part[((long)blockIdx.x * 32 + 8 * j + c) * 2 + 1] = red[t][8 + c];
        }
}

// One thread per channel: the block partials in order, then
// FIN_STATS: batch statistics of a pre-activation over m voxels -> mean,
//   rstd (kept for the backward pass), the affine form A = gamma rstd, B =
//   beta - mean A of the normalisation, and the running statistics
//   (momentum, unbiased variance);
// FIN_BWD: the backward sums -> dgamma = sum dy xhat, dbeta = sum dy into the
//   gradient, and dz = C1 dy + C2 z + C3 with C1 = gamma rstd, C2 = -gamma
//   rstd^2 sum(dy xhat) / m, C3 = -gamma rstd sum(dy) / m - C2 mean;
// FIN_SUM: sum x into out (a bias gradient).
enum FinMode { FIN_STATS = 0, FIN_BWD = 1, FIN_SUM = 2 };

// 1024 threads: lane k of channel c (thread 32 k + c) sums the partials of
// blocks k, k + 32, ... in order, then thread c adds the 32 lane sums in order.
__global__ __launch_bounds__(1024) void k_chan_finalize(int mode, const double* part, int blocks, long m,
                                                        const float* gamma, const float* beta, float* mean,
                                                        float* rstd, float* A, float* B, float* Cc, float* run_mean,
                                                        float* run_var, float* out0, float* out1) {
    __shared__ double lanes[32][32][2];
    const int c = threadIdx.x & 31, k = threadIdx.x >> 5;
    double a1 = 0.0, a2 = 0.0;
    int b = k;
    for (; b + 96 < blocks; b += 128) {  // four independent loads in flight
        double2 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = *reinterpret_cast<const double2*>(part + ((long)(b + 32 * u) * 32 + c) * 2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a1 += q[u].x;
            a2 += q[u].y;
        }
    }
    for (; b < blocks; b += 32) {
        a1 += part[((long)b * 32 + c) * 2 + 0];
        a2 += part[((long)b * 32 + c) * 2 + 1];
    }
    lanes[k][c][0] = a1;
    lanes[k][c][1] = a2;
    __syncthreads();
    if (k != 0) return;
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < 32; ++j) {
        s1 += lanes[j][c][0];
        s2 += lanes[j][c][1];
    }
    if (mode == FIN_STATS) {
        const double mu = s1 / (double)m;
        double var = s2 / (double)m - mu * mu;
        if (var < 0.0) var = 0.0;
        const double r = 1.0 / sqrt(var + (double)kBnEps);
        mean[c] = (float)mu;
        rstd[c] = (float)r;
        const double a = (double)gamma[c] * r;
        A[c] = (float)a;
        B[c] = (float)((double)beta[c] - mu * a);
        run_mean[c] = (float)((1.0 - kBnMomentum) * run_mean[c] + kBnMomentum * mu);
        run_var[c] = (float)((1.0 - kBnMomentum) * run_var[c] + kBnMomentum * var * (double)m / (double)(m - 1));
    } else if (mode == FIN_BWD) {
        out0[c] = (float)s2;  // dgamma
        out1[c] = (float)s1;  // dbeta
        const double gr = (double)gamma[c] * rstd[c];
        const double c2 = -gr * rstd[c] * s2 / (double)m;
        A[c] = (float)gr;
        B[c] = (float)c2;
        Cc[c] = (float)(-gr * s1 / (double)m - c2 * mean[c]);
    } else {
        out0[c] = (float)s1;
    }
}

// out = bf16([ReLU](A x + B y + C)) per channel over a bf16 [nvox][32] tensor
// (y only when HAS_Y).
template <bool HAS_Y, bool RELU>
__global__ __launch_bounds__(kBlock) void k_affine(const uint16_t* X, const uint16_t* Y, const float* A,
                                                   const float* B, const float* Cc, long nvox, uint16_t* out) {
    const long n = nvox * 4;
    // the grid stride is a multiple of 4, so each thread keeps one channel group
    const int j = (int)(threadIdx.x & 3);
    float a8[8], b8[8], c8[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        a8[c] = A[8 * j + c];
        b8[c] = HAS_Y ? B[8 * j + c] : 0.f;
        c8[c] = Cc[8 * j + c];
    }
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        float x[8], y[8], o[8];
        unpack8(*reinterpret_cast<const uint4*>(X + i * 8), x);
        if constexpr (HAS_Y) unpack8(*reinterpret_cast<const uint4*>(Y + i * 8), y);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float v = a8[c] * x[c] + c8[c];
            if constexpr (HAS_Y) v += b8[c] * y[c];
            o[c] = RELU ? fmaxf(v, 0.f) : v;
        }
        *reinterpret_cast<uint4*>(out + i * 8) = pack8(o);
    }
}

// Backward of the pooling at a level: de = [ReLU mask of e] (dp routed to the
// first maximum of each window + dskip), per fine voxel (fine sizes given).
__global__ __launch_bounds__(kBlock) void k_pool2_bwd(const uint16_t* e, const uint16_t* dp, const uint16_t* dskip,
                                                      uint16_t* de, int nvol, int nz, int ny, int nx) {
    // a volume holds fewer than 2^31 voxels (checked by the caller): 32-bit
    // index arithmetic
    const unsigned cz = nz / 2, cy = ny / 2, cx = nx / 2;
    const unsigned total = (unsigned)nvol * cz * cy * cx * 4u;
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        const unsigned j = i & 3u;
        unsigned v = i >> 2;
        const unsigned x = v % cx;
        v /= cx;
        const unsigned y = v % cy;
        v /= cy;
        const unsigned z = v % cz;
        const unsigned vol = v / cz;
        long f[8];
        float ev[8][8];
        uint4 kq[8];
        // every load of the window is issued before the first is used
#pragma unroll
        for (int s = 0; s < 8; ++s)
            f[s] = (((long)vol * nz + 2 * z + (s >> 2)) * ny + 2 * y + ((s >> 1) & 1)) * nx + 2 * x + (s & 1);
        uint4 eq[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) eq[s] = *reinterpret_cast<const uint4*>(e + f[s] * 32 + 8 * j);
        const uint4 gq = *reinterpret_cast<const uint4*>(dp + (long)(i >> 2) * 32 + 8 * j);
#pragma unroll
        for (int s = 0; s < 8; ++s) kq[s] = *reinterpret_cast<const uint4*>(dskip + f[s] * 32 + 8 * j);
#pragma unroll
        for (int s = 0; s < 8; ++s) unpack8(eq[s], ev[s]);
        float g[8];
        unpack8(gq, g);
        int arg[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            // first maximum, tracked by value (no run-time index into ev,
            // which would put the array in scratch memory)
            int best = 0;
            float bv = ev[0][c];
#pragma unroll
            for (int s = 1; s < 8; ++s) {
                const bool gt = ev[s][c] > bv;
                best = gt ? s : best;
                bv = gt ? ev[s][c] : bv;
            }
            arg[c] = best;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            float k[8], o[8];
            unpack8(kq[s], k);
#pragma unroll
            for (int c = 0; c < 8; ++c) o[c] = ev[s][c] > 0.f ? (arg[c] == s ? g[c] : 0.f) + k[c] : 0.f;
            *reinterpret_cast<uint4*>(de + f[s] * 32 + 8 * j) = pack8(o);
        }
    }
}

// Backward data of the transposed convolution: d in[z][y][x][ci] = sum_s
// sum_co g[2z+a][2y+b][2x+c][co] W[s][ci][co], D[ci][voxel] = sum_s W_s
// G_s^T on the MFMA, one wave per run of 32 coarse voxels; masked by the
// ReLU pattern of relu_src when MASK.
template <bool MASK>
__global__ __launch_bounds__(kBlock) void k_upconv_dgrad(UpBwdArgs a) {
    // the wave index read from the first lane: the run, the row bases and the
    // buffer descriptors derived from it are then scalar (no per-lane loop
    // around each buffer access)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int m = lane & 31, h = lane >> 5;
    const int runs = (a.nx + 31) / 32;
    const long total = (long)a.nvol * a.nz * a.ny * runs;
    const long run = (long)blockIdx.x * 4 + wave;
    if (run >= total) return;  // whole waves only; no block barrier below
    const int xr = (int)(run % runs);
    long r = run / runs;
    const int y = (int)(r % a.ny);
    r /= a.ny;
    const int z = (int)(r % a.nz);
    const long vol = r / a.nz;
    const int x = xr * 32 + m;
    const bool xok = x < a.nx;
    const int NZ = 2 * a.nz, NY = 2 * a.ny, NX = 2 * a.nx;
    v8bf gb[8][2], w[8][2];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const long row = ((vol * NZ + 2 * z + (s >> 2)) * NY + 2 * y + ((s >> 1) & 1)) * (long)NX;
        const __amdgpu_buffer_rsrc_t g_rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(a.g) + row * 32, 0, (uint32_t)NX * 64u, kWord3);
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            const uint32_t off = xok ? (uint32_t)((2 * x + (s & 1)) * 64 + 32 * kh + 16 * h) : kOutside;
            gb[s][kh] = __builtin_bit_cast(v8bf, __builtin_amdgcn_raw_buffer_load_b128(g_rs, off, 0, 0));
            w[s][kh] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a.wt + ((s * 2 + kh) * 64 + lane) * 8));
        }
    }
    const long crow = ((vol * a.nz + z) * a.ny + y) * (long)a.nx;
    v4u keep[2];
    if constexpr (MASK) {
        const __amdgpu_buffer_rsrc_t k_rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(a.relu_src) + crow * 32, 0, (uint32_t)a.nx * 64u, kWord3);
#pragma unroll
        for (int p = 0; p < 2; ++p)
            keep[p] = __builtin_amdgcn_raw_buffer_load_b128(k_rs, xok ? (uint32_t)(x * 64 + 32 * p + 16 * h) : kOutside,
                                                            0, 0);
    }
    v16f d = v16f{};
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[s][kh], gb[s][kh], d, 0, 0, 0);
    const __amdgpu_buffer_rsrc_t out_rs =
        __builtin_amdgcn_make_buffer_rsrc(a.out + crow * 32, 0, (uint32_t)a.nx * 64u, kWord3);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        float lo[4], hi[4];  // channels 16 p + 8 h + (0..3, 4..7) after the swap
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(d[8 * p + c]),
                                                             __float_as_uint(d[8 * p + 4 + c]), false, false);
            lo[c] = __uint_as_float(sw[0]);
            hi[c] = __uint_as_float(sw[1]);
        }
        v4u q;
        q[0] = pack2(lo[0], lo[1]);
        q[1] = pack2(lo[2], lo[3]);
        q[2] = pack2(hi[0], hi[1]);
        q[3] = pack2(hi[2], hi[3]);
        if constexpr (MASK) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t u = keep[p][k];
                const uint32_t lo_keep = ((u & 0x8000u) == 0u && (u & 0x7fffu) != 0u) ? 0x0000ffffu : 0u;
                const uint32_t hi_keep = ((u & 0x80000000u) == 0u && (u & 0x7fff0000u) != 0u) ? 0xffff0000u : 0u;
                q[k] &= lo_keep | hi_keep;
            }
        }
        __builtin_amdgcn_raw_buffer_store_b128(q, out_rs, xok ? (uint32_t)(x * 64 + 32 * p + 16 * h) : kOutside, 0, 0);
    }
}

// Weight gradient of the transposed convolution: dW[s][ci][co] = sum over
// coarse voxels of in[v][ci] g[fine(v, s)][co].  Per run of 32 coarse voxels
// the block puts in and the 8 sub-position gradients into LDS channel-major
// ([channel][voxel], so that MFMA operands along the voxel index are
// contiguous); wave w accumulates D_s[ci][co] = In^T G_s for s = 2w, 2w + 1
// over the block's runs and writes its partial sums at the end.
constexpr int kUpWgBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_upconv_wgrad(UpBwdArgs a, float* part) {
    __shared__ __align__(16) uint16_t tin[32][40];    // [ci][voxel], rows padded (80-byte rows)
    __shared__ __align__(16) uint16_t tg[8][32][40];  // [s][co][voxel]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 31, h = lane >> 5;
    const int runs = (a.nx + 31) / 32;
    const long total = (long)a.nvol * a.nz * a.ny * runs;
    const int NZ = 2 * a.nz, NY = 2 * a.ny, NX = 2 * a.nx;
    v16f acc[2] = {v16f{}, v16f{}};
    for (long run = blockIdx.x; run < total; run += gridDim.x) {
        const int xr = (int)(run % runs);
        long r = run / runs;
        const int y = (int)(r % a.ny);
        r /= a.ny;
        const int z = (int)(r % a.nz);
        const long vol = r / a.nz;
        // 9 tensors x 32 voxels x 4 chunks = 1152 chunks of 8 channels
        uint4 q[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int c = tid + k * kBlock;  // chunk: tensor tt (0: in, 1 + s: g_s), voxel vx, channel chunk jj
            const int tt = c / 128, vx = (c / 4) % 32, jj = c % 4;
            const int x = (xr * 32 + vx);
            q[k] = make_uint4(0u, 0u, 0u, 0u);
            if (c < 1152 && x < a.nx) {
                if (tt == 0) {
                    q[k] = *reinterpret_cast<const uint4*>(a.in + (((vol * a.nz + z) * a.ny + y) * (long)a.nx + x) * 32 +
                                                           8 * jj);
                } else {
                    const int s = tt - 1;
                    const long f = ((vol * NZ + 2 * z + (s >> 2)) * NY + 2 * y + ((s >> 1) & 1)) * (long)NX + 2 * x +
                                   (s & 1);
                    q[k] = *reinterpret_cast<const uint4*>(a.g + f * 32 + 8 * jj);
                }
            }
        }
        __syncthreads();  // the previous run's operands are consumed
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int c = tid + k * kBlock;
            if (c < 1152) {
                const int tt = c / 128, vx = (c / 4) % 32, jj = c % 4;
                uint16_t* dst = tt == 0 ? &tin[0][0] : &tg[tt - 1][0][0];
                const uint32_t u[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    dst[(8 * jj + 2 * e) * 40 + vx] = (uint16_t)(u[e] & 0xffffu);
                    dst[(8 * jj + 2 * e + 1) * 40 + vx] = (uint16_t)(u[e] >> 16);
                }
            }
        }
        __syncthreads();
        // A[m = ci][k = voxel]: lane (ci, h) reads voxels 16 kh + 8 h .. + 7 of channel ci
#pragma unroll
        for (int kh = 0; kh < 2; ++kh) {
            const v8bf av = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(&tin[m][16 * kh + 8 * h]));
#pragma unroll
            for (int u2 = 0; u2 < 2; ++u2) {
                const int s = 2 * wave + u2;
                const v8bf bv = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(&tg[s][m][16 * kh + 8 * h]));
                acc[u2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[u2], 0, 0, 0);
            }
        }
    }
    // D[ci][co] in lane co + 32 ((ci / 4) % 2), register (ci / 8) 4 + ci % 4
#pragma unroll
    for (int u2 = 0; u2 < 2; ++u2) {
        const int s = 2 * wave + u2;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int ci = (i / 4) * 8 + 4 * h + (i % 4);
            part[((long)blockIdx.x * 8 + s) * 1024 + ci * 32 + m] = acc[u2][i];
        }
    }
}

// out[e] = sum over blocks of part[block][e] (fixed order), e < n; eight
// independent loads in flight per step.
__global__ __launch_bounds__(kBlock) void k_sum_blocks(const float* part, int blocks, int n, float* out) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    // partials added in block order, 32 loads in flight per thread (the grid
    // is only n / kBlock blocks, so latency, not bandwidth, sets the time)
    float acc = 0.f;
    int b = 0;
    for (; b + 32 <= blocks; b += 32) {
        float q[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) q[u] = part[(long)(b + u) * n + e];
#pragma unroll
        for (int u = 0; u < 32; ++u) acc += q[u];
    }
    for (; b < blocks; ++b) acc += part[(long)b * n + e];
    out[e] = acc;
}

}  // namespace

hipError_t unet_pool(const uint16_t* in, uint16_t* out, int nvol, int nz, int ny, int nx, hipStream_t st) {
    const long total = (long)nvol * (nz / 2) * (ny / 2) * (nx / 2) * 4;
    if (total <= 0) return hipSuccess;
    long blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_pool2, dim3((unsigned)blocks), dim3(kBlock), 0, st, in, out, nvol, nz, ny, nx);
    return hipGetLastError();
}

hipError_t unet_upconv(const UpArgs& a, hipStream_t st) {
    if ((long)a.nx * 2 * 64 >= (long)kOutside) return hipErrorInvalidValue;
    const long runs = (long)a.nvol * a.nz * a.ny * ((a.nx + 31) / 32);
    if (runs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_upconv, dim3((unsigned)((runs + 3) / 4)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t unet_prep_up(const float* W, int transposed, uint16_t* wf, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_up, dim3(8 * 2 * 64 * 8 / kBlock), dim3(kBlock), 0, st, W, transposed, wf);
    return hipGetLastError();
}

hipError_t unet_fold_bn(const float* W, const float* gamma, const float* beta, const float* mean, const float* var,
                        int cin, float* wout, float* bout, hipStream_t st) {
    const int n = 27 * cin * 32 + 32;
    hipLaunchKernelGGL(k_fold_bn, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, W, gamma, beta, mean, var, cin,
                       wout, bout);
    return hipGetLastError();
}

static unsigned grid_of(long work, long cap) {
    long b = (work + kBlock - 1) / kBlock;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

size_t unet_chan_part_bytes() { return (size_t)kChanBlocks * 32 * 2 * sizeof(double); }

hipError_t unet_chan_sums(int mode, const uint16_t* X, const uint16_t* Y, const float* mean, const float* rstd,
                          long nvox, double* part, int* blocks, hipStream_t st) {
    long b = (nvox + 63) / 64;
    if (b > kChanBlocks) b = kChanBlocks;
    if (b < 1) b = 1;
    *blocks = (int)b;
    if (mode == 0)
        hipLaunchKernelGGL(k_chan_sums<0>, dim3((unsigned)b), dim3(kBlock), 0, st, X, Y, mean, rstd, nvox, part);
    else
        hipLaunchKernelGGL(k_chan_sums<1>, dim3((unsigned)b), dim3(kBlock), 0, st, X, Y, mean, rstd, nvox, part);
    return hipGetLastError();
}

hipError_t unet_chan_finalize(int mode, const double* part, int blocks, long m, const float* gamma, const float* beta,
                              float* mean, float* rstd, float* A, float* B, float* C, float* run_mean,
                              float* run_var, float* out0, float* out1, hipStream_t st) {
    hipLaunchKernelGGL(k_chan_finalize, dim3(1), dim3(1024), 0, st, mode, part, blocks, m, gamma, beta, mean, rstd, A,
                       B, C, run_mean, run_var, out0, out1);
    return hipGetLastError();
}

hipError_t unet_affine(const uint16_t* X, const uint16_t* Y, const float* A, const float* B, const float* C, int relu,
                       long nvox, uint16_t* out, hipStream_t st) {
    const dim3 g(grid_of(nvox * 4, 1 << 20)), b(kBlock);
    if (Y != nullptr && relu) hipLaunchKernelGGL((k_affine<true, true>), g, b, 0, st, X, Y, A, B, C, nvox, out);
    else if (Y != nullptr) hipLaunchKernelGGL((k_affine<true, false>), g, b, 0, st, X, Y, A, B, C, nvox, out);
    else if (relu) hipLaunchKernelGGL((k_affine<false, true>), g, b, 0, st, X, Y, A, B, C, nvox, out);
    else hipLaunchKernelGGL((k_affine<false, false>), g, b, 0, st, X, Y, A, B, C, nvox, out);
    return hipGetLastError();
}

hipError_t unet_pool_bwd(const uint16_t* e, const uint16_t* dp, const uint16_t* dskip, uint16_t* de, int nvol, int nz,
                         int ny, int nx, hipStream_t st) {
    const long total = (long)nvol * (nz / 2) * (ny / 2) * (nx / 2) * 4;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_of(total, 16384)), dim3(kBlock), 0, st, e, dp, dskip, de, nvol, nz, ny, nx);
    return hipGetLastError();
}

hipError_t unet_upconv_dgrad(const UpBwdArgs& a, hipStream_t st) {
    if ((long)a.nx * 2 * 64 >= (long)kOutside) return hipErrorInvalidValue;
    const long runs = (long)a.nvol * a.nz * a.ny * ((a.nx + 31) / 32);
    if (runs <= 0) return hipSuccess;
    const dim3 g((unsigned)((runs + 3) / 4)), b(kBlock);
    if (a.relu_src != nullptr) hipLaunchKernelGGL(k_upconv_dgrad<true>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_upconv_dgrad<false>, g, b, 0, st, a);
    return hipGetLastError();
}

size_t unet_upwgrad_part_bytes() { return (size_t)kUpWgBlocks * 8 * 1024 * sizeof(float); }

hipError_t unet_upconv_wgrad(const UpBwdArgs& a, float* part, float* gw, hipStream_t st) {
    const long runs = (long)a.nvol * a.nz * a.ny * ((a.nx + 31) / 32);
    const int blocks = (int)(runs < kUpWgBlocks ? (runs < 1 ? 1 : runs) : kUpWgBlocks);
    hipLaunchKernelGGL(k_upconv_wgrad, dim3(blocks), dim3(kBlock), 0, st, a, part);
    hipLaunchKernelGGL(k_sum_blocks, dim3(8 * 1024 / kBlock), dim3(kBlock), 0, st, (const float*)part, blocks, 8 * 1024,
                       gw);
    return hipGetLastError();
}

}  // namespace clampk
