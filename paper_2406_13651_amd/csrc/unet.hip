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
    const int cz = nz / 2, cy = ny / 2, cx = nx / 2;
    const long total = (long)nvol * cz * cy * cx * 4;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < total; i += (long)gridDim.x * kBlock) {
        const int j = (int)(i & 3);
        long v = i >> 2;
        const int x = (int)(v % cx);
        v /= cx;
        const int y = (int)(v % cy);
        v /= cy;
        const int z = (int)(v % cz);
        const long vol = v / cz;
        uint4 m;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const long f = ((vol * nz + 2 * z + (s >> 2)) * ny + 2 * y + ((s >> 1) & 1)) * nx + 2 * x + (s & 1);
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
        *reinterpret_cast<uint4*>(out + (i >> 2) * 32 + j * 8) = m;
    }
}

// One wave per run of 32 coarse voxels along x (lane m = voxel x0 + m, half
// h).  D[co][voxel] = W_s^T X^T for each sub-position s on the MFMA (K = 32
// input channels as two halves): lane (m, h) gets channels 8 g + 4 h + 0..3
// (g = 0..3) of output voxel (2z + a, 2y + b, 2(x0 + m) + c); with the bias
// added, a swap between the lane halves gives it 8 consecutive channels 16 p +
// 8 h + 0..7 (p = 0, 1) in fp32, to which the skip is added before rounding.
__global__ __launch_bounds__(kBlock) void k_upconv(UpArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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

// Fragment e = ((s 2 + kh) 64 + l) 8 + k8 holds W[s][ci = 16 kh + 8 (l / 32) + k8][co = l % 32]
// (the A operand W^T of sub-position s, input-channel half kh).
__global__ __launch_bounds__(kBlock) void k_prep_up(const float* W, uint16_t* wf) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= 8 * 2 * 64 * 8) return;
    const int k8 = e % 8, l = (e / 8) % 64, kh = (e / 512) % 2, s = e / 1024;
    const int ci = 16 * kh + 8 * (l / 32) + k8, co = l % 32;
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

hipError_t unet_prep_up(const float* W, uint16_t* wf, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_up, dim3(8 * 2 * 64 * 8 / kBlock), dim3(kBlock), 0, st, W, wf);
    return hipGetLastError();
}

hipError_t unet_fold_bn(const float* W, const float* gamma, const float* beta, const float* mean, const float* var,
                        int cin, float* wout, float* bout, hipStream_t st) {
    const int n = 27 * cin * 32 + 32;
    hipLaunchKernelGGL(k_fold_bn, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, W, gamma, beta, mean, var, cin,
                       wout, bout);
    return hipGetLastError();
}

}  // namespace clampk
