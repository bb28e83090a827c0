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

constexpr int kCnnBlock = 256;

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void tap_offset(int t, int& dz, int& dy, int& dx) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// Row index of the MFMA output register i of lane l (the column is l % 32).
__device__ __forceinline__ int d_row(int l, int i) { return (l / 32) * 4 + (i / 4) * 8 + (i % 4); }

// ---------------------------------------------------------------------------
// Convolution (forward or backward-data) on 32-voxel x runs.
template <int CIN, int EPI>
__global__ __launch_bounds__(kCnnBlock) void k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * (kCnnBlock / 64) + (threadIdx.x >> 6);
    const int tiles_x = a.nx / 32;
    const long tiles = (long)a.nvol * a.nz * a.ny * tiles_x;
    if (tile >= tiles) return;  // no barriers in this kernel
    const int xt = tile % tiles_x;
    long r = tile / tiles_x;
    const int y = (int)(r % a.ny);
    r /= a.ny;
    const int z = (int)(r % a.nz);
    const int n = (int)(r / a.nz);
    const int m = lane & 31;
    const int kh = (lane >> 5) * 4;
    const int x = xt * 32 + m;
    v16f acc = {};
    for (int t = 0; t < 27; ++t) {
        int dz, dy, dx;
        tap_offset(t, dz, dy, dx);
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        const bool ok = zz >= 0 && zz < a.nz && yy >= 0 && yy < a.ny && xx >= 0 && xx < a.nx;
        const uint16_t* src = a.in + ((((long)n * a.nz + (ok ? zz : 0)) * a.ny + (ok ? yy : 0)) * a.nx + (ok ? xx : 0)) * CIN;
        const uint16_t* wt = a.w + ((long)t * 32 + m) * CIN;
#pragma unroll
        for (int cb = 0; cb < CIN / 8; ++cb) {
            v4s av = {0, 0, 0, 0};
            if (ok) av = *reinterpret_cast<const v4s*>(src + cb * 8 + kh);
            const v4s bv = *reinterpret_cast<const v4s*>(wt + cb * 8 + kh);
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
        }
    }
    const long row0 = (((long)n * a.nz + z) * a.ny + y) * a.nx + xt * 32;
    const int ch = lane & 31;
    float scale = 1.f;
    if constexpr (EPI == EPI_FINAL) {
        if (a.scale != nullptr) scale = *a.scale;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const long v = row0 + d_row(lane, i);
        const float val = acc[i];
        if constexpr (EPI == EPI_RELU) {
            a.out[v * 32 + ch] = f2bf(fmaxf(val + a.bias[ch], 0.f));
        } else if constexpr (EPI == EPI_FINAL) {
            if (ch == 0) a.out_f32[v] = a.xin[v] + scale * (val + a.bias[0]);
        } else {  // EPI_DGRAD: multiply by the ReLU mask of the layer input
            const float keep = bf2f(a.relu_src[v * 32 + ch]) > 0.f ? 1.f : 0.f;
            a.out[v * 32 + ch] = f2bf(val * keep);
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

// grad[W + (t * cin + ci) * cout + co] = sum over chunks of part[c][t][co][ci];
// grad[b + co] = sum over chunks of bias partials.
__global__ __launch_bounds__(kCnnBlock) void k_wgrad_reduce(const float* part, int chunks, int cin, int cout,
                                                            float* gw) {
    const int e = blockIdx.x * kCnnBlock + threadIdx.x;
    if (e >= 27 * cin * cout) return;
    const int co = e % cout;
    const int ci = (e / cout) % cin;
    const int t = e / (cout * cin);
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[((long)c * 27 + t) * 1024 + co * 32 + ci];
    gw[e] = (float)s;
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
__global__ __launch_bounds__(kCnnBlock) void k_bias_reduce(const float* part, int nblocks, int cout, float* gb) {
    const int co = threadIdx.x;
    if (co >= cout) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * 32 + co];
    gb[co] = (float)s;
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

// BF16 weight copies of one layer from the fp32 parameters W[t][cin][cout]:
// forward wf[t][32][CINP] (output channel major) and backward-data
// wd[t][32][COUTP] = W[26 - t] with the channel roles swapped; padded
// entries are zero.  Also the zero-padded bias copy.
__global__ __launch_bounds__(kCnnBlock) void k_prep(const float* W, const float* b, int cin, int cout, int cinp,
                                                    int coutp, uint16_t* wf, uint16_t* wd, float* bias32) {
    const int e = blockIdx.x * kCnnBlock + threadIdx.x;
    if (e < 27 * 32 * cinp) {  // wf[t][n][k]
        const int k = e % cinp, nn = (e / cinp) % 32, t = e / (cinp * 32);
        wf[e] = (k < cin && nn < cout) ? f2bf(W[(t * cin + k) * cout + nn]) : (uint16_t)0;
    }
    if (wd != nullptr && e < 27 * 32 * coutp) {  // wd[t][n = ci][k = co]
        const int k = e % coutp, nn = (e / coutp) % 32, t = e / (coutp * 32);
        wd[e] = (k < cout && nn < cin) ? f2bf(W[((26 - t) * cin + nn) * cout + k]) : (uint16_t)0;
    }
    if (e < 32) bias32[e] = e < cout ? b[e] : 0.f;
}

// ---------------------------------------------------------------------------
// Launchers
static int grid_for(long work, int per_block, int cap) {
    long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

hipError_t cnn_conv(int cin, int epi, const ConvArgs& a, hipStream_t st) {
    const long tiles = (long)a.nvol * a.nz * a.ny * (a.nx / 32);
    const dim3 grid((unsigned)((tiles + 3) / 4));
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
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((27 * cin * cout + kCnnBlock - 1) / kCnnBlock), dim3(kCnnBlock), 0, st,
                       a.part, chunks, cin, cout, gw);
    const int nb = grid_for(a.nvox, 8, 2048);
    if (cg == 8)
        hipLaunchKernelGGL(k_bias_partial<8>, dim3(nb), dim3(kCnnBlock), 0, st, a.g, a.nvox, bias_part);
    else
        hipLaunchKernelGGL(k_bias_partial<32>, dim3(nb), dim3(kCnnBlock), 0, st, a.g, a.nvox, bias_part);
    hipLaunchKernelGGL(k_bias_reduce, dim3(1), dim3(kCnnBlock), 0, st, bias_part, nb, cout, gb);
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

hipError_t cnn_prep(const float* W, const float* b, int cin, int cout, int cinp, int coutp, uint16_t* wf,
                    uint16_t* wd, float* bias32, hipStream_t st) {
    const int n = 27 * 32 * (cinp > coutp ? cinp : coutp);
    hipLaunchKernelGGL(k_prep, dim3((n + kCnnBlock - 1) / kCnnBlock), dim3(kCnnBlock), 0, st, W, b, cin, cout, cinp,
                       coutp, wf, wd, bias32);
    return hipGetLastError();
}

}  // namespace clampk
