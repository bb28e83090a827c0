// The 3D operator with a zero-padded aperture (Sec. II-B eq. A with the
// orthonormal 3D DFT; Sec. II-A: the pupil stack is zero-padded in range, so
// only K of the nz range frequencies hold data).  The aperture is a cylinder:
// the pupil disk times the K range frequencies nearest DC.  A = D(a) F3 runs
// as the per-slice pipeline (column and row passes of the 2D DFT) plus a
// range pass on the pupil samples only:
//   A^H R = F2^H [ F_z^H (R zero-filled outside the box) ],
//   A d   = box crop of F_z (F2 d restricted to the pupil).
// Compact range layouts, per look: [K][P] (box index k, pupil sample p) for
// the residual and A d, [nz][P] for the per-slice compact data the column
// passes read and write.  Box index k holds range frequency w = k for
// k < ceil(K/2) and w = nz - K + k otherwise.
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "internal.h"
#include "passes.hpp"

namespace clampk {

constexpr int kZCols = 16;  // pupil samples per range-pass block

static int range_grid_cap(size_t work, int cap) {
    const size_t g = (work + kBlock - 1) / kBlock;
    return (int)(g < 1 ? 1 : (g < (size_t)cap ? g : (size_t)cap));
}

// Box index of range frequency w, or -1 outside the box.
__device__ __forceinline__ int box_index(int w, int nz, int K) {
    const int hi = (K + 1) / 2;  // non-negative frequencies 0 .. hi - 1
    if (w < hi) return w;
    const int k = K - (nz - w);
    return k >= hi ? k : -1;
}
__device__ __forceinline__ int box_freq(int k, int nz, int K) { return k < (K + 1) / 2 ? k : nz - K + k; }

// Range DFT of kZCols pupil samples of one look.  S = +1: inverse, box [K][P]
// in, all slices [nz][P] out, part = sum |in|^2.  S = -1: forward, [nz][P]
// in, box [K][P] out, part = sum |out|^2.  Orthonormal (1/sqrt(nz)).
template <int NZ, int S>
__global__ __launch_bounds__(kBlock) void k_zpass(ZArgs a) {
    constexpr int TPC = kBlock / kZCols;  // threads per column
    static_assert(NZ % TPC == 0, "range length must be a multiple of the threads per column");
    __shared__ float2 tw[NZ];
    __shared__ float2 tile[NZ * kZCols];
    const SceneTables& s = a.s;
    const int P = s.P, K = s.K;
    const int tiles = (P + kZCols - 1) / kZCols;
    const int look = blockIdx.x / tiles, tile_i = blockIdx.x % tiles;
    const int tid = threadIdx.x, c = tid % kZCols, t = tid / kZCols;
    const int p = tile_i * kZCols + c;
    const bool col_ok = p < P;
    const float scale = rsqrtf((float)NZ);
    float acc = 0.f;
    // every load of the column first (positions outside the box or past P
    // read a valid sample and are replaced by zero), then the tile stores
    const int pc = col_ok ? p : P - 1;
    float2 vin[NZ / TPC];
#pragma unroll
    for (int j = 0; j < NZ / TPC; ++j) {
        const int z = t + j * TPC;
        if constexpr (S > 0) {
            const int k = box_index(z, NZ, K);
            vin[j] = a.in[((size_t)look * K + (k >= 0 ? k : 0)) * P + pc];
        } else {
            vin[j] = a.in[((size_t)look * NZ + z) * P + pc];
        }
    }
    for (int i = tid; i < NZ; i += kBlock) tw[i] = s.tw_z[i];
#pragma unroll
    for (int j = 0; j < NZ / TPC; ++j) {
        const int z = t + j * TPC;
        float2 v = make_float2(0.f, 0.f);
        if constexpr (S > 0) {
            if (col_ok && box_index(z, NZ, K) >= 0) {
                v = vin[j];
                acc += cabs2(v);
            }
        } else {
            if (col_ok) v = vin[j];
        }
        tile[z * kZCols + c] = v;
    }
    fft_lds<NZ, TPC, S, 0>(tile + c, kZCols, t, tw);
#pragma unroll
    for (int j = 0; j < NZ / TPC; ++j) {
        const int z = t + j * TPC;
        const float2 v = cscale(tile[z * kZCols + c], scale);
        if constexpr (S > 0) {
            if (col_ok) a.out[((size_t)look * NZ + z) * P + p] = v;
        } else {
            const int k = box_index(z, NZ, K);
            if (col_ok && k >= 0) {
                a.out[((size_t)look * K + k) * P + p] = v;
                acc += cabs2(v);
            }
        }
    }
    double sum[1] = {acc};
    block_sum_store<1>(sum, a.part + (size_t)look * tiles + tile_i);
}

// out[look][k][p] = y[look][w_k][pupil position of p] (and keep * that into
// out_keep when given); part[look][block] = sum |y|^2 over the support.
__global__ __launch_bounds__(kBlock) void k_range_gather(SceneTables s, const float2* y, float2* out,
                                                         float2* out_keep, float keep, double* part) {
    const int look = blockIdx.y;
    const size_t per = (size_t)s.K * s.P;
    const size_t slice = (size_t)s.ny * s.nx;
    float acc = 0.f;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < per; i += (size_t)gridDim.x * kBlock) {
        const int k = (int)(i / s.P), p = (int)(i % s.P);
        const float2 v = y[((size_t)look * s.nz + box_freq(k, s.nz, s.K)) * slice + s.cpos[p]];
        out[(size_t)look * per + i] = v;
        if (out_keep != nullptr) out_keep[(size_t)look * per + i] = cscale(v, keep);
        acc += cabs2(v);
    }
    double sum[1] = {acc};
    block_sum_store<1>(sum, part + (size_t)look * gridDim.x + blockIdx.x);
}

// full[look][w][u][v] = cmp[look][k(w)][pidx(u, v)] on the support, 0 elsewhere.
__global__ __launch_bounds__(kBlock) void k_range_scatter(SceneTables s, size_t total, const float2* cmp,
                                                          float2* full) {
    const size_t slice = (size_t)s.ny * s.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
        const size_t zl = i / slice;
        const int look = (int)(zl / s.nz), w = (int)(zl % s.nz);
        const int k = box_index(w, s.nz, s.K);
        const int p = s.pidx[i % slice];
        float2 v = make_float2(0.f, 0.f);
        if (k >= 0 && p >= 0) v = cmp[((size_t)look * s.K + k) * s.P + p];
        full[i] = v;
    }
}

int zpass_blocks(const SceneTables& s) { return (s.P + kZCols - 1) / kZCols; }
int gather_blocks(const SceneTables& s) { return range_grid_cap((size_t)s.K * s.P, 1024); }

hipError_t launch_zpass(int dir, const ZArgs& a, hipStream_t st) {
    if (a.looks <= 0) return hipSuccess;
    const dim3 grid((unsigned)(a.looks * zpass_blocks(a.s)));
    switch (a.s.nz) {
#define CASE(N)                                                                                        \
    case N:                                                                                            \
        if (dir > 0) hipLaunchKernelGGL((k_zpass<N, 1>), grid, dim3(kBlock), 0, st, a);                \
        else hipLaunchKernelGGL((k_zpass<N, -1>), grid, dim3(kBlock), 0, st, a);                       \
        break;
        CLAMP_RANGE_SIZES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_range_gather(const SceneTables& s, int looks, const float2* y, float2* out, float2* out_keep,
                               float keep, double* part, hipStream_t st) {
    if (looks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_range_gather, dim3(gather_blocks(s), looks), dim3(kBlock), 0, st, s, y, out, out_keep, keep,
                       part);
    return hipGetLastError();
}

hipError_t launch_range_scatter(const SceneTables& s, int looks, const float2* cmp, float2* full, hipStream_t st) {
    const size_t total = (size_t)looks * s.nz * s.ny * s.nx;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_range_scatter, dim3(range_grid_cap(total, 8192)), dim3(kBlock), 0, st, s, total, cmp, full);
    return hipGetLastError();
}

}  // namespace clampk
