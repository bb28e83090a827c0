// Work items of the forward-agent passes as device functions.  A work item
// is one unit that a block processes: a group of rows of one slice of one
// look (row passes), a tile of band columns of one slice of one look (column
// passes), or one look (step size and diagnostics).  The single-scene
// kernels map one block to one item; the batched kernels walk a queue of
// items of many scenes, choosing the FFT length of each item at run time.
// LDS buffers are passed in, so a batched kernel can share one allocation
// between items of different lengths.
#pragma once

#include <math.h>

#include "fft.hpp"
#include "internal.h"

namespace clampk {

constexpr int kRowPad = 4;  // one float2 of LDS padding per 16 row samples

// Non-temporal loads and stores, for streams that do not fit the caches
// between their writer and reader anyway: the pointwise streams of the update
// pass and the Mann step, the residual update, and the band buffers between
// the column and row passes.  They then do not displace cached data that the
// other passes reuse (measured at 256x256x64, 16 looks: update pass 428 ->
// 355 us, whole iteration 1.30 -> 1.16 ms).
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ void st_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

template <int N>
__host__ __device__ constexpr int row_lds_floats2() {
    return rows_per_block(N) * lds_len<N, kRowPad>();
}

// Sum of K doubles over the block, written by thread 0 to out[0..K).
template <int K>
__device__ __forceinline__ void block_sum_store(double (&v)[K], double* out) {
    __shared__ double red[K][kBlock / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        v[k] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += red[k][w];
            out[k] = s;
        }
    }
    __syncthreads();  // red may be reused by the next item
}

// v[k] += p[i * stride + k] (k < K) for i = threadIdx.x, + kBlock, ... below
// count, with eight rows of loads in flight per thread (rows past count
// re-read the last one and are not added).  The order of the additions is
// fixed, so the sums are deterministic.
template <int K>
__device__ __forceinline__ void strided_sums(const double* p, int count, int stride, double* v) {
    for (int i0 = threadIdx.x; i0 < count; i0 += 8 * kBlock) {
        double x[8][K];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * kBlock;
            const double* q = p + (size_t)(i < count ? i : count - 1) * stride;
#pragma unroll
            for (int k = 0; k < K; ++k) x[u][k] = q[k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (i0 + u * kBlock < count) {
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] += x[u][k];
            }
        }
    }
}

__device__ __forceinline__ void wave_or_fault(uint32_t bits, uint32_t* fault) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off);
    if ((threadIdx.x & 63) == 0 && bits != 0u && fault != nullptr) atomicOr(fault, bits);
}

// Read-only device tables (the batch's scene table and work queues) seen
// through the constant address space.  Nothing writes them while a kernel
// runs, so a read at a wave-uniform address is a scalar load that the
// compiler may issue again where a field is used instead of holding the
// whole block in registers -- as it does for kernel arguments.
// (The host pass of this file compiles the kernels' declarations only, and
// has no constant address space.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using ConstAS = const __attribute__((address_space(4))) T;
#else
template <class T>
using ConstAS = const T;
#endif
template <class T>
__device__ __forceinline__ ConstAS<T>& const_ref(const T* p) {
    return *(ConstAS<T>*)p;
}

// Copy of a wave-uniform argument block from device memory into scalar
// registers: the private copy cannot alias the item's stores, and
// readfirstlane keeps it out of the vector register file.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "argument blocks are whole dwords");
    T out;
    const int* src = reinterpret_cast<const int*>(p);
    int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// Interval factor and the derived constants of the surrogate r-update.
struct BetaVals {
    float beta, inv_beta, k_up, k_dn;
};
__host__ __device__ inline BetaVals beta_vals(double beta) {
    BetaVals b;
    b.beta = (float)beta;
    b.inv_beta = (float)(1.0 / beta);
    b.k_up = (float)((1.0 + beta) / (beta * beta));  // xi = beta r'
    b.k_dn = (float)(beta * (1.0 + beta));           // xi = r' / beta
    return b;
}

// Exact proximal map of the EM surrogate for one voxel (eq. surrogate-prox):
// argmin over r > 0 of log r + s/r + (r - v)^2 / (2 sigma^2).  Its stationary
// points are the positive roots of r^3 - v r^2 + sigma^2 r - sigma^2 s (the
// derivative times sigma^2 r^2, negative at r = 0, so a positive root exists).
// With r = t + v/3 the cubic is t^3 + p t + q; its roots come from the
// trigonometric form when it has three real roots and from Cardano's form
// (the cube root taken on the side without cancellation) when it has one,
// each polished by two Newton steps, all in float64.  The positive root with
// the smallest objective is returned (the objective is not convex for r > 2 s
// and can have two local minima).
__device__ __forceinline__ float exact_prox(float sf, float vf, float s2f) {
    const double s = sf, v = vf, q2 = s2f;
    const double sh = v / 3.0;
    const double p = q2 - v * v / 3.0;
    const double q = -2.0 * v * v * v / 27.0 + v * q2 / 3.0 - q2 * s;
    const double disc = 0.25 * q * q + p * p * p / 27.0;
    double root[3];
    int nr;
    if (disc > 0.0) {
        const double a = -0.5 * q;
        const double u = cbrt(a + copysign(sqrt(disc), a));
        root[0] = (u != 0.0 ? u - p / (3.0 * u) : 0.0) + sh;
        nr = 1;
    } else {
        const double m = 2.0 * sqrt(fmax(-p / 3.0, 0.0));
        const double c = m > 0.0 ? fmin(fmax(3.0 * q / (p * m), -1.0), 1.0) : 0.0;
        const double th = acos(c) / 3.0;
        const double third = 2.0943951023931954923;  // 2 pi / 3
        root[0] = m * cos(th) + sh;
        root[1] = m * cos(th - third) + sh;
        root[2] = m * cos(th - 2.0 * third) + sh;
        nr = 3;
    }
    double best = 0.0, best_phi = 0.0;
    bool found = false;
    for (int k = 0; k < nr; ++k) {
        double r = root[k];
        for (int it = 0; it < 2; ++it) {
            const double f = ((r - v) * r + q2) * r - q2 * s;
            const double df = (3.0 * r - 2.0 * v) * r + q2;
            if (df != 0.0) r -= f / df;
        }
        if (r > 0.0) {
            const double phi = log(r) + s / r + (r - v) * (r - v) / (2.0 * q2);
            if (!found || phi < best_phi) {
                best = r;
                best_phi = phi;
                found = true;
            }
        }
    }
    return (float)best;  // 0 (flagged by the caller) only if no positive root was found
}

// Surrogate r-update of one voxel at the anchor r0 and prox point v, with the
// updated mean m1: covariance diagonal c = sigma_w^2 r0 / (alpha r0 +
// sigma_w^2) (A^H A ~ alpha I), s = c + |m1|^2, then the quadratic surrogate
// of App. A (ROW_UPDATE) or the exact surrogate prox (ROW_UPDATE_EXACT).
// Fault bits: 1 for a non-finite result or mean, 2 for r <= 0.
template <int MODE, class A>
__device__ __forceinline__ float r_update_voxel(const A& a, const BetaVals& bv, float r0, float v, float2 m1,
                                                uint32_t& fb) {
    const float c = a.s2w * r0 / (a.alpha * r0 + a.s2w);
    const float sv = c + cabs2(m1);
    float rn;
    if constexpr (MODE == ROW_UPDATE_EXACT) {
        rn = exact_prox(sv, v, a.sigma2);
        if (!(rn == rn) || !isfinite(m1.x) || !isfinite(m1.y)) fb |= 1u;
    } else {
        // quadratic surrogate of r/r' + s/r, interpolating its derivative at
        // r' and xi; written with s/r' first so that small anchors stay in
        // float32 range
        const float inv = 1.f / r0;
        const float sr = sv * inv;
        const float dq = inv * (1.f - sr);                  // q'(r')
        const float D = dq + (r0 - v) * a.inv_sigma2;       // rho'(r')
        const bool down = D > 0.f;
        const float xi = down ? r0 * bv.inv_beta : r0 * bv.beta;
        const float qa = sr * inv * inv * (down ? bv.k_dn : bv.k_up);
        const float qb = dq - qa * r0;
        rn = (v - a.sigma2 * qb) / (1.f + a.sigma2 * qa);
        if (!(rn == rn) || !isfinite(m1.x) || !isfinite(m1.y)) fb |= 1u;
        rn = fminf(fmaxf(rn, fminf(r0, xi)), fmaxf(r0, xi));
    }
    if (!(rn > 0.f)) fb |= 2u;
    return rn;
}

// LDS buffers of a row item: twiddles, band position and band column tables
// (length NX each) and the padded row buffers.
struct RowLds {
    float2* tw;
    int* bpos;
    int* bcol;
    float2* buf;
};

// Row transform of h (h[k] = element t + k TR of the row): in registers where
// fft_regs applies (power-of-two rows), else through rb with fft_lds.  With
// OUT_REGS the result returns to h; otherwise it is left in rb in natural
// order, for gathers across the row by the row's own wave.
template <int NX, int TR, int S, int PAD, bool OUT_REGS, int PX>
__device__ __forceinline__ void row_fft(float2 (&h)[PX], float2* rb, int t, const float2* tw) {
    if constexpr (NX % TR == 0 && fft_regs_ok<NX, TR>()) {
        fft_regs<NX, TR, S, PAD, true, OUT_REGS, true>(h, rb, 1, t, tw);
    } else {
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            if (NX % TR == 0 || x < NX) rb[lds_pos<PAD>(x)] = h[k];
        }
        fft_lds<NX, TR, S, PAD, true>(rb, 1, t, tw);
        if constexpr (OUT_REGS) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) h[k] = rb[lds_pos<PAD>(x)];
            }
        }
    }
}

// Pointwise step of the gradient pass on one row held in h (the inverse row
// FFT of the band already applied): d = A^H r / sigma_w^2 - omega mu with
// omega = 1 / (r' + sigma_w^2 / alpha), written back into h, plus the
// thread's shares of ||d||^2, sum omega |d|^2 and sum omega |mu|^2.
template <int NX, int TR, int PX, class A>
__device__ __forceinline__ void row_grad_pointwise(const A& a, float2 (&h)[PX], int t, const float2 (&m)[PX],
                                                   const float (&rp)[PX], float& dd, float& wd, float& wm) {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int x = t + k * TR;
        if (NX % TR == 0 || x < NX) {
            const float2 ahr = cscale(h[k], a.scale);
            const float om = 1.f / (rp[k] + a.floor_w);
            const float2 d = make_float2(ahr.x * a.inv_s2w - om * m[k].x, ahr.y * a.inv_s2w - om * m[k].y);
            h[k] = d;
            const float d2 = cabs2(d);
            dd += d2;
            wd += om * d2;
            wm += om * cabs2(m[k]);
        }
    }
}

// ---------------------------------------------------------------------------
// Row pass over rows [rgroup * RPB, rgroup * RPB + RPB) of look `look`;
// `slot` indexes the look's partial-sum slots.  `load_tables` reloads the
// row tables (the caller skips it when the previous item had the same scene).
template <int NX, int MODE, class A>
__device__ __forceinline__ void row_item(const A& a, int look, int rgroup, size_t slot, const RowLds& L,
                                         bool load_tables, BetaVals bv) {
    constexpr int TR = row_threads(NX);
    constexpr int RPB = rows_per_block(NX);
    constexpr int PX = (NX + TR - 1) / TR;          // row samples per thread
    constexpr int PAD = kRowPad;
    constexpr int RS = lds_len<NX, PAD>();          // padded row length in LDS
    // ROW_UPDATE_EXACT is the update pass with the exact surrogate prox in
    // place of the quadratic surrogate (a separate instantiation, so that the
    // float64 root solve does not raise the register count of the other)
    constexpr bool UPD = (MODE == ROW_UPDATE || MODE == ROW_UPDATE_EXACT);
    constexpr bool FUSED = (MODE == ROW_GRAD || UPD);
    // Stream prefetch pays off for the gradient pass; the update pass already
    // runs near the read/write bandwidth ceiling and loads its streams late.
    constexpr bool PREFETCH = (MODE == ROW_GRAD);
    const auto& s = a.s;
    const int tid = threadIdx.x;
    const int ri = tid / TR, t = tid % TR;
    const int rows = s.nz * s.ny;
    const int row = rgroup * RPB + ri;
    const bool active = row < rows;
    const size_t img = ((size_t)look * rows + (active ? row : 0)) * NX;
    const int arow = active ? row : 0;
    const size_t band = ((size_t)look * s.nz + arow / s.ny) * s.ny * s.Bs + band_row_off(arow % s.ny, s.ny);

    float2 m[FUSED ? PX : 1];
    float rp[FUSED ? PX : 1];
    float wv[UPD ? PX : 1];
    auto load_streams = [&]() {
        if (active) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) {
                    if constexpr (UPD) {
                        m[k] = ld_stream(&a.mu[img + x]);
                        rp[k] = ld_stream(&a.r[img + x]);
                        wv[k] = ld_stream(&a.w[img + x]);
                    } else {
                        m[k] = a.mu[img + x];
                        rp[k] = a.r[img + x];
                    }
                }
            }
        }
    };
    __syncthreads();  // the previous item's readers of the LDS buffers are done
    if (load_tables) {
        for (int i = tid; i < NX; i += kBlock) {
            L.tw[i] = s.tw_x[i];
            L.bpos[i] = s.band_pos[i];
            const int bc = s.band_cols[i < s.B ? i : 0];  // unconditional: one wait for all three tables
            L.bcol[i] = i < s.B ? bc : 0;
        }
        __syncthreads();
    }
    float2* rb = L.buf + ri * RS;

    // the row in registers: h[k] = element t + k TR (zero for inactive rows)
    float2 h[PX];
    if constexpr (MODE == ROW_FWD) {
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            h[k] = (active && (NX % TR == 0 || x < NX)) ? a.img_in[img + x] : make_float2(0.f, 0.f);
        }
    } else {
        // The row's band samples: all PX loads are issued before the first
        // is used (samples off the band read the row's first band sample and
        // are replaced by zero), then the pointwise streams are prefetched
        // behind them.
        float2 bin[PX];
        int bp[PX];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            bp[k] = (active && (NX % TR == 0 || x < NX)) ? L.bpos[x] : -1;
            bin[k] = ld_stream(a.band_in + band + (bp[k] >= 0 ? bp[k] : 0));  // inactive rows read row 0
        }
        if constexpr (PREFETCH) load_streams();
#pragma unroll
        for (int k = 0; k < PX; ++k) h[k] = bp[k] >= 0 ? bin[k] : make_float2(0.f, 0.f);
    }

    if constexpr (MODE == ROW_INV) {
        row_fft<NX, TR, +1, PAD, true>(h, rb, t, L.tw);
        if (active) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) a.img_out[img + x] = cscale(h[k], a.scale);
            }
        }
    } else if constexpr (MODE == ROW_FWD) {
        row_fft<NX, TR, -1, PAD, false>(h, rb, t, L.tw);
        if (active)
            for (int b = t; b < s.B; b += TR)
                a.band_out[band + band_col_off(b, s.ny)] = cscale(rb[lds_pos<PAD>(L.bcol[b])], a.scale);
    } else if constexpr (MODE == ROW_GRAD) {
        row_fft<NX, TR, +1, PAD, true>(h, rb, t, L.tw);
        float dd = 0.f, wd = 0.f, wm = 0.f;
        if (active) row_grad_pointwise<NX, TR>(a, h, t, m, rp, dd, wd, wm);
        row_fft<NX, TR, -1, PAD, false>(h, rb, t, L.tw);
        if (active)
            for (int b = t; b < s.B; b += TR)
                st_stream(a.band_out + band + band_col_off(b, s.ny), cscale(rb[lds_pos<PAD>(L.bcol[b])], a.scale));
        double acc[3] = {dd, wd, wm};
        block_sum_store<3>(acc, a.part + slot * 3);
    } else {  // ROW_UPDATE
        row_fft<NX, TR, +1, PAD, true>(h, rb, t, L.tw);
        if constexpr (!PREFETCH) load_streams();
        const float gamma = (float)a.diag[(size_t)look * kDiag];
        float wm1 = 0.f;
        uint32_t fb = 0u;
        if (active) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) {
                    const float2 ahr = cscale(h[k], a.scale);
                    const float r0 = rp[k];
                    const float v = wv[k];
                    const float om = 1.f / (r0 + a.floor_w);
                    const float2 d = make_float2(ahr.x * a.inv_s2w - om * m[k].x, ahr.y * a.inv_s2w - om * m[k].y);
                    const float2 m1 = make_float2(m[k].x + gamma * d.x, m[k].y + gamma * d.y);
                    st_stream(&a.mu[img + x], m1);
                    const float rn = r_update_voxel<MODE>(a, bv, r0, v, m1, fb);
                    st_stream(&a.r[img + x], rn);
                    wm1 += om * cabs2(m1);
                }
            }
        }
        wave_or_fault(fb, a.fault);
        double acc[1] = {wm1};
        block_sum_store<1>(acc, a.part + slot);
    }
}

// ---------------------------------------------------------------------------
// Update pass with the Mann step of Alg. 1 fused in: the block walks every
// look of rows [rgroup * RPB, rgroup * RPB + RPB).  Per look it does what
// row_item's update does (recompute d, mu += gamma d, the r-update), with the
// prox point v = u_l + 2 rho xbar_old, and writes u_l' = v - 2 rho r_l; across
// looks it keeps, per voxel, sum_j upsilon_j r_j and sum_j (r_j - w_bar)^2,
// where w_bar = sum_j upsilon_j w_j is the average of the Mann state passed
// in (G(w)), which the previous call left in f.wbar.  After the last look it
// adds the prior agent (its w and H(w)) and writes x_bar = sum_j upsilon_j
// (2 r_j - w_j) = 2 sum_j upsilon_j r_j - w_bar, the new average w_bar +
// 2 rho (sum_j upsilon_j r_j - w_bar) and the prior's new w.  Partial sums:
// sum omega |mu'|^2 per (look, block) into a.part, the convergence error's
// (sum_j (r_j - w_bar)^2, N w_bar^2) per block into f.part.
template <int NX>
__host__ __device__ constexpr int mann_lds_floats() {
    return 2 * kBlock * ((NX + row_threads(NX) - 1) / row_threads(NX));
}

// LDS: ups[64] holds the agent weights, keep[mann_lds_floats<NX>()] each
// thread's x_bar and w_bar of the previous call ([k][thread], conflict-free),
// read back at every look instead of held in registers.
template <int NX, int MODE, class A, class F>
__device__ __forceinline__ void row_update_mann(const A& a, const F& f, int rgroup, int nblk,
                                                const RowLds& L, BetaVals bv, float* ups, float* keep) {
    constexpr int TR = row_threads(NX);
    constexpr int RPB = rows_per_block(NX);
    constexpr int PX = (NX + TR - 1) / TR;
    constexpr int PAD = kRowPad;
    constexpr int RS = lds_len<NX, PAD>();
    const auto& s = a.s;
    const int tid = threadIdx.x;
    const int ri = tid / TR, t = tid % TR;
    const int rows = s.nz * s.ny;
    const int row = rgroup * RPB + ri;
    const bool active = row < rows;
    const size_t n = (size_t)rows * NX;
    const int arow = active ? row : 0;
    const size_t pix = (size_t)arow * NX;
    for (int i = tid; i < NX; i += kBlock) {
        L.tw[i] = s.tw_x[i];
        L.bpos[i] = s.band_pos[i];
        const int bc = s.band_cols[i < s.B ? i : 0];
        L.bcol[i] = i < s.B ? bc : 0;
    }
    // the agent weights go to LDS with constant indices: indexing the
    // argument block by the look would make a private copy of it
    if (tid == 0) {
#pragma unroll
        for (int j = 0; j < 64; ++j) ups[j] = f.ups[j];
    }
    float2* rb = L.buf + ri * RS;
    float* xo = keep;                  // xo[k * kBlock + tid]
    float* wb = keep + PX * kBlock;    // wb[k * kBlock + tid]
    float sr[PX], e2[PX];
    {
        // all loads issued before the first is used (samples past the row
        // end and inactive rows read the row's first sample)
        float a0[PX], a1[PX];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            const size_t i = pix + ((NX % TR == 0 || x < NX) ? x : 0);
            a0[k] = ld_stream(f.xbar + i);
            a1[k] = ld_stream(f.wbar + i);
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            xo[k * kBlock + tid] = a0[k];
            wb[k * kBlock + tid] = a1[k];
            sr[k] = e2[k] = 0.f;
        }
    }
    __syncthreads();
    uint32_t fb = 0u;
    for (int l = 0; l < a.looks; ++l) {
        const size_t img = (size_t)l * n + pix;
        const size_t band = ((size_t)l * s.nz + arow / s.ny) * s.ny * s.Bs + band_row_off(arow % s.ny, s.ny);
        float2 h[PX];
        {
            float2 bin[PX];
            int bp[PX];
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                bp[k] = (active && (NX % TR == 0 || x < NX)) ? L.bpos[x] : -1;
                bin[k] = ld_stream(a.band_in + band + (bp[k] >= 0 ? bp[k] : 0));
            }
#pragma unroll
            for (int k = 0; k < PX; ++k) h[k] = bp[k] >= 0 ? bin[k] : make_float2(0.f, 0.f);
        }
        row_fft<NX, TR, +1, PAD, true>(h, rb, t, L.tw);
        float2 m[PX];
        float rp[PX], uv[PX];
        if (active) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) {
                    m[k] = ld_stream(&a.mu[img + x]);
                    rp[k] = ld_stream(&a.r[img + x]);
                    uv[k] = ld_stream(&f.u[img + x]);
                }
            }
        }
        const float gamma = (float)a.diag[(size_t)l * kDiag];
        const float ul = ups[l];
        float wm1 = 0.f;
        if (active) {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int x = t + k * TR;
                if (NX % TR == 0 || x < NX) {
                    const float2 ahr = cscale(h[k], a.scale);
                    const float r0 = rp[k];
                    const float om = 1.f / (r0 + a.floor_w);
                    const float2 d = make_float2(ahr.x * a.inv_s2w - om * m[k].x, ahr.y * a.inv_s2w - om * m[k].y);
                    const float2 m1 = make_float2(m[k].x + gamma * d.x, m[k].y + gamma * d.y);
                    st_stream(&a.mu[img + x], m1);
                    const float v = uv[k] + f.two_rho * xo[k * kBlock + tid];
                    const float rn = r_update_voxel<MODE>(a, bv, r0, v, m1, fb);
                    st_stream(&a.r[img + x], rn);
                    st_stream(&f.u[img + x], v - f.two_rho * rn);
                    sr[k] += ul * rn;
                    const float e = rn - wb[k * kBlock + tid];
                    e2[k] += e * e;
                    wm1 += om * cabs2(m1);
                }
            }
        }
        double acc[1] = {wm1};
        block_sum_store<1>(acc, a.part + (size_t)l * nblk + rgroup);
    }
    const bool prior = f.wprior != nullptr;
    const float up = prior ? ups[a.looks] : 0.f;
    const float N = (float)f.n_agents;
    double num = 0.0, den = 0.0;
    // the prior agent's output and w, every load issued before the first is
    // used (without a prior the loads read x_bar, with weight 0, and nothing
    // of them is stored)
    float rpv[PX], wpv[PX];
    {
        const float* rsrc = prior ? f.rprior : f.xbar;
        const float* wsrc = prior ? f.wprior : f.xbar;
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            const size_t i = pix + ((NX % TR == 0 || x < NX) ? x : 0);
            rpv[k] = rsrc[i];
            wpv[k] = ld_stream(wsrc + i);
        }
    }
    if (active) {
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int x = t + k * TR;
            if (NX % TR == 0 || x < NX) {
                const float wbk = wb[k * kBlock + tid];
                const float e = rpv[k] - wbk;
                const float s_r = prior ? sr[k] + up * rpv[k] : sr[k];
                const float nm = e2[k] + (prior ? e * e : 0.f);
                const float xb = 2.f * s_r - wbk;
                if (prior) st_stream(f.wprior + pix + x, wpv[k] + f.two_rho * (xb - rpv[k]));
                st_stream(f.xbar + pix + x, xb);
                st_stream(f.wbar + pix + x, wbk + f.two_rho * (s_r - wbk));
                num += (double)nm;
                den += (double)N * ((double)wbk * wbk);
            }
        }
    }
    wave_or_fault(fb, a.fault);
    double acc2[2] = {num, den};
    block_sum_store<2>(acc2, f.part + (size_t)rgroup * 2);
}

// ---------------------------------------------------------------------------
// Inverse column pass of one tile from the column-major compact layout: the
// tile's columns are transformed and written as band columns.  `item` =
// zl * tiles + tile, which is also the partial-sum slot of the scene.
template <int NY, class A>
__device__ __forceinline__ void col_inv_item(const A& a, int item, float2* tw, float2* tile,
                                             bool load_tables) {
    constexpr int TC = col_tile_cols(NY);
    constexpr int TPC = kBlock / TC;
    const auto& s = a.s;
    const int tid = threadIdx.x;
    const int tile_i = item % s.tiles;
    const int zl = item / s.tiles;  // look * nz + z
    const int c0 = tile_i * TC;
    // the twiddles (when this block loads them) travel with the first loads,
    // not after the barrier
    constexpr int TWL = (NY + kBlock - 1) / kBlock;
    float2 twv[TWL];
    if (load_tables) {
#pragma unroll
        for (int j = 0; j < TWL; ++j) {
            const int i = tid + j * kBlock;
            twv[j] = s.tw_y[i < NY ? i : 0];
        }
    }
    const float2* src = a.cmp_in + (size_t)zl * s.P;
    const int co = tid % TC, bo = c0 + co;
    float2* dst = a.band_out + (size_t)zl * s.ny * s.Bs + (size_t)tile_i * s.ny * TC + co;  // the tile's block
    double acc[1] = {0.0};
    if constexpr (fft_regs_ok<NY, TPC>()) {
        // Each thread fetches its own transform inputs, rows tid / TC + k TPC
        // of band column bo, straight into registers: the compact index of
        // each from pidxb (-1 off the pupil), then the samples, every load
        // issued before the first is used.  No tile to clear, no scatter
        // through LDS.
        constexpr int PT = NY / TPC;
        const int yo = tid / TC;
        const bool col = bo < s.B;
        int pi[PT];
#pragma unroll
        for (int k = 0; k < PT; ++k) pi[k] = col ? s.pidxb[(size_t)(yo + k * TPC) * s.Bs + bo] : -1;
        float2 h[PT];
#pragma unroll
        for (int k = 0; k < PT; ++k) h[k] = src[pi[k] >= 0 ? pi[k] : 0];
        float f = 0.f;
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            if (pi[k] < 0) h[k] = make_float2(0.f, 0.f);
            f += cabs2(h[k]);
        }
        acc[0] = f;
        __syncthreads();  // the previous item's readers of the LDS buffers are done
        if (load_tables) {
#pragma unroll
            for (int j = 0; j < TWL; ++j) {
                const int i = tid + j * kBlock;
                if (i < NY) tw[i] = twv[j];
            }
        }
        // the transform opens with a block barrier (the twiddles are then in
        // place); its last stage leaves each thread rows yo + k TPC, which it
        // stores into the tile's block
        fft_regs<NY, TPC, +1, 0, true, true, false>(h, tile + co, TC, yo, tw);
        if (col) {
#pragma unroll
            for (int k = 0; k < PT; ++k) st_stream(dst + (size_t)(yo + k * TPC) * TC, cscale(h[k], a.scale));
        }
    } else {
        // Scatter of column bc's pupil samples p in [p0, p1): lane l takes
        // p0 + l, p0 + l + TPC, ..., all loads issued before the first is
        // used (positions past p1 re-read the column's last sample and are
        // dropped); a column holds at most NY = CH * TPC samples, so one
        // chunk, loaded before the tile is cleared, covers it.
        constexpr int CH = NY / TPC;
        const int c = tid / TPC, lane = tid % TPC, bc = c0 + c;
        int p0 = 0, p1 = 0;
        if (bc < s.B) {
            p0 = s.col_off[bc];
            p1 = s.col_off[bc + 1];
        }
        float2 v[CH];
        int ry[CH];
        const int base = p0 + lane;
        if (base < p1) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int p = base + k * TPC;
                const int pc = p < p1 ? p : p1 - 1;
                v[k] = src[pc];
                ry[k] = s.row_idx[pc];
            }
        }
        __syncthreads();  // the previous item's readers of the LDS buffers are done
        if (load_tables) {
#pragma unroll
            for (int j = 0; j < TWL; ++j) {
                const int i = tid + j * kBlock;
                if (i < NY) tw[i] = twv[j];
            }
        }
        for (int i = tid; i < NY * TC; i += kBlock) tile[i] = make_float2(0.f, 0.f);
        __syncthreads();
        float f = 0.f;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (base + k * TPC < p1) {
                tile[ry[k] * TC + c] = v[k];
                f += cabs2(v[k]);
            }
        }
        acc[0] = f;
        fft_lds<NY, TPC, +1>(tile + co, TC, tid / TC, tw);
        if (bo < s.B)
            for (int y = tid / TC; y < NY; y += TPC) st_stream(dst + (size_t)y * TC, cscale(tile[y * TC + co], a.scale));
    }
    if (a.part != nullptr) block_sum_store<1>(acc, a.part + item);
}

// Forward column pass over a stream of items (all of column length NY): the
// block walks items first, first + stride, ..., keeping the next item's band
// rows in registers, loaded while the current item's column FFTs run.
// `item_of(i)` returns the (ColArgs, scene item index) of stream position i.
// The twiddle table must already be in `tw` (it depends on NY only).
template <int NY, class ItemOf>
__device__ __forceinline__ void col_fwd_stream(int first, int count, int stride, ItemOf item_of, const float2* tw,
                                               float2* tile) {
    constexpr int TC = col_tile_cols(NY);
    constexpr int TPC = kBlock / TC;
    constexpr int PT = NY / TPC;
    static_assert(NY % TPC == 0, "column length must be a multiple of the threads per column");
    const int tid = threadIdx.x;
    const int c_ld = tid % TC, y_ld = tid / TC;
    float2 pre[PT];
    auto load = [&](int pos) {
        const auto ai = item_of(pos);
        const auto& a = ai.get();
        const auto& s = a.s;
        const int bc = (ai.item % s.tiles) * TC + c_ld;
        // the tile's contiguous block of the band buffer
        const float2* src = a.band_in + (size_t)(ai.item / s.tiles) * s.ny * s.Bs +
                            (size_t)(ai.item % s.tiles) * s.ny * TC + c_ld;
#pragma unroll
        for (int k = 0; k < PT; ++k)
            pre[k] = bc < s.B ? src[(size_t)(y_ld + k * TPC) * TC] : make_float2(0.f, 0.f);
    };
    int pos = first;
    if (pos < count) load(pos);
    for (; pos < count; pos += stride) {
        const auto ai = item_of(pos);
        const auto& a = ai.get();
        const auto& s = a.s;
        const int tile_i = ai.item % s.tiles;
        const int zl = ai.item / s.tiles;
        // the item's band rows move to h (rows y_ld + k TPC of column c_ld),
        // and pre is free for the next item's prefetch
        float2 h[PT];
#pragma unroll
        for (int k = 0; k < PT; ++k) h[k] = pre[k];
        // Rows of column bc's pupil samples p0 + lane + k TPC (at most NY =
        // PT * TPC of them), loaded before the next item's prefetch so that
        // waiting for them does not wait for it; positions past p1 re-read
        // the column's last row and are not stored.
        const int c = tid / TPC, lane = tid % TPC, bc = tile_i * TC + c;
        int p0 = 0, p1 = 0;
        int ry[PT];
        if (bc < s.B) {
            p0 = s.col_off[bc];
            p1 = s.col_off[bc + 1];
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const int p = p0 + lane + k * TPC;
                ry[k] = s.row_idx[p < p1 ? p : p1 - 1];
            }
        }
        if (pos + stride < count) load(pos + stride);
        // the transform's opening block barrier also orders it after the
        // previous item's readers of `tile`
        if constexpr (fft_regs_ok<NY, TPC>()) {
            fft_regs<NY, TPC, -1, 0, true, false, false>(h, tile + c_ld, TC, y_ld, tw);
        } else {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PT; ++k) tile[(y_ld + k * TPC) * TC + c_ld] = h[k];
            fft_lds<NY, TPC, -1>(tile + c_ld, TC, y_ld, tw);
        }
        double acc[1] = {0.0};
        if (bc < s.B) {
            float2* dst = a.cmp_out + (size_t)zl * s.P;
            float f = 0.f;
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const int p = p0 + lane + k * TPC;
                if (p < p1) {
                    const float2 val = cscale(tile[ry[k] * TC + c], a.scale);
                    dst[p] = val;
                    f += cabs2(val);
                }
            }
            acc[0] = f;
        }
        if (a.part != nullptr) block_sum_store<1>(acc, a.part + ai.item);
    }
}

// Column-pass item handles for col_fwd_stream: by pointer (kernel
// arguments) or by private copy (arguments read from device memory).
struct ColItemRef {
    const ColArgs* args;
    int item;
    __device__ const ColArgs& get() const { return *args; }
};
struct ColItemVal {
    ColArgs args;
    int item;
    __device__ const ColArgs& get() const { return args; }
};
struct ColItemConst {
    ConstAS<ColArgs>* args;
    int item;
    __device__ ConstAS<ColArgs>& get() const { return *args; }
};

// ---------------------------------------------------------------------------
// Exact step size of one look from the partial sums of the three passes, and
// h before the mu-step: h = ||resid||^2 / (2 sigma_w^2) + sum omega |mu|^2 / 2,
// which is eq. mu-objective less the constant ||(1 - a) y||^2 / (2 sigma_w^2)
// of the samples off the pupil.  Look 0 also zeroes the counter of looks the
// diagnostics pass has finished.
__device__ __forceinline__ void gamma_item(int look, const GammaArgs& a) {
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    strided_sums<3>(a.prow + (size_t)look * a.nrow * 3, a.nrow, 3, v);
    strided_sums<1>(a.pcf + (size_t)look * a.ncol, a.ncol, 1, v + 3);
    strided_sums<1>(a.pci + (size_t)look * a.ncol, a.ncol, 1, v + 4);
    __shared__ double tot[5];
    block_sum_store<5>(v, tot);
    if (threadIdx.x == 0) {
        const double dd = tot[0], wd = tot[1], wm = tot[2], ad = tot[3], r2 = tot[4];
        const double den = ad * a.inv_s2w + wd;
        const double g = dd > 0.0 ? dd / den : 0.0;
        double* o = a.diag + (size_t)look * kDiag;
        o[DG_GAMMA] = g;
        o[DG_DD] = dd;
        o[DG_AD] = ad;
        o[DG_H0] = 0.5 * (r2 * a.inv_s2w + wm);
        o[DG_WD] = wd;
        if (!(g >= 0.0) || !isfinite(g)) atomicOr(a.fault, 4u | 1u);
        if (look == 0) *a.counter = 0u;
    }
}

// resid -= gamma D(a) F d over entries [begin, end) of one look; returns the
// thread's share of ||resid||^2.
__device__ __forceinline__ float resid_range(float2* R, const float2* D, float g, size_t begin, size_t end,
                                             size_t stride) {
    float f = 0.f;
    for (size_t i = begin + threadIdx.x; i < end; i += stride) {
        float2 x = ld_stream(R + i);
        const float2 d = ld_stream(D + i);
        x.x -= g * d.x;
        x.y -= g * d.y;
        st_stream(R + i, x);
        f += cabs2(x);
    }
    return f;
}

// Diagnostics after the mu-step of one look: h after (the same omega as h
// before, so h before - h after = gamma ||d||^2 / 2 up to rounding), the
// look's mu-residual of eq. residual in its noise-floored form, ||d|| /
// ||A^H y / sigma_w^2|| with d the gradient the step used (0 without
// ||A^H y||^2), and ||resid||^2.  The block that finishes the last look of the
// call writes the summary row diag[looks]: the mu-residual averaged over looks
// (eq. residual), and the sums of h before and after, in look order.
__device__ __forceinline__ void diag_after_item(int look, const DiagArgs& a) {
    double v[2] = {0.0, 0.0};
    strided_sums<1>(a.pupd + (size_t)look * a.nrow, a.nrow, 1, v);
    strided_sums<1>(a.pres + (size_t)look * a.nres, a.nres, 1, v + 1);
    __shared__ double tot[2];
    block_sum_store<2>(v, tot);
    __shared__ int last;
    if (threadIdx.x == 0) {
        double* o = a.diag + (size_t)look * kDiag;
        o[DG_H1] = 0.5 * (tot[1] / a.s2w + tot[0]);
        o[DG_R2] = tot[1];
        double m2 = 0.0;
        if (a.ahy2 != nullptr) {
            const double y2 = a.ahy2[look];
            m2 = y2 > 0.0 ? a.s2w * sqrt(o[DG_DD] / y2) : 0.0;
        }
        o[DG_MURES] = m2;
        __threadfence();  // this look's row is visible before it is counted
        last = atomicAdd(a.counter, 1u) == (unsigned)(a.looks - 1);
    }
    __syncthreads();
    if (last) {
        // every look's row is written: one thread per look reads its row, and
        // thread 0 sums them in look order
        __shared__ double rows[3][kBlock];
        __threadfence();
        const volatile double* d = a.diag;
        for (int l0 = 0; l0 < a.looks; l0 += kBlock) {
            const int l = l0 + (int)threadIdx.x;
            if (l < a.looks) {
                rows[0][threadIdx.x] = d[(size_t)l * kDiag + DG_MURES];
                rows[1][threadIdx.x] = d[(size_t)l * kDiag + DG_H0];
                rows[2][threadIdx.x] = d[(size_t)l * kDiag + DG_H1];
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double m = l0 == 0 ? 0.0 : a.diag[(size_t)a.looks * kDiag + 0];
                double h0 = l0 == 0 ? 0.0 : a.diag[(size_t)a.looks * kDiag + 1];
                double h1 = l0 == 0 ? 0.0 : a.diag[(size_t)a.looks * kDiag + 2];
                const int cnt = a.looks - l0 < kBlock ? a.looks - l0 : kBlock;
                for (int i = 0; i < cnt; ++i) {
                    m += rows[0][i];
                    h0 += rows[1][i];
                    h1 += rows[2][i];
                }
                double* srow = a.diag + (size_t)a.looks * kDiag;
                srow[0] = m;
                srow[1] = h0;
                srow[2] = h1;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double* srow = a.diag + (size_t)a.looks * kDiag;
            srow[0] /= a.looks;
            for (int k = 3; k < kDiag; ++k) srow[k] = 0.0;
        }
    }
}

// Mann step of voxel i with every agent's w and r in registers (NA >=
// n_agents); returns (sum_j (r_j - w_bar)^2, n_agents w_bar^2).  The loads
// are unconditional so that all of them are in flight at once: padding agents
// re-read the last agent and carry weight 0 (ups[j] = 0 for j >= n_agents).
template <int NA>
__device__ __forceinline__ void mace_voxel(const MaceArgs& a, const float* ups, unsigned n, unsigned i, double& num,
                                           double& den) {
    float wv[NA], rv[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        const size_t base = (size_t)(j < a.n_agents ? j : a.n_agents - 1) * n;
        wv[j] = ld_stream(a.w + base + i);
        rv[j] = ld_stream(a.r + base + i);
    }
    float wb = 0.f, rb = 0.f;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        wb += ups[j] * wv[j];
        rb += ups[j] * rv[j];
    }
    const float xb = 2.f * rb - wb;
    float wbn = 0.f, nm = 0.f;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        if (j < a.n_agents) {
            const float dr = rv[j] - wb;
            nm += dr * dr;
            const float wn = wv[j] + a.two_rho * (xb - rv[j]);
            st_stream(a.w + (size_t)j * n + i, wn);
            wbn += ups[j] * wn;
        }
    }
    st_stream(a.wbar + i, wbn);
    num += nm;
    den += (double)a.n_agents * wb * wb;
}

// Periodic 7-tap Gaussian smoothing along z, y and x in one pass over the
// volume: one call produces an output tile of kGaussTY rows x TX voxels over
// range slices z0 .. z0 + kGaussCZ - 1.  Tiles are numbered z chunk fastest,
// then x, then y: tile t has bz = t % zc, bx = (t / zc) % (nx / TX),
// by = t / (zc nx / TX), so that consecutive tiles share their halos.  Every
// (kGaussTY + 6) x (TX + 6) window of the input slices z0 - 3 .. z0 +
// kGaussCZ + 2 is loaded into registers up front, so that the block waits
// for memory once, not once per slice, and is filtered along z there, each
// thread over its own window positions.  Then, output slice by output slice,
// the z-filtered window goes to LDS and is filtered along x, then along y
// (the separable filter's three passes commute).  p holds
// nx, ny, nz (ny a multiple of kGaussTY, nx of TX), the taps g[7], in and
// out (not overlapping).
template <int TX>
__host__ __device__ constexpr int gauss_in_floats() { return (kGaussTY + 6) * (TX + 6); }
template <int TX>
__host__ __device__ constexpr int gauss_xf_floats() { return (kGaussTY + 6) * TX; }

template <int TX, class P>
__device__ __forceinline__ void gauss3d_tile(const P& p, int tile, float* tin, float* txf) {
    constexpr int W = TX + 6, H = kGaussTY + 6;
    constexpr int NIN = H * W;
    constexpr int LPT = (NIN + kBlock - 1) / kBlock;
    constexpr int OPT = kGaussTY * TX / kBlock;
    constexpr int NZW = kGaussCZ + 6;  // input slices of a chunk
    static_assert(OPT >= 1 && kGaussTY * TX % kBlock == 0, "a tile's outputs divide among the threads");
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const float* in = p.in;
    float* out = p.out;
    float g[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) g[k] = p.g[k];
    const int tid = threadIdx.x;
    const int zc = (nz + kGaussCZ - 1) / kGaussCZ, tx = nx / TX;
    const int bz = tile % zc, bx = (tile / zc) % tx, by = tile / (zc * tx);
    const int x0 = bx * TX, y0 = by * kGaussTY, z0 = bz * kGaussCZ;
    const int zend = z0 + kGaussCZ < nz ? z0 + kGaussCZ : nz;
    const unsigned slice = (unsigned)nx * (unsigned)ny;
    unsigned goff[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int e = tid + j * kBlock;
        const int r = (e < NIN ? e : 0) / W, c = (e < NIN ? e : 0) % W;
        int gy = y0 - 3 + r, gx = x0 - 3 + c;
        gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        goff[j] = (unsigned)gy * nx + gx;
    }
    // the chunk's input windows, all loads issued before the first is used
    // (in a chunk cut short by the end of the volume the slices past it wrap
    // periodically and are filtered, but no output of theirs is stored)
    float pre[NZW][LPT];
#pragma unroll
    for (int sl = 0; sl < NZW; ++sl) {
        int zz = (z0 - 3 + sl) % nz;
        zz = zz < 0 ? zz + nz : zz;
        const float* src = in + (size_t)zz * slice;
#pragma unroll
        for (int j = 0; j < LPT; ++j) pre[sl][j] = src[goff[j]];
    }
    // Two barriers per output slice: the previous slice's second barrier has
    // every reader of tin behind it before tin is rewritten, and this
    // slice's first one every reader of txf before txf is rewritten.
#pragma unroll
    for (int o = 0; o < kGaussCZ; ++o) {
        if (z0 + o >= zend) break;  // uniform over the block
        // the window of output slice z0 + o filtered along z, in registers
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int e = tid + j * kBlock;
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 7; ++k) acc += g[k] * pre[o + k][j];
            if (e < NIN) tin[e] = acc;
        }
        __syncthreads();
        for (int e = tid; e < H * TX; e += kBlock) {
            const int r = e / TX, c = e % TX;
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 7; ++k) acc += g[k] * tin[r * W + c + k];
            txf[e] = acc;
        }
        __syncthreads();
        const size_t zo = (size_t)(z0 + o) * slice;
#pragma unroll
        for (int q = 0; q < OPT; ++q) {
            const int oq = tid + q * kBlock;
            const int oy = oq / TX, ox = oq % TX;
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 7; ++k) acc += g[k] * txf[(oy + k) * TX + ox];
            out[zo + (size_t)(y0 + oy) * nx + x0 + ox] = acc;
        }
    }
}

}  // namespace clampk
