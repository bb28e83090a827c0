// Complex FFT building blocks for gfx950: Stockham autosort stages with
// radix 2, 3, 4 and 8 butterflies, run in place on an LDS vector that a
// group of threads shares.  Each stage reads its butterfly inputs into
// registers, waits for the group, applies twiddles and the butterfly, and
// writes the outputs to their autosorted positions, so the result is in
// natural order with no bit reversal.
//
// Twiddles come from a table tw[m] = exp(-2 pi i m / N), m < N, computed in
// float64 on the host and rounded to float32; the inverse direction uses its
// conjugate.  Transforms are unnormalised; callers apply the orthonormal
// scale.
#pragma once

#include <hip/hip_runtime.h>

namespace clampk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// a * (S i), S = +1 or -1
template <int S>
__device__ __forceinline__ float2 mul_si(float2 a) {
    return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// In-register DFTs X_k = sum_j v_j exp(S 2 pi i j k / R).
template <int R, int S> struct Bfly;

template <int S> struct Bfly<2, S> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int S> struct Bfly<3, S> {
    __device__ __forceinline__ static void run(float2* v) {
        const float h = 0.86602540378443864676f;  // sqrt(3)/2
        float2 t = cadd(v[1], v[2]);
        float2 u = cscale(mul_si<S>(csub(v[1], v[2])), h);
        float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, u);
        v[2] = csub(m, u);
    }
};

template <int S> struct Bfly<4, S> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        float2 a2 = cadd(v[1], v[3]), a3 = mul_si<S>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    }
};

template <int S> struct Bfly<8, S> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Bfly<4, S>::run(e);
        Bfly<4, S>::run(o);
        const float h = 0.70710678118654752440f;
        // W = exp(S 2 pi i / 8): W^1 = (1 + S i) h, W^2 = S i, W^3 = (-1 + S i) h
        float2 o1 = make_float2((o[1].x - S * o[1].y) * h, (o[1].y + S * o[1].x) * h);
        float2 o2 = mul_si<S>(o[2]);
        float2 o3 = make_float2((-o[3].x - S * o[3].y) * h, (-o[3].y + S * o[3].x) * h);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

// Radix plan: as many radix-8 stages as possible, then 4, 2 and 3.
__host__ __device__ constexpr int next_radix(int n) {
    return (n % 8 == 0) ? 8 : (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : 3;
}
__host__ __device__ constexpr int radix_at(int n, int s) {
    for (int i = 0; i < s; ++i) n /= next_radix(n);
    return next_radix(n);
}
__host__ __device__ constexpr int num_stages(int n) {
    int c = 0;
    while (n > 1) {
        n /= next_radix(n);
        ++c;
    }
    return c;
}
__host__ __device__ constexpr bool fft_len_ok(int n) {
    if (n < 2) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Position of element i of a padded LDS vector: one float2 of padding after
// every 16 elements (PADSH = 4) spreads the radix-R autosort stores over the
// LDS banks; PADSH = 0 means no padding.  (An XOR swizzle of bits 3..7 into
// bits 0..4, free of bank conflicts in every stage under a 64-bank model,
// measured no faster in the row passes and cost the gradient pass a wave.)
template <int PADSH>
__host__ __device__ constexpr int lds_pos(int i) {
    if constexpr (PADSH > 0) return i + (i >> PADSH);
    else return i;
}
template <int N, int PADSH>
__host__ __device__ constexpr int lds_len() {
    return lds_pos<PADSH>(N - 1) + 1;
}

// Synchronisation of the threads that share one transform: the block
// (__syncthreads), or, when each group lies inside one wave (WAVE), the wave
// alone.  A wave's LDS operations execute in issue order, so the wave-local
// form only has to keep the compiler from moving LDS accesses across it.
template <bool WAVE>
__device__ __forceinline__ void group_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One Stockham stage and the ones after it.  buf[lds_pos(i) * stride] is
// element i of this group's vector; t in [0, T) is the thread's rank in the
// group.  Every thread of the block (of the wave, for WAVE) must call this.
template <int N, int T, int S, int PADSH, int STAGE, int NS, bool WAVE>
__device__ __forceinline__ void fft_stages(float2* buf, int stride, int t, const float2* tw) {
    if constexpr (STAGE < num_stages(N)) {
        constexpr int R = radix_at(N, STAGE);
        constexpr int NB = N / R;
        constexpr int PER = (NB + T - 1) / T;
        constexpr int TWSTEP = N / (NS * R);
        float2 v[PER][R];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int j = t + p * T;
            if ((NB % T == 0) || j < NB) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[p][r] = buf[lds_pos<PADSH>(j + r * NB) * stride];
            }
        }
        group_sync<WAVE>();
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int j = t + p * T;
            if ((NB % T == 0) || j < NB) {
                const int k = j % NS;
                if constexpr (NS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        float2 w = tw[r * k * TWSTEP];
                        if constexpr (S > 0) w.y = -w.y;
                        v[p][r] = cmul(v[p][r], w);
                    }
                }
                Bfly<R, S>::run(v[p]);
                const int base = (j / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) buf[lds_pos<PADSH>(base + r * NS) * stride] = v[p][r];
            }
        }
        group_sync<WAVE>();
        fft_stages<N, T, S, PADSH, STAGE + 1, NS * R, WAVE>(buf, stride, t, tw);
    }
}

// Unnormalised length-N DFT of buf (S = -1 forward, +1 inverse), in place.
// Starts with a group synchronisation, so writes made to buf before the call
// are visible, and ends with one, so the result is visible to the group (the
// block, or with WAVE the wave, which must then hold every thread of the
// group: T divides 64 and groups start at multiples of T).
template <int N, int T, int S, int PADSH = 0, bool WAVE = false>
__device__ __forceinline__ void fft_lds(float2* buf, int stride, int t, const float2* tw) {
    static_assert(fft_len_ok(N), "FFT length must be 2^a 3^b");
    static_assert(!WAVE || (T <= 64 && 64 % T == 0), "a wave-local transform must lie inside one wave");
    group_sync<WAVE>();
    fft_stages<N, T, S, PADSH, 0, 1, WAVE>(buf, stride, t, tw);
}

// Transforms with the data in registers: the T threads of a group hold h[k] =
// element t + k T.  This applies when every stage's N / R butterflies divide
// evenly among the T threads: the first stage can then take its inputs
// j + r N / R0 (j = t + p T) from h[p + r N / (R0 T)], and the last stage can
// write its outputs j + r N / RL to h[p + r N / (RL T)], each on the thread
// that holds it.  The stages between go through buf as in fft_lds; the group
// synchronises as a block, or (WAVE) as a wave when it lies inside one.
template <int N, int T>
__host__ __device__ constexpr bool fft_regs_ok() {
    for (int st = 0; st < num_stages(N); ++st)
        if ((N / radix_at(N, st)) % T != 0) return false;
    return true;
}

template <int N, int T, int S, int PADSH, int STAGE, int NS, bool IN_REGS, bool OUT_REGS, bool WAVE>
__device__ __forceinline__ void fft_regs_stages(float2 (&h)[N / T], float2* buf, int stride, int t,
                                                const float2* tw) {
    constexpr int NST = num_stages(N);
    if constexpr (STAGE < NST) {
        constexpr int R = radix_at(N, STAGE);
        constexpr int NB = N / R;
        constexpr int PER = NB / T;
        constexpr int TWSTEP = N / (NS * R);
        constexpr bool FIRST_FROM_REGS = IN_REGS && STAGE == 0;
        constexpr bool LAST_IN_REGS = OUT_REGS && STAGE == NST - 1;
        float2 v[PER][R];
        if constexpr (FIRST_FROM_REGS) {
#pragma unroll
            for (int p = 0; p < PER; ++p)
#pragma unroll
                for (int r = 0; r < R; ++r) v[p][r] = h[p + r * PER];
        } else {
#pragma unroll
            for (int p = 0; p < PER; ++p)
#pragma unroll
                for (int r = 0; r < R; ++r) v[p][r] = buf[lds_pos<PADSH>(t + p * T + r * NB) * stride];
            group_sync<WAVE>();
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int j = t + p * T;
            const int k = j % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[r * k * TWSTEP];
                    if constexpr (S > 0) w.y = -w.y;
                    v[p][r] = cmul(v[p][r], w);
                }
            }
            Bfly<R, S>::run(v[p]);
            if constexpr (LAST_IN_REGS) {
                // outputs j + r NS (NS = N / R in the last stage) = element t + (p + r NS / T) T
#pragma unroll
                for (int r = 0; r < R; ++r) h[p + r * (NS / T)] = v[p][r];
            } else {
                const int base = (j / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) buf[lds_pos<PADSH>(base + r * NS) * stride] = v[p][r];
            }
        }
        if constexpr (!LAST_IN_REGS) group_sync<WAVE>();
        fft_regs_stages<N, T, S, PADSH, STAGE + 1, NS * R, IN_REGS, OUT_REGS, WAVE>(h, buf, stride, t, tw);
    }
}

// Unnormalised length-N DFT (see fft_regs_ok) of the group's vector, held in
// h (IN_REGS) or in buf[lds_pos(i) * stride]; the result goes to h (OUT_REGS)
// or to buf in natural order, visible to the group.  Starts with a group
// synchronisation, so earlier reads and writes of buf by the group are done.
template <int N, int T, int S, int PADSH, bool IN_REGS, bool OUT_REGS, bool WAVE>
__device__ __forceinline__ void fft_regs(float2 (&h)[N / T], float2* buf, int stride, int t, const float2* tw) {
    static_assert(fft_len_ok(N) && fft_regs_ok<N, T>(), "length and group size outside the register form");
    static_assert(!WAVE || (T <= 64 && 64 % T == 0), "a wave-local transform must lie inside one wave");
    group_sync<WAVE>();
    fft_regs_stages<N, T, S, PADSH, 0, 1, IN_REGS, OUT_REGS, WAVE>(h, buf, stride, t, tw);
}

}  // namespace clampk
