// Learned prior agent: a residual 3D CNN denoiser with BF16 MFMA kernels.
//
// Network: 8 convolutions of 3x3x3 taps with biases and zero padding,
// channels 1 -> 32 -> ... -> 32 -> 1, ReLU after the first seven, output
// H(x) = x + N(x).  Applied to a volume w of any scale it runs on w / m with
// m = mean(w) and returns w + m N(w / m).
//
// Storage: activations and gradients are channels-last bfloat16, [voxel][C]
// with C = 8 for one-channel tensors (channel 0 used) and 32 otherwise;
// weights are fp32 masters with bf16 copies laid out per MFMA fragment.
// Every convolution with 32 output channels (forward, backward data, weight
// gradient) is an implicit GEMM on gfx950's 32x32x16 bf16 MFMA with fp32
// accumulation; the one-channel output layer of the forward pass uses bf16
// dot products on the vector ALUs instead.  The kernels below describe their
// tilings.  Lane layout (64 lanes, l = lane): A[m][k] in
// lane m + 32 (k / 8), element k % 8; B[k][n] in lane n + 32 (k / 8), element
// k % 8; D[m][n] in lane n + 32 ((m / 4) % 2), register (m / 8) 4 + m % 4.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cnn.h"

namespace clampk {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// Word 3 of a raw buffer resource (32-bit data, no format conversion) and a
// byte offset that lies outside every buffer the kernels address (at most
// one output slice, < 2^31 bytes): stores there are dropped, loads read 0.
constexpr int kBufferWord3 = 0x00020000;
constexpr uint32_t kBufferOutside = 0x80000000u;
// Cache policy of the input-slice loads: non-temporal (the slices stream
// through once per layer; measured faster for both the forward layers and
// training).  Output stores stay cached: the next layer reads them.
constexpr int kNonTemporal = 2;

constexpr int kCnnBlock = 256;

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

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

// Row index of the MFMA output register i of lane l (the column is l % 32).
__device__ __forceinline__ int d_row(int l, int i) { return (l / 32) * 4 + (i / 4) * 8 + (i % 4); }

// ---------------------------------------------------------------------------
// Convolution (forward or backward-data), tiled implicit GEMM on the
// 32x32x16 bf16 MFMA.
//
// A block of 16 / RPW waves (RPW output rows per wave: 4, or 2 for the
// forward layers) owns an output tile of 16 rows x 32 x-voxels and walks a
// chunk of range slices.  Input slices (tile plus a one-voxel halo: 18 rows x
// 34 voxels, zero outside the volume) live in two LDS slots: output slice z
// takes its dz = -1 and dz = 0 taps from the slots holding input z - 1 and z,
// then input z + 1 (fetched into registers during the previous step) replaces
// input z - 1 and the dz = +1 taps follow, while input z + 2 is fetched.
// Every weight fragment of the layer stays in LDS for the whole block, so the
// MFMA loop reads only LDS.  Wave w computes rows RPW w .. RPW w + RPW - 1;
// for each (dz, dy) tap pair and K fragment q it reads the RPW + 2 input rows
// its output rows need once and applies each to up to three output rows (the
// dy taps).  K
// fragments: for 32 input channels q = (dx, channel half), 6 per (dz, dy); for
// 8 input channels q pairs two dx taps (q = 0: dx = -1 in k 0..7 and dx = 0 in
// k 8..15; q = 1: dx = +1 and zeros).  The product is formed transposed,
// D[channel][voxel] = W^T X^T (weights as the A operand, inputs as B), so that
// each lane ends with 16 output channels of one voxel in runs of four
// consecutive channels; after bias and ReLU a swap between the lane halves
// makes 16-byte runs of eight channels, stored straight to the channels-last
// output.
//
// LDS layouts.  Input slot: 16-byte chunks; for 32 channels the chunk j of
// voxel (row ys, column xs) sits at (ys * 34 + xs) * 4 + (j ^ ((xs >> 2) & 3)),
// so that the 16 lanes of one 128-bit LDS access phase (16 consecutive voxels,
// one chunk each) hit 16 distinct 16-byte bank groups of the 256-byte bank
// window.  Weights: wq[g = 3 dz + dy][q][h][n][8] (see prep_q_elem), 16 lanes of
// one phase reading 16 consecutive fragments rows.
constexpr int kTileRows = 16;
constexpr int kTileCols = 32;
constexpr int kRingRows = kTileRows + 2;
constexpr int kRingCols = kTileCols + 2;

// NT: threads of the block that fills the slots.
template <int CIN, int NT = kCnnBlock>
struct TileGeo {
    static constexpr int kChunks = CIN / 8;                              // 16-byte chunks per voxel
    static constexpr int kSlice = kRingRows * kRingCols * kChunks;      // chunks per input slot
    static constexpr int kQ = CIN == 32 ? 6 : 2;                         // K fragments per (dz, dy)
    static constexpr int kW = 9 * kQ * 64;                               // weight chunks (16 bytes)
    static constexpr int kFill = (kSlice + NT - 1) / NT;                 // chunks per thread per slice
    static constexpr int kSlot = kFill * NT;                             // slot size, padded for branch-free stores
};

template <int CIN>
__device__ __forceinline__ int ring_pos(int ys, int xs, int j) {
    if constexpr (CIN == 32) return (ys * kRingCols + xs) * 4 + (j ^ ((xs >> 2) & 3));
    else return ys * kRingCols + xs;
}

// Loads of input slice zin of the block's tile (with halo) into registers,
// branch-free: buffer loads relative to the slice, whose size is 0 when the
// slice lies outside the volume or is not wanted (live = false), and an
// offset outside it for halo voxels outside the volume -- those read 0.
template <int CIN, int NT = kCnnBlock>
__device__ __forceinline__ void tile_fetch(const ConvArgs& a, const uint16_t* in, int zin, int y0, int x0,
                                           uint4 (&pre)[TileGeo<CIN, NT>::kFill], bool live = true) {
    using G = TileGeo<CIN, NT>;
    const bool zok = live && zin >= 0 && zin < a.nz;
    const long plane = (long)a.ny * a.nx;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(in) + (zok ? zin : 0) * plane * CIN, 0, zok ? (uint32_t)(plane * CIN * 2) : 0u,
        kBufferWord3);
#pragma unroll
    for (int i = 0; i < G::kFill; ++i) {
        const int e = threadIdx.x + i * NT;
        const int j = e % G::kChunks, vox = e / G::kChunks;
        const int xs = vox % kRingCols, ys = vox / kRingCols;
        const int y = y0 - 1 + ys, x = x0 - 1 + xs;
        const bool ok = e < G::kSlice && y >= 0 && y < a.ny && x >= 0 && x < a.nx;
        const uint32_t off = ok ? (uint32_t)(((y * a.nx + x) * CIN + j * 8) * 2) : kBufferOutside;
        const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kNonTemporal);
        pre[i] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// Store of a fetched slice into an LDS slot of kSlot chunks.  The chunks past
// the slice (e >= kSlice) are stored unguarded into the padding -- ring_pos
// maps them to e itself, up to a permutation of its four chunks -- which
// keeps the store free of branches.
template <int CIN, int NT = kCnnBlock>
__device__ __forceinline__ void tile_store(uint4* slot, const uint4 (&pre)[TileGeo<CIN, NT>::kFill]) {
    using G = TileGeo<CIN, NT>;
#pragma unroll
    for (int i = 0; i < G::kFill; ++i) {
        const int e = threadIdx.x + i * NT;
        const int j = e % G::kChunks, vox = e / G::kChunks;
        slot[ring_pos<CIN>(vox / kRingCols, vox % kRingCols, j)] = pre[i];
    }
}

template <int CIN, int NT = kCnnBlock>
using RingSlots = uint4[2][TileGeo<CIN, NT>::kSlot];

// Persistent work split of the convolutions: output tile-slices, numbered
// t = ((vol tiles_y + yt) tiles_x + xt) nz + z (z fastest), go to blocks in
// contiguous runs of a.span, and a block walks its run in range order,
// starting a new segment (with its two-slice halo prologue) only where the
// run crosses into the next tile.
struct ConvSeg {
    int xt, yt, vol, z0, z1;
};

__device__ __forceinline__ bool next_seg(const ConvArgs& a, long& t, long tend, ConvSeg& g) {
    if (t >= tend) return false;
    const long col = t / a.nz;
    g.z0 = (int)(t - col * a.nz);
    const long rem = tend - t;
    g.z1 = rem < a.nz - g.z0 ? g.z0 + (int)rem : a.nz;
    g.xt = (int)(col % a.tiles_x);
    g.yt = (int)((col / a.tiles_x) % a.tiles_y);
    g.vol = (int)(col / ((long)a.tiles_x * a.tiles_y));
    t += g.z1 - g.z0;
    return true;
}

// Segment prologue: inputs z0 - 1 and z0 into the two slots (fetched
// together), input z0 + 1 into registers.  The leading barrier keeps the
// previous segment's readers away from the slots.
template <int CIN, int NT>
__device__ __forceinline__ void seg_prologue(const ConvArgs& a, const uint16_t* in, int z0, int y0, int x0,
                                             RingSlots<CIN, NT>& ring, uint4 (&pre)[TileGeo<CIN, NT>::kFill]) {
    uint4 pre0[TileGeo<CIN, NT>::kFill];
    tile_fetch<CIN, NT>(a, in, z0 - 1, y0, x0, pre0);
    tile_fetch<CIN, NT>(a, in, z0, y0, x0, pre);
    __syncthreads();
    tile_store<CIN, NT>(ring[0], pre0);
    tile_store<CIN, NT>(ring[1], pre);
    tile_fetch<CIN, NT>(a, in, z0 + 1, y0, x0, pre);
    __syncthreads();
}

// One stage of a convolution step: the MFMA operands of range offset dz
// (index 0..2) and K fragment q -- the RPW + 2 input rows of the wave's RPW
// output rows (X) and the weights of the three row offsets dy (W) -- and
// the 3 RPW products they feed: acc[r] += W[dy]^T X[r + dy]^T.  Operands of
// the next stage are loaded while the current stage's products run, so that
// LDS latency overlaps the matrix cores.
template <int RPW>
struct ConvFrag {
    v8bf X[RPW + 2];
    v8bf W[3];
};

template <int CIN, int RPW>
__device__ __forceinline__ void frag_load(const uint4* slot, const uint4* wsh, int dz, int q, int wave, int m, int h,
                                          ConvFrag<RPW>& f) {
    using G = TileGeo<CIN>;
    int xs, j;
    if constexpr (CIN == 32) {
        xs = m + (q >> 1);
        j = 2 * (q & 1) + h;
    } else {
        xs = m + (q == 0 ? h : 2);
        j = 0;
    }
#pragma unroll
    for (int rr = 0; rr < RPW + 2; ++rr)
        f.X[rr] = __builtin_bit_cast(v8bf, slot[ring_pos<CIN>(RPW * wave + rr, xs, j)]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
        f.W[dy] = __builtin_bit_cast(v8bf, wsh[(((dz * 3 + dy) * G::kQ + q) * 2 + h) * 32 + m]);
}

template <int RPW>
__device__ __forceinline__ void frag_mma(const ConvFrag<RPW>& f, v16f (&acc)[RPW]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int r = 0; r < RPW; ++r)
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.W[dy], f.X[r + dy], acc[r], 0, 0, 0);
}

// Instruction order of one pipelined stage (mask 0x100: LDS reads, 0x200: LDS
// writes, 0x8: MFMA): each of the next stage's RPW + 5 LDS reads issues
// beside one of the current stage's 3 RPW MFMAs (two of them beside the
// first MFMA when the reads outnumber the products), so that they complete
// long before they are waited on, and up to three LDS writes of a slice
// refill ride on the stage's last three MFMAs.
// (The arguments are constants once the stage loops are unrolled.)
template <int RPW>
__device__ __forceinline__ void sched_stage(bool loads, int writes) {
    constexpr int NM = 3 * RPW, NR = RPW + 5;
    constexpr int PAIRED = NR < NM - 3 ? NR : NM - 3;  // reads beside the MFMAs before the last three
    if (loads) {
        if constexpr (NR > PAIRED) __builtin_amdgcn_sched_group_barrier(0x100, NR - PAIRED, 0);
#pragma unroll
        for (int i = 0; i < PAIRED; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x8, 1, 0);
        }
        if constexpr (NM - 3 > PAIRED) __builtin_amdgcn_sched_group_barrier(0x8, NM - 3 - PAIRED, 0);
    } else {
        __builtin_amdgcn_sched_group_barrier(0x8, NM - 3, 0);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i < writes) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x8, 1, 0);
    }
}

// LDS writes of the slice refill carried by stage q (three per stage).
template <int CIN, int NT>
__device__ constexpr int store_share(int q) {
    const int left = TileGeo<CIN, NT>::kFill - 3 * q;
    return left <= 0 ? 0 : left < 3 ? left : 3;
}

// Output run p (0 or 1) of one lane of a 32-channel output row: the lane
// (voxel, half h) holds channels 8 g + 4 h + 0..3 (g = 0..3) in acc; with
// RELU the bias is added and negatives cut, the values go to bf16, and a
// swap between the lane halves turns groups 2 p and 2 p + 1 into the 8
// consecutive channels 16 p + 8 h + 0..7 of the returned 16-byte run.
template <bool RELU>
__device__ __forceinline__ v4u out_run(const v16f& acc, int p, const float (&bias_r)[16]) {
    uint32_t d[2][2];  // [group 2 p + e][channel pair]
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = 4 * (2 * p + e) + 2 * c;
            float lo = acc[i], hi = acc[i + 1];
            if constexpr (RELU) {
                lo = fmaxf(lo + bias_r[i], 0.f);
                hi = fmaxf(hi + bias_r[i + 1], 0.f);
            }
            d[e][c] = pack_bf16x2(lo, hi);
        }
    const auto s0 = __builtin_amdgcn_permlane32_swap(d[0][0], d[1][0], false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(d[0][1], d[1][1], false, false);
    return v4u{s0[0], s1[0], s0[1], s1[1]};
}

// RPW output rows per wave: 16 / RPW waves per block (one per SIMD at
// RPW = 4, two at RPW = 2), each slot fill shared by all of them.
template <int RPW>
constexpr int conv_threads() { return 64 * kTileRows / RPW; }

template <int CIN, int EPI, int RPW>
__global__ __launch_bounds__(conv_threads<RPW>(), 1) void k_conv(ConvArgs a) {
    static_assert(EPI == EPI_RELU || EPI == EPI_DGRAD || EPI == EPI_RAW, "the final layer runs in k_conv_final");
    constexpr int NT = conv_threads<RPW>();
    constexpr int NRD = RPW + 5;  // LDS reads of one stage
    using G = TileGeo<CIN, NT>;
    __shared__ RingSlots<CIN, NT> ring;
    __shared__ uint4 wsh[G::kW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;

    // weight fragments, once per block: every load in flight, then into LDS
    {
        constexpr int kWl = (G::kW + NT - 1) / NT;
        const uint4* wq4 = reinterpret_cast<const uint4*>(a.wq);
        uint4 w[kWl];
#pragma unroll
        for (int i = 0; i < kWl; ++i) {
            const int e = threadIdx.x + i * NT;
            w[i] = e < G::kW ? wq4[e] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < kWl; ++i) {
            const int e = threadIdx.x + i * NT;
            if (e < G::kW) wsh[e] = w[i];
        }
    }
    // output channel of accumulator register i: (i / 4) 8 + 4 h + i % 4
    float bias_r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) bias_r[i] = EPI == EPI_RELU ? a.bias[(i >> 2) * 8 + 4 * h + (i & 3)] : 0.f;

    long t = (long)blockIdx.x * a.span;
    const long total = (long)a.nvol * a.tiles_x * a.tiles_y * a.nz;
    const long tend = t + a.span < total ? t + a.span : total;
    ConvSeg sg;
    while (next_seg(a, t, tend, sg)) {
        const int x0 = sg.xt * kTileCols, y0 = sg.yt * kTileRows;
        const int z0 = sg.z0, z1 = sg.z1;
        const long vol_off = (long)sg.vol * a.nz * a.ny * a.nx;
        const uint16_t* in = a.in + vol_off * CIN;
        uint4 pre[G::kFill];
        seg_prologue<CIN, NT>(a, in, z0, y0, x0, ring, pre);

        int old = 0;  // slot of input z - 1; the other slot holds input z
        for (int z = z0; z < z1; ++z) {
            v16f acc[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) acc[r] = v16f{};
            constexpr int S = G::kQ;  // stages per range offset
            // output slice z: its byte size, element offset, and the byte offset of
            // lane (m, h)'s 16-byte run p of row r of the wave (outside the slice for
            // rows past the volume)
            const uint32_t slice_bytes = (uint32_t)(a.ny * a.nx) * 64u;
            const long slice_off = vol_off + (long)z * a.ny * a.nx;
            auto out_off = [&](int r, int p) {
                const int y = y0 + RPW * wave + r;
                return y < a.ny ? (uint32_t)((y * a.nx + x0 + m) * 64 + 16 * h + 32 * p) : kBufferOutside;
            };
            v4u keep[RPW][2];  // backward-data pass: ReLU mask of the layer input at the outputs
            ConvFrag<RPW> f[2];
            // dz = 0: input z - 1
            frag_load<CIN, RPW>(ring[old], wsh, 0, 0, wave, m, h, f[0]);
            __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (q + 1 < S) {
                    frag_load<CIN, RPW>(ring[old], wsh, 0, q + 1, wave, m, h, f[(q + 1) & 1]);
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(true, 0);
                } else {
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(false, 0);
                }
            }
            __syncthreads();  // every wave is done with input z - 1
            // dz = 1: input z; meanwhile input z + 1 replaces z - 1 and z + 2 is fetched
            frag_load<CIN, RPW>(ring[old ^ 1], wsh, 1, 0, wave, m, h, f[0]);
            tile_store<CIN, NT>(ring[old], pre);
            tile_fetch<CIN, NT>(a, in, z + 2, y0, x0, pre, z + 1 < z1);
            if constexpr (EPI == EPI_DGRAD) {
                const __amdgpu_buffer_rsrc_t keep_rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<uint16_t*>(a.relu_src) + slice_off * 32, 0, slice_bytes, kBufferWord3);
#pragma unroll
                for (int r = 0; r < RPW; ++r)
#pragma unroll
                    for (int p = 0; p < 2; ++p) keep[r][p] = __builtin_amdgcn_raw_buffer_load_b128(keep_rs, out_off(r, p), 0, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (q + 1 < S) {
                    frag_load<CIN, RPW>(ring[old ^ 1], wsh, 1, q + 1, wave, m, h, f[(q + 1) & 1]);
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(true, store_share<CIN, NT>(q));
                } else {
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(false, store_share<CIN, NT>(q));
                }
            }
            __syncthreads();  // input z + 1 is in place
            // dz = 2: input z + 1
            frag_load<CIN, RPW>(ring[old], wsh, 2, 0, wave, m, h, f[0]);
            __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (q + 1 < S) {
                    frag_load<CIN, RPW>(ring[old], wsh, 2, q + 1, wave, m, h, f[(q + 1) & 1]);
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(true, 0);
                } else {
                    frag_mma(f[q & 1], acc);
                    sched_stage<RPW>(false, 0);
                }
            }
            old ^= 1;

            // epilogue: lane (voxel x0 + m, half h) of output row RPW wave + r holds
            // channels 8 g + 4 h + 0..3 (g = 0..3); a swap between the lane halves
            // turns the pairs of groups (2 p, 2 p + 1) into 8 consecutive channels
            // 16 p + 8 h + 0..7 per lane, stored as one 16-byte run.  Buffer
            // stores relative to the output slice: rows past the volume get an
            // offset beyond its size, which the hardware drops -- no branch, so
            // that the number of stores in flight is fixed and the next step's
            // wait for its prefetched slice need not wait for them.
            const __amdgpu_buffer_rsrc_t out_rs =
                __builtin_amdgcn_make_buffer_rsrc(a.out + slice_off * 32, 0, slice_bytes, kBufferWord3);
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const uint32_t off = out_off(r, p);
                    v4u q = out_run<EPI == EPI_RELU>(acc[r], p, bias_r);
                    if constexpr (EPI == EPI_DGRAD) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) q[k] &= relu_keep2(keep[r][p][k]);
                    }
                    __builtin_amdgcn_raw_buffer_store_b128(q, out_rs, off, 0, 0);
                }
            }
        }
    }
}

// First layer of the forward pass (one input channel, 32 output channels,
// bias and ReLU), straight from the fp32 volume.  The input of voxel v is
// bf16(x[v] / m) (m = *scale, 1 without one), rounded as cnn_pack rounds it
// for the 8-channel form.  With one channel, the 27 taps form the MFMA's K
// dimension (padded to 32), so that an output row of 32 voxels takes two
// 32x32x16 products where the 8-channel form takes eighteen.  Lane (voxel n,
// half h) of K fragment f holds, for voxel n, the inputs of
//   f = 0: range offset h, in-slice taps e = 0..7,
//   f = 1, h = 0: range offset 2, in-slice taps e = 0..7,
//   f = 1, h = 1: in-slice tap 8 of range offsets e = 0, 1, 2, then zeros,
// where in-slice tap j is (dy, dx) = (j / 3, j % 3) (offsets +1); the model's
// tap index is 9 dz + j (cnn_prep_first orders the weights alike).  The
// weights W^T [32 channels][32 K] are the A operand and stay in registers.
// The output tile is that of k_conv (16 rows x 32 x-voxels, wave w on rows
// 4w..4w+3), and so are the persistent runs of tile-slices and the epilogue.
// Input slices with halo (18 x 34 bf16) sit in a ring of four LDS slots:
// step z reads the slots of inputs z - 1, z, z + 1 and writes input z + 2
// (fetched into registers a step earlier) into the fourth, so one barrier
// per step orders the writes before the next step's reads.
constexpr int kFirstSlots = 4;
constexpr int kFirstSlice = kRingRows * kRingCols;                      // voxels of an input slice with halo
constexpr int kFirstFill = (kFirstSlice + kCnnBlock - 1) / kCnnBlock;   // values per thread per slice
constexpr int kFirstSlot = kFirstFill * kCnnBlock;                      // slot size, padded for unguarded writes

// In-slot offset of in-slice tap j.
__host__ __device__ constexpr int first_tap_off(int j) { return (j / 3) * kRingCols + j % 3; }

// Loads of input slice zin of the tile (with halo) as fp32, branch-free as
// in tile_fetch: halo voxels outside the volume and slices outside it read 0.
__device__ __forceinline__ void first_fetch(const ConvArgs& a, const float* in, int zin, int y0, int x0,
                                            float (&pre)[kFirstFill], bool live) {
    const bool zok = live && zin >= 0 && zin < a.nz;
    const long plane = (long)a.ny * a.nx;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(in) + (zok ? zin : 0) * plane, 0, zok ? (uint32_t)(plane * 4) : 0u, kBufferWord3);
#pragma unroll
    for (int i = 0; i < kFirstFill; ++i) {
        const int e = threadIdx.x + i * kCnnBlock;
        const int xs = e % kRingCols, ys = e / kRingCols;
        const int y = y0 - 1 + ys, x = x0 - 1 + xs;
        const bool ok = e < kFirstSlice && y >= 0 && y < a.ny && x >= 0 && x < a.nx;
        const uint32_t off = ok ? (uint32_t)((y * a.nx + x) * 4) : kBufferOutside;
        pre[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    }
}

// Input slice zi of the ring: slot zi mod 4 (zi >= -1), as an element offset.
__device__ __forceinline__ int first_slot(int zi) { return ((zi + 4) & 3) * kFirstSlot; }

__device__ __forceinline__ void first_store(uint16_t* ring, int zi, const float (&pre)[kFirstFill], float inv) {
    uint16_t* slot = ring + first_slot(zi);
#pragma unroll
    for (int i = 0; i < kFirstFill; ++i) slot[threadIdx.x + i * kCnnBlock] = f2bf(pre[i] * inv);
}

__global__ __launch_bounds__(kCnnBlock, 2) void k_conv_first(ConvArgs a) {
    __shared__ uint16_t ring[kFirstSlots * kFirstSlot];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    const float inv = a.scale != nullptr ? 1.f / *a.scale : 1.f;
    // weight fragments: lane (channel m, half h) of fragment f (cnn_prep_first)
    v8bf W[2];
    {
        const uint4* wq4 = reinterpret_cast<const uint4*>(a.wq);
#pragma unroll
        for (int f = 0; f < 2; ++f) W[f] = __builtin_bit_cast(v8bf, wq4[(2 * f + h) * 32 + m]);
    }
    // output channel of accumulator register i: (i / 4) 8 + 4 h + i % 4
    float bias_r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) bias_r[i] = a.bias[(i >> 2) * 8 + 4 * h + (i & 3)];

    long t = (long)blockIdx.x * a.span;
    const long total = (long)a.nvol * a.tiles_x * a.tiles_y * a.nz;
    const long tend = t + a.span < total ? t + a.span : total;
    ConvSeg sg;
    while (next_seg(a, t, tend, sg)) {
        const int x0 = sg.xt * kTileCols, y0 = sg.yt * kTileRows;
        const int z0 = sg.z0, z1 = sg.z1;
        const long vol_off = (long)sg.vol * a.nz * a.ny * a.nx;
        const float* in = a.xin + vol_off;
        // prologue: inputs z0 - 1, z0, z0 + 1 into their slots, z0 + 2 into
        // registers; the leading barrier keeps the previous segment's readers
        // away from the slots
        float pre[kFirstFill];
        {
            float p0[kFirstFill], p1[kFirstFill], p2[kFirstFill];
            first_fetch(a, in, z0 - 1, y0, x0, p0, true);
            first_fetch(a, in, z0, y0, x0, p1, true);
            first_fetch(a, in, z0 + 1, y0, x0, p2, z0 + 1 <= z1);
            __syncthreads();
            first_store(ring, z0 - 1, p0, inv);
            first_store(ring, z0, p1, inv);
            first_store(ring, z0 + 1, p2, inv);
            first_fetch(a, in, z0 + 2, y0, x0, pre, z0 + 2 <= z1);
            __syncthreads();
        }
        for (int z = z0; z < z1; ++z) {
            // input z + 2 into its slot (read from the next step on), input
            // z + 3 into registers
            first_store(ring, z + 2, pre, inv);
            first_fetch(a, in, z + 3, y0, x0, pre, z + 3 <= z1);
            const int s0 = first_slot(z - 1), s1 = first_slot(z), s2 = first_slot(z + 1);
            const int sh = h ? s1 : s0;  // fragment 0: range offset h
            v16f acc[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int base = (4 * wave + r) * kRingCols + m;
                uint32_t v0[8], v1[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    v0[e] = ring[sh + base + first_tap_off(e)];
                    // fragment 1: lanes h = 0 read range offset 2, tap e; lanes
                    // h = 1 read tap 8 of range offset e (e < 3), else zero
                    const int i1 = e < 3 ? (h ? (e == 0 ? s0 : e == 1 ? s1 : s2) + base + first_tap_off(8)
                                              : s2 + base + first_tap_off(e))
                                         : s2 + base + first_tap_off(e);
                    const uint32_t u = ring[i1];
                    v1[e] = (e >= 3 && h) ? 0u : u;
                }
                const v8bf B0 = __builtin_bit_cast(
                    v8bf, v4u{v0[0] | (v0[1] << 16), v0[2] | (v0[3] << 16), v0[4] | (v0[5] << 16), v0[6] | (v0[7] << 16)});
                const v8bf B1 = __builtin_bit_cast(
                    v8bf, v4u{v1[0] | (v1[1] << 16), v1[2] | (v1[3] << 16), v1[4] | (v1[5] << 16), v1[6] | (v1[7] << 16)});
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W[0], B0, v16f{}, 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W[1], B1, acc[r], 0, 0, 0);
            }
            // epilogue as k_conv's: rows past the volume get an offset outside
            // the output slice, which the hardware drops
            const uint32_t slice_bytes = (uint32_t)(a.ny * a.nx) * 64u;
            const long slice_off = vol_off + (long)z * a.ny * a.nx;
            const __amdgpu_buffer_rsrc_t out_rs =
                __builtin_amdgcn_make_buffer_rsrc(a.out + slice_off * 32, 0, slice_bytes, kBufferWord3);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = y0 + 4 * wave + r;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const uint32_t off =
                        y < a.ny ? (uint32_t)((y * a.nx + x0 + m) * 64 + 16 * h + 32 * p) : kBufferOutside;
                    __builtin_amdgcn_raw_buffer_store_b128(out_run<true>(acc[r], p, bias_r), out_rs, off, 0, 0);
                }
            }
            __syncthreads();  // slot z + 2 written; slot z - 1 free for input z + 3
        }
    }
}

// Final layer of the forward pass (32 input channels, one output channel):
// out[v] = xin[v] + scale (b + sum_t P_t[v + off(t)]) with the tap partials
// P_t[u] = sum_ci x[u][ci] W[t][ci] of every input voxel u.  A direct
// convolution would read 27 x 64 bytes of input per output from LDS for one
// output channel; instead the matrix cores form all 27 partials of each input
// voxel at once (D[t][u] = W^T X^T on the 32x32x16 MFMA, taps padded to 32),
// they go to LDS as fp32 P[t][u], and each output gathers its 27 partials
// (108 bytes).  Per input slice z' of the block's tile (18 x 34 voxels with
// the halo, flattened to u = ys 34 + xs and cut into 20 chunks of 32), each
// wave computes 5 chunks straight from global memory (operands in MFMA
// layout, prefetched one slice ahead), then each thread adds the partials of
// its two outputs (x = lane, rows r and r + 8) into three rolling sums, for
// output slices z' + 1, z' and z' - 1 (range taps dz = 0, 1, 2); after input
// z' the sum of output z' - 1 is complete and is stored.
constexpr int kFinHalo = kRingRows * kRingCols;      // voxels of an input slice with halo
constexpr int kFinChunks = (kFinHalo + 31) / 32;     // chunks of 32 voxels
constexpr int kFinCols = kFinChunks * 32;             // voxel columns of P
constexpr int kFinPerWave = (kFinChunks + 3) / 4;    // chunks per wave

// MFMA operands of input slice zin: for chunk k of this wave (c = wave + 4 k)
// and channel half e, lane (n, hh) gets channels 16 e + 8 hh .. + 7 of voxel
// u = 32 c + n (zero outside the volume, the halo or the slice).
__device__ __forceinline__ void final_fetch(const ConvArgs& a, const uint16_t* in, int zin, int y0, int x0, int wave,
                                           int n, int hh, v4u (&xb)[kFinPerWave][2]) {
    const bool zok = zin >= 0 && zin < a.nz;
    const long plane = (long)a.ny * a.nx;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(in) + (zok ? zin : 0) * plane * 32, 0, zok ? (uint32_t)(plane * 64) : 0u, kBufferWord3);
#pragma unroll
    for (int k = 0; k < kFinPerWave; ++k) {
        const int u = 32 * (wave + 4 * k) + n;
        const int ys = u / kRingCols, xs = u % kRingCols;
        const int y = y0 - 1 + ys, x = x0 - 1 + xs;
        const bool ok = u < kFinHalo && y >= 0 && y < a.ny && x >= 0 && x < a.nx;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t off = ok ? (uint32_t)((y * a.nx + x) * 64 + 32 * e + 16 * hh) : kBufferOutside;
            xb[k][e] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        }
    }
}

__global__ __launch_bounds__(kCnnBlock) void k_conv_final(ConvArgs a) {
    static_assert(kCnnBlock == 8 * kTileCols && kTileRows == 16, "two output rows per thread");
    static_assert(4 * kFinPerWave >= kFinChunks, "four waves cover the chunks");
    __shared__ float P[27][kFinCols];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 31, hh = lane >> 5;
    const int x = tid & 31, r0 = tid >> 5;  // gather: output rows r0 and r0 + 8 of the tile

    // A operand W^T: lane (t, hh), channel half e holds W[t][16 e + 8 hh + 0..7]
    // (zero for the padding taps t >= 27), from the fragment layout
    // wq[g][q][h][n][8] at output channel 0 (g = t / 3, q = 2 (t % 3) + e)
    v8bf wa[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (n < 27) w = *reinterpret_cast<const uint4*>(a.wq + ((((n / 3) * 6 + 2 * (n % 3) + e) * 2 + hh) * 32) * 8);
        wa[e] = __builtin_bit_cast(v8bf, w);
    }
    const float bias = a.bias[0];
    const float scale = a.scale != nullptr ? *a.scale : 1.f;

    long t = (long)blockIdx.x * a.span;
    const long total = (long)a.nvol * a.tiles_x * a.tiles_y * a.nz;
    const long tend = t + a.span < total ? t + a.span : total;
    ConvSeg sg;
    while (next_seg(a, t, tend, sg)) {
        const int x0 = sg.xt * kTileCols, y0 = sg.yt * kTileRows;
        const int z0 = sg.z0, z1 = sg.z1;
        const long vol_off = (long)sg.vol * a.nz * a.ny * a.nx;
        const uint16_t* in = a.in + vol_off * 32;
        v4u xb[kFinPerWave][2];
        final_fetch(a, in, z0 - 1, y0, x0, wave, n, hh, xb);
        // rolling sums of outputs z' - 1, z', z' + 1 for the two rows
        float s_lo[2] = {0.f, 0.f}, s_mid[2] = {0.f, 0.f}, s_hi[2] = {0.f, 0.f};
        for (int zi = z0 - 1; zi <= z1; ++zi) {
            // tap partials of input slice zi into P, chunk by chunk
            __syncthreads();  // the previous slice's gathers are done with P
#pragma unroll
            for (int k = 0; k < kFinPerWave; ++k) {
                const int c = wave + 4 * k;
                v16f d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[0], __builtin_bit_cast(v8bf, xb[k][0]), v16f{}, 0,
                                                                 0, 0);
                d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[1], __builtin_bit_cast(v8bf, xb[k][1]), d, 0, 0, 0);
                if (c < kFinChunks) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int tap = (i / 4) * 8 + 4 * hh + (i % 4);  // D row of register i
                        if (tap < 27) P[tap][32 * c + n] = d[i];
                    }
                }
            }
            if (zi < z1) final_fetch(a, in, zi + 1, y0, x0, wave, n, hh, xb);
            __syncthreads();
            // gather: input zi feeds output zi + 1 - dz through the taps of range offset dz
            float g[3][2];
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    float acc = 0.f;
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
                            acc += P[9 * dz + 3 * dy + dx][(r0 + 8 * k + dy) * kRingCols + x + dx];
                    g[dz][k] = acc;
                }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                s_lo[k] += g[2][k];   // output zi - 1
                s_mid[k] += g[1][k];  // output zi
                s_hi[k] += g[0][k];   // output zi + 1
            }
            const int zo = zi - 1;
            if (zo >= z0) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int y = y0 + r0 + 8 * k;
                    if (y < a.ny) {
                        const long v = vol_off + ((long)zo * a.ny + y) * a.nx + x0 + x;
                        a.out_f32[v] = a.xin[v] + scale * (s_lo[k] + bias);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                s_lo[k] = s_mid[k];
                s_mid[k] = s_hi[k];
                s_hi[k] = 0.f;
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

// ---------------------------------------------------------------------------
// Weight and bias gradients of one layer, tiled implicit GEMM on the 32x32x16
// bf16 MFMA.  For every tap t: D_t[co][ci] = sum_v g[v][co] act[v + off(t)][ci]
// (the MFMA's M = co, N = ci, K = 16 voxels along x), and the bias gradient
// sum_v g[v][co] as an MFMA against ones.
//
// A persistent grid walks work items (volume, 8 output rows x 32 x-voxels,
// chunk of range slices).  Per range slice z the block holds in LDS, channel
// major ("transposed", x contiguous): g of the 8 x 32 output tile (two
// slots), and act of slices z - 1, z, z + 1 over 10 rows x 32 x-voxels (x0 ..
// x0 + 31) in a ring of four slots, with the one-voxel x halo of each row and
// channel (voxels x0 - 1 and x0 + 32) in a separate array
// [slot][row][side][channel], where the 64 lanes of a wave read 64
// consecutive dwords.  While step z runs, the filling waves store act slice
// z + 2 and g slice z + 1, loaded during the previous step, into the slots
// step z does not read, and load the next ones: one barrier per step, and
// the loads have a whole step to arrive.  Global data is channels-last; each
// fill unit loads 8 voxels x 8 channels and transposes them in registers
// (byte permutes).
// The MFMA's K = 16 voxels: lanes h = 0 and 1 of a channel take the x-voxels
// x0 + 16 h .. x0 + 16 h + 15 over the two MFMAs of an output row (the K
// index only has to agree between A and B).  The dx = -1 and +1 operands come
// from the lane's two aligned 8-voxel chunks and one dword on either side:
// the inner one from the other half of the wave (permlane32_swap), the outer
// one from the halo array; no per-tap LDS dword read.
// Eight waves per block, two per SIMD (each holds 7 accumulator tiles, 112
// AGPRs), so that one wave's LDS waits, fills and barriers overlap the other's
// MFMAs.  Wave (tg, kh): taps 7 tg .. 7 tg + 6 (tg = 3: taps 21 .. 26 and the
// bias), output rows 4 kh .. 4 kh + 3.  The two row halves of a tap group
// are added through LDS at the end, and the block writes its sums to
// part[block][28][32][32] (tap 27 = bias); k_wgrad_reduce adds the blocks'
// partial sums in a fixed order.
// Channel planes are padded to an odd number of 16-byte chunks (41 and 33) so
// that the lanes of one 128-bit LDS phase hit distinct bank groups.
constexpr int kWgRows = 8;
constexpr int kWgBlock = 512;
constexpr int kActPlane4 = 41;  // uint4 per channel plane of an act slot (10 x 32 bf16 + 8 pad)
constexpr int kGPlane4 = 33;    // uint4 per channel plane of the g tile (8 x 32 bf16 + 8 pad)
constexpr int kHaloSlot = 10 * 2 * 32;  // dwords of an act slot's halo array
static_assert(2 * 7 * 16 * 64 * sizeof(float) <= 4 * 32 * kActPlane4 * sizeof(uint4),
              "the act slots hold two tap groups' sums for the row-half combine");

// 8 x 8 bf16 transpose: in[v][k] = dword k (channels 2k, 2k + 1) of voxel v;
// out[c][p] = dword p (voxels 2p, 2p + 1) of channel c.
__device__ __forceinline__ void transpose8(const uint32_t (&in)[8][4], uint32_t (&out)[8][4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t lo = in[2 * p][k], hi = in[2 * p + 1][k];
            out[2 * k][p] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
            out[2 * k + 1][p] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);
        }
}

// Loads 8 voxels (x, x + 1, .., x + 7 of one row) x 8 channels (group cg) of
// a channels-last tensor with C stored channels.  Where `ok` is false (or the
// group is past C) the lanes read the tensor's first 16 bytes instead, and
// the returned flag is false: the caller zeroes them with mask8x8 when it
// consumes them, so that nothing waits on the loads before then.
template <int C>
__device__ __forceinline__ bool load8x8(const uint16_t* base, long vox0, int cg, bool ok, uint32_t (&v)[8][4]) {
    ok = ok && cg * 8 < C;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint4 q = *reinterpret_cast<const uint4*>(base + (ok ? (vox0 + e) * C + cg * 8 : 0));
        v[e][0] = q.x;
        v[e][1] = q.y;
        v[e][2] = q.z;
        v[e][3] = q.w;
    }
    return ok;
}

__device__ __forceinline__ void mask8x8(bool ok, uint32_t (&v)[8][4]) {
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[e][k] = ok ? v[e][k] : 0u;
}

// Operand of tap dx of an 8-voxel chunk c (voxels x .. x + 7): dx = 0 takes
// x - 1 .. x + 6 (before: the dword holding x - 2, x - 1), dx = 2 takes
// x + 1 .. x + 8 (after: the dword holding x + 8, x + 9).
__device__ __forceinline__ uint4 shifted_chunk(uint4 c, uint32_t before, uint32_t after, int dx) {
    if (dx == 1) return c;
    uint4 q;
    if (dx == 0) {
        q.x = __builtin_amdgcn_alignbyte(c.x, before, 2);
        q.y = __builtin_amdgcn_alignbyte(c.y, c.x, 2);
        q.z = __builtin_amdgcn_alignbyte(c.z, c.y, 2);
        q.w = __builtin_amdgcn_alignbyte(c.w, c.z, 2);
    } else {
        q.x = __builtin_amdgcn_alignbyte(c.y, c.x, 2);
        q.y = __builtin_amdgcn_alignbyte(c.z, c.y, 2);
        q.z = __builtin_amdgcn_alignbyte(c.w, c.z, 2);
        q.w = __builtin_amdgcn_alignbyte(after, c.w, 2);
    }
    return q;
}

template <int TG, int CA, int CG>
__device__ __forceinline__ void wgrad_block(const WgradArgs& a, uint4 (*act)[32 * kActPlane4],
                                            uint32_t (*halo)[kHaloSlot], uint4 (*gt)[32 * kGPlane4], int wave) {
    constexpr int T0 = 7 * TG;
    constexpr int NT = TG == 3 ? 6 : 7;
    constexpr bool BIAS = TG == 3;
    const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5, kh = wave & 1;
    const int u = threadIdx.x;
    v16f acc[NT];
    v16f accb = {};
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v16f{};
    v8bf ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;

    // fill-unit coordinates: act units 0..239 on threads 0..239 (chunk a_xc of
    // a row: 0 and 5 are the halo chunks), g units 0..127 on threads 384..511
    // (waves 6 and 7); the role is uniform per wave, and one prefetch buffer
    // serves both
    const bool act_role = u < 256, g_role = u >= 384;
    const int a_xc = u % 6, a_ys = (u / 6) % 10, a_cg = u / 60;
    const int gu = u - 384, g_xc = gu & 3, g_r = (gu >> 2) & 7, g_cg = gu >> 5;
    uint32_t pf[8][4], tr[8][4];
    bool pf_ok = false;

    for (int item = blockIdx.x; item < a.items; item += gridDim.x) {
        int b = item;
        const int xt = b % a.tiles_x;
        b /= a.tiles_x;
        const int yt = b % a.tiles_y;
        b /= a.tiles_y;
        const int zc = b % a.zchunks;
        const int vol = b / a.zchunks;
        const int x0 = xt * 32, y0 = yt * kWgRows, z0 = zc * a.zc;
        const int z1 = z0 + a.zc < a.nz ? z0 + a.zc : a.nz;
        const long vol_off = (long)vol * a.nz * a.ny * a.nx;

        auto fetch_act = [&](int zin) {
            const int y = y0 - 1 + a_ys, x = x0 - 8 + 8 * a_xc;
            const bool ok = u < 240 && zin >= 0 && zin < a.nz && y >= 0 && y < a.ny && x >= 0 && x < a.nx;
            pf_ok = load8x8<CA>(a.act, ok ? vol_off + ((long)zin * a.ny + y) * a.nx + x : 0, a_cg, ok, pf);
        };
        auto fetch_g = [&](int zz) {
            const int y = y0 + g_r, x = x0 + 8 * g_xc;
            const bool ok = gu >= 0 && gu < 128 && zz < a.nz && y < a.ny;
            pf_ok = load8x8<CG>(a.g, ok ? vol_off + ((long)zz * a.ny + y) * a.nx + x : 0, g_cg, ok, pf);
        };
        auto store_act = [&](int zin) {
            if (u < 240) {
                mask8x8(pf_ok, pf);
                transpose8(pf, tr);
                const int s = (zin + 4) & 3;
                if (a_xc == 0 || a_xc == 5) {  // keep the dword next to the tile: x0 - 2, x0 - 1 or x0 + 32, x0 + 33
                    uint32_t* hs = halo[s] + (a_ys * 2 + (a_xc == 5 ? 1 : 0)) * 32 + a_cg * 8;
#pragma unroll
                    for (int k = 0; k < 8; ++k) hs[k] = a_xc == 0 ? tr[k][3] : tr[k][0];
                } else {
                    uint4* slot = act[s];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        slot[(a_cg * 8 + k) * kActPlane4 + a_ys * 4 + a_xc - 1] =
                            make_uint4(tr[k][0], tr[k][1], tr[k][2], tr[k][3]);
                }
            }
        };
        auto store_g = [&](int zz) {
            if (gu >= 0 && gu < 128) {
                mask8x8(pf_ok, pf);
                transpose8(pf, tr);
                uint4* gs = gt[zz & 1];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    gs[(g_cg * 8 + k) * kGPlane4 + g_r * 4 + g_xc] = make_uint4(tr[k][0], tr[k][1], tr[k][2], tr[k][3]);
            }
        };

        // Ring of four act slots (slice zin in slot zin mod 4) and two g
        // slots: step z reads act slices z - 1 .. z + 1 and g slice z, while
        // the filling waves store act slice z + 2 and g slice z + 1 (loaded a
        // step earlier) into the slots it does not read; one barrier per step.
        __syncthreads();  // the previous item's reads are done
        if (act_role) {
            fetch_act(z0 - 1);
            store_act(z0 - 1);
            fetch_act(z0);
            store_act(z0);
            fetch_act(z0 + 1);
            store_act(z0 + 1);
            if (z0 + 1 < z1) fetch_act(z0 + 2);
        } else if (g_role) {
            fetch_g(z0);
            store_g(z0);
            if (z0 + 1 < z1) fetch_g(z0 + 1);
        }
        __syncthreads();

        for (int z = z0; z < z1; ++z) {
            const uint4* gz = gt[z & 1];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int r = 4 * kh + rr;
                // A of the row's two MFMAs: g at x0 + 16 h .. + 7 and x0 + 16 h + 8 .. + 15
                const v8bf A0 = __builtin_bit_cast(v8bf, gz[m * kGPlane4 + r * 4 + 2 * h]);
                const v8bf A1 = __builtin_bit_cast(v8bf, gz[m * kGPlane4 + r * 4 + 2 * h + 1]);
                if constexpr (BIAS) {
                    accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, ones, accb, 0, 0, 0);
                    accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, ones, accb, 0, 0, 0);
                }
#pragma unroll
                for (int pair = 0; pair < 9; ++pair) {
                    const int t_lo = pair * 3;
                    if (t_lo + 2 < T0 || t_lo >= T0 + NT) continue;  // no tap of this wave
                    const int dz = pair / 3, dy = pair % 3, s = (z + dz + 3) & 3;
                    const uint4* row = act[s] + m * kActPlane4 + (r + dy) * 4 + 2 * h;
                    const uint4 c0 = row[0], c1 = row[1];
                    const uint32_t hw = halo[s][(r + dy) * 64 + lane];
                    // lanes h = 0 need the upper half's c0.x (x0 + 16, 17); lanes h = 1 the lower half's c1.w (x0 + 14, 15)
                    const uint32_t v = h ? c0.x : c1.w;
                    const auto sw = __builtin_amdgcn_permlane32_swap(v, v, false, false);
                    const uint32_t inner = h ? sw[0] : sw[1];
                    const uint32_t before = h ? inner : hw, after = h ? hw : inner;
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const int t = t_lo + dx;
                        if (t < T0 || t >= T0 + NT) continue;
                        const uint4 b0 = shifted_chunk(c0, before, c1.x, dx);
                        const uint4 b1 = shifted_chunk(c1, c0.w, after, dx);
                        acc[t - T0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, __builtin_bit_cast(v8bf, b0),
                                                                               acc[t - T0], 0, 0, 0);
                        acc[t - T0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, __builtin_bit_cast(v8bf, b1),
                                                                               acc[t - T0], 0, 0, 0);
                    }
                }
            }
            if (z + 1 < z1) {
                if (act_role) {
                    store_act(z + 2);
                    if (z + 2 < z1) fetch_act(z + 3);
                } else if (g_role) {
                    store_g(z + 1);
                    if (z + 2 < z1) fetch_g(z + 2);
                }
                __syncthreads();  // slices z + 2 and z + 1 are in; step z's slots are free for step z + 1's fill
            }
        }
    }
    // The two waves of a tap group (kh = 0, 1) hold sums over different
    // output rows.  kh = 1 hands its sums to kh = 0 through LDS (the act
    // slots, free once every wave is past its last item), two tap groups at a
    // time, and kh = 0 writes the block's partial sums D[co][ci] (co =
    // d_row(lane, i), ci = m) to part[block][28][32][32], tap 27 the bias.
    // Every wave passes the same four barriers.
    float* red = reinterpret_cast<float*>(&act[0][0]);
    float* dst = a.part + (long)blockIdx.x * 28 * 1024;
#pragma unroll
    for (int phase = 0; phase < 2; ++phase) {
        constexpr int kSlot = 7 * 16 * 64;  // floats of one tap group's sums
        const bool mine = (TG >> 1) == phase;
        float* slot = red + (TG & 1) * kSlot;
        __syncthreads();  // the tiles (phase 0) or the previous phase's slots are free
        if (mine && kh == 1) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) slot[(t * 16 + i) * 64 + lane] = acc[t][i];
            if constexpr (BIAS) {
#pragma unroll
                for (int i = 0; i < 16; ++i) slot[(6 * 16 + i) * 64 + lane] = accb[i];
            }
        }
        __syncthreads();
        if (mine && kh == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    dst[(T0 + t) * 1024 + d_row(lane, i) * 32 + m] = acc[t][i] + slot[(t * 16 + i) * 64 + lane];
            if constexpr (BIAS) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    dst[27 * 1024 + d_row(lane, i) * 32 + m] = accb[i] + slot[(6 * 16 + i) * 64 + lane];
            }
        }
    }
}

template <int CA, int CG>
__global__ __launch_bounds__(kWgBlock, 1) void k_wgrad(WgradArgs a) {
    __shared__ uint4 act[4][32 * kActPlane4];
    __shared__ uint32_t halo[4][kHaloSlot];
    __shared__ uint4 gt[2][32 * kGPlane4];
    const int wave = threadIdx.x >> 6;
    switch (wave >> 1) {
        case 0: wgrad_block<0, CA, CG>(a, act, halo, gt, wave); break;
        case 1: wgrad_block<1, CA, CG>(a, act, halo, gt, wave); break;
        case 2: wgrad_block<2, CA, CG>(a, act, halo, gt, wave); break;
        default: wgrad_block<3, CA, CG>(a, act, halo, gt, wave); break;
    }
}

// gw[(t * cin + ci) * cout + co] = sum over chunks of part[c][t][co][ci] and
// gb[co] = sum over chunks of part[c][27][co][0]: a block covers 16
// consecutive positions p = t * 1024 + co * 32 + ci; thread (p, l) sums
// chunks l, l + 16, ... in order, then the 16 partial sums are added in order
// (a fixed summation order, so runs are bitwise repeatable).
__global__ __launch_bounds__(kCnnBlock) void k_wgrad_reduce(const float* part, int chunks, int cin, int cout,
                                                            float* gw, float* gb) {
    __shared__ double red[16][16];
    const int pl = threadIdx.x & 15, l = threadIdx.x >> 4;
    const int p = blockIdx.x * 16 + pl;
    double s = 0.0;
    // chunks l, l + 16, ... in order, eight loads in flight
    int c = l;
    for (; c + 7 * 16 < chunks; c += 8 * 16) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(long)(c + 16 * u) * 28 * 1024 + p];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < chunks; c += 16) s += part[(long)c * 28 * 1024 + p];
    red[l][pl] = s;
    __syncthreads();
    if (l == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k][pl];
        const int ci = p & 31, co = (p >> 5) & 31, tap = p >> 10;
        if (tap < 27) {
            if (ci < cin && co < cout) gw[(tap * cin + ci) * cout + co] = (float)t;
        } else if (ci == 0 && co < cout) {
            gb[co] = (float)t;
        }
    }
}

// Gradient-norm clipping state: clip[0] the running norm of the (clipped)
// gradients, clip[1] the factor for the coming step -- min(1, kClipRatio x
// running norm / norm), 1 on the first step, 0 for a non-finite norm (the
// step is skipped).  The squared norm is summed in a fixed order: block b of
// k_grad_sq adds the float4s b x kCnnBlock + tid, stepping by the grid, into
// clip's partial sums (float64, from byte 8), then k_grad_clip adds those in
// block order.
constexpr float kClipRatio = 3.f;
constexpr float kClipDecay = 0.95f;

__global__ __launch_bounds__(kCnnBlock) void k_grad_sq(const float* g, int n, double* part) {
    // the unaligned head (if any) and the tail one by one
    const int head = (int)((16 - (reinterpret_cast<uintptr_t>(g) & 15)) & 15) / 4;
    const int h = head < n ? head : n;
    const int n4 = (n - h) / 4;
    const float4* g4 = reinterpret_cast<const float4*>(g + h);
    const int tid = blockIdx.x * kCnnBlock + threadIdx.x, stride = kNormBlocks * kCnnBlock;
    double acc = 0.0;
    for (int i = tid; i < n4; i += stride) {
        const float4 v = g4[i];
        acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    }
    if (tid < h) acc += (double)g[tid] * g[tid];
    for (int i = h + 4 * n4 + tid; i < n; i += stride) acc += (double)g[i] * g[i];
    double a[1] = {acc};
    cnn_block_sum<1>(a, part + blockIdx.x);
}

__global__ void k_grad_clip(const double* part, float* clip) {
    if (threadIdx.x != 0) return;
    double sq = 0.0;
    for (int b = 0; b < kNormBlocks; ++b) sq += part[b];
    const float norm = (float)sqrt(sq);
    const float run = clip[0];
    float c;
    if (!isfinite(norm)) {
        c = 0.f;
    } else if (run <= 0.f) {
        c = 1.f;
        clip[0] = norm;
    } else {
        const float cap = kClipRatio * run;
        c = norm > cap ? cap / norm : 1.f;
        clip[0] = kClipDecay * run + (1.f - kClipDecay) * fminf(norm, cap);
    }
    clip[1] = c;
}

// Adam with bias correction on the flat parameter vector, with the gradient
// scaled by the clipping factor (factor 0: no update at all).
__global__ __launch_bounds__(kCnnBlock) void k_adam(float* p, float* m, float* v, const float* g, int n, float lr,
                                                    float b1, float b2, float eps, float c1, float c2,
                                                    const float* clip) {
    const int i = blockIdx.x * kCnnBlock + threadIdx.x;
    const float c = clip[1];
    if (i >= n || !(c > 0.f)) return;
    const float gi = c * g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Weight fragments of the tiled convolution: wq[g = 3 dz + dy][q][h][n][8]
// (bf16) holds k = 8 h .. 8 h + 7 of K fragment q for output channel n, for
// the input-channel count CINP (8 or 32), from the fp32 W[t][cin][cout].
// Forward: the effective weight is W[t][ci][co]; backward data (flip):
// W[26 - t][co][ci] with the channel roles swapped.  Entries beyond the real
// channel counts and the zero half of the last 8-channel fragment are zero.
__device__ __forceinline__ void prep_q_elem(const float* W, int cin, int cout, int flip, int cinp, uint16_t* wq,
                                            int e) {
    const int nq = cinp == 32 ? 6 : 2;
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

// A layer's operands in one launch: the forward fragments (blocks 0 ..
// nb_f - 1), the backward-data fragments (the next nb_d blocks; none without
// wqd) and, in the last block, the zero-padded fp32 copy of the bias.
__global__ __launch_bounds__(kCnnBlock) void k_prep_layer(const float* W, const float* b, int cin, int cout,
                                                         int cinp, int coutp, uint16_t* wq, uint16_t* wqd,
                                                         float* bias32, int nb_f, int nb_d) {
    const int blk = blockIdx.x;
    if (blk < nb_f) {
        prep_q_elem(W, cin, cout, 0, cinp, wq, blk * kCnnBlock + threadIdx.x);
    } else if (blk < nb_f + nb_d) {
        prep_q_elem(W, cin, cout, 1, coutp, wqd, (blk - nb_f) * kCnnBlock + threadIdx.x);
    } else {
        const int e = threadIdx.x;
        if (e < 32) bias32[e] = e < cout ? b[e] : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Launchers
static int grid_for(long work, int per_block, int cap) {
    long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

// Launch of a persistent convolution: as many blocks as fit on the chip at
// once (resident blocks per CU, which the kernel's LDS and registers decide,
// times the CU count; computed once per kernel), each with a contiguous run
// of output tile-slices.
template <void (*K)(ConvArgs), int NT = kCnnBlock>
static hipError_t launch_conv(ConvArgs a, long total, hipStream_t st) {
    static int cap = 0;
    if (cap == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K, NT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        cap = per_cu * cnn_wgrad_grid();
    }
    a.span = (int)((total + cap - 1) / cap);
    const unsigned grid = (unsigned)((total + a.span - 1) / a.span);
    hipLaunchKernelGGL(K, dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

// Rows per wave of the 8- and 32-channel convolutions: two for the forward
// layers, four for the backward-data ones.
template <int EPI>
constexpr int conv_rpw() { return EPI == EPI_RELU ? 2 : 4; }

// First-layer fragments (k_conv_first): wq[f][h][n][8] = W[t][n] with the
// model tap t = 9 dz + j of K element (f, h, k8) -- f = 0: dz = h, j = k8;
// f = 1, h = 0: dz = 2, j = k8; f = 1, h = 1: dz = k8, j = 8 for k8 < 3,
// else 0 -- for W [27][1][32] (tap, input, output).
__global__ __launch_bounds__(kCnnBlock) void k_prep_first(const float* W, uint16_t* wq) {
    const int e = blockIdx.x * kCnnBlock + threadIdx.x;
    if (e >= 2 * 2 * 32 * 8) return;
    const int k8 = e % 8, n = (e / 8) % 32, hh = (e / 256) % 2, f = e / 512;
    int t = -1;
    if (f == 0) t = 9 * hh + k8;
    else if (hh == 0) t = 18 + k8;
    else if (k8 < 3) t = 9 * k8 + 8;
    wq[e] = f2bf(t >= 0 ? W[t * 32 + n] : 0.f);
}

hipError_t cnn_prep_first(const float* W, uint16_t* wq, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_first, dim3(4), dim3(kCnnBlock), 0, st, W, wq);
    return hipGetLastError();
}

hipError_t cnn_conv(int cin, int epi, ConvArgs a, hipStream_t st) {
    // one slice of a 32-channel tensor must stay below the buffer offset that marks "outside"
    if ((long)a.ny * a.nx * 64 >= (long)kBufferOutside) return hipErrorInvalidValue;
    a.tiles_x = a.nx / kTileCols;
    a.tiles_y = (a.ny + kTileRows - 1) / kTileRows;
    const long total = (long)a.nvol * a.tiles_x * a.tiles_y * a.nz;
    if (total <= 0) return hipSuccess;
    if (cin == 1 && epi == EPI_RELU) return launch_conv<k_conv_first>(a, total, st);
#define CONV(C, E) launch_conv<k_conv<C, E, conv_rpw<E>()>, conv_threads<conv_rpw<E>()>()>(a, total, st)
    if (cin == 8 && epi == EPI_RELU) return CONV(8, EPI_RELU);
    if (cin == 32 && epi == EPI_RELU) return CONV(32, EPI_RELU);
    if (cin == 32 && epi == EPI_FINAL) return launch_conv<k_conv_final>(a, total, st);
    if (cin == 8 && epi == EPI_DGRAD) return CONV(8, EPI_DGRAD);
    if (cin == 32 && epi == EPI_DGRAD) return CONV(32, EPI_DGRAD);
    if (cin == 8 && epi == EPI_RAW) return CONV(8, EPI_RAW);
    if (cin == 32 && epi == EPI_RAW) return CONV(32, EPI_RAW);
#undef CONV
    return hipErrorInvalidValue;
}

size_t cnn_wq_elems(int cinp) { return (size_t)9 * (cinp == 32 ? 6 : 2) * 32 * 16; }


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

int cnn_wgrad_grid() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
        cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    }
    return cus;
}

size_t cnn_wgrad_part_bytes() { return (size_t)cnn_wgrad_grid() * 28 * 1024 * sizeof(float); }

hipError_t cnn_wgrad(int ca, int cg, WgradArgs a, int cin, int cout, float* gw, float* gb, hipStream_t st) {
    a.tiles_x = a.nx / 32;
    a.tiles_y = (a.ny + kWgRows - 1) / kWgRows;
    const long tiles = (long)a.nvol * a.tiles_x * a.tiles_y;
    const int grid_max = cnn_wgrad_grid();
    a.zc = 16;
    while (a.zc > 2 && tiles * ((a.nz + a.zc - 1) / a.zc) < 2L * grid_max) a.zc /= 2;
    a.zchunks = (a.nz + a.zc - 1) / a.zc;
    const long items = tiles * a.zchunks;
    if (items >= (1L << 31)) return hipErrorInvalidValue;
    a.items = (int)items;
    const int grid = (int)(items < grid_max ? items : grid_max);
#define LAUNCH(A, G) hipLaunchKernelGGL((k_wgrad<A, G>), dim3(grid), dim3(kWgBlock), 0, st, a)
    if (ca == 8 && cg == 32) LAUNCH(8, 32);
    else if (ca == 32 && cg == 32) LAUNCH(32, 32);
    else if (ca == 32 && cg == 8) LAUNCH(32, 8);
    else return hipErrorInvalidValue;
#undef LAUNCH
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(28 * 1024 / 16), dim3(kCnnBlock), 0, st, a.part, grid, cin, cout, gw, gb);
    return hipGetLastError();
}

hipError_t cnn_adam(float* p, float* m, float* v, const float* g, int n, float lr, int step, float* clip,
                    hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
    double* part = reinterpret_cast<double*>(clip + 2);
    hipLaunchKernelGGL(k_grad_sq, dim3(kNormBlocks), dim3(kCnnBlock), 0, st, g, n, part);
    hipLaunchKernelGGL(k_grad_clip, dim3(1), dim3(64), 0, st, (const double*)part, clip);
    hipLaunchKernelGGL(k_adam, dim3((n + kCnnBlock - 1) / kCnnBlock), dim3(kCnnBlock), 0, st, p, m, v, g, n, lr, b1, b2,
                       eps, c1, c2, (const float*)clip);
    return hipGetLastError();
}

hipError_t cnn_prep(const float* W, const float* b, int cin, int cout, int cinp, int coutp, uint16_t* wq,
                    uint16_t* wqd, float* bias32, hipStream_t st) {
    const int nb_f = (int)((cnn_wq_elems(cinp) + kCnnBlock - 1) / kCnnBlock);
    const int nb_d = wqd != nullptr ? (int)((cnn_wq_elems(coutp) + kCnnBlock - 1) / kCnnBlock) : 0;
    hipLaunchKernelGGL(k_prep_layer, dim3(nb_f + nb_d + 1), dim3(kCnnBlock), 0, st, W, b, cin, cout, cinp, coutp, wq,
                       wqd, bias32, nb_f, nb_d);
    return hipGetLastError();
}

}  // namespace clampk
