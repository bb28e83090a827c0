// Batched passes: every stage of a CLAMP iteration over many scenes of
// uneven size and look count, as persistent launches over device queues of
// work items (scene, look, row group or column tile).  The FFT passes launch
// once per FFT length present in the batch, each kernel compiled for its
// length so that registers and LDS match the single-scene kernels; the other
// stages launch once for all scenes.  The interval factor beta of the
// surrogate r-update comes from a device table indexed by a device iteration
// counter, so one iteration has no host-side arguments that change and can be
// captured once in a HIP graph and replayed.
#include "passes.hpp"

namespace clampk {

#define CLAMP_SIZES(X) X(32) X(64) X(128) X(192) X(256) X(384) X(512)

// Row pass over the segment [off, off + count) of the row queue, whose items
// all have row length NX.  PERSIST: a capped grid whose blocks walk the
// segment; otherwise one block per item, which keeps the item loop's
// hoisted values out of the registers (85 against 106 at NX = 256); held to
// six waves per SIMD there, as the single-scene row kernels run (79
// registers, no spills up to NX = 256).
template <int NX, int MODE, bool PERSIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(!PERSIST && NX <= 256 ? 6 : 1))) void kb_row(
    BatchLaunch b, int off, int count) {
    __shared__ float2 tw[NX];
    __shared__ int bpos[NX];
    __shared__ int bcol[NX];
    __shared__ float2 buf[row_lds_floats2<NX>()];
    const RowLds L{tw, bpos, bcol, buf};
    BetaVals bv{1.f, 1.f, 1.f, 1.f};
    if constexpr (MODE == ROW_UPDATE) {
        const int k = *b.iter;
        bv = beta_vals(b.beta_table[k < b.beta_len ? k : b.beta_len - 1]);
    }
    const BatchItem* q = b.queue[Q_ROW] + off;
    if constexpr (!PERSIST) {
        const BatchItem w = const_ref(q + blockIdx.x);
        // the scene's arguments stay in the (read-only) table, read by scalar loads
        const auto& a = const_ref((MODE == ROW_GRAD) ? &b.scenes[w.scene].grad : &b.scenes[w.scene].update);
        row_item<NX, MODE>(a, w.a, w.b, (size_t)w.a * row_blocks(a.s) + w.b, L, true, bv);
    } else {
        int prev = -1;
        for (int it = blockIdx.x; it < count; it += gridDim.x) {
            const BatchItem w = const_ref(q + it);
            const auto& a = const_ref((MODE == ROW_GRAD) ? &b.scenes[w.scene].grad : &b.scenes[w.scene].update);
            const bool load = w.scene != prev;
            prev = w.scene;
            row_item<NX, MODE>(a, w.a, w.b, (size_t)w.a * row_blocks(a.s) + w.b, L, load, bv);
        }
    }
}

// The update pass with the Mann step fused in, one block per row-group item
// (scene, row group) of the segment starting at `off`, walking every look of
// the scene (row_update_mann); three waves per SIMD, as the single-scene
// kernel.
template <int NX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void kb_row_mann(BatchLaunch b,
                                                                                              int off) {
    __shared__ float2 tw[NX];
    __shared__ int bpos[NX];
    __shared__ int bcol[NX];
    __shared__ float2 buf[row_lds_floats2<NX>()];
    __shared__ float ups[64];
    __shared__ float keep[mann_lds_floats<NX>()];
    const RowLds L{tw, bpos, bcol, buf};
    const int k = *b.iter;
    const BetaVals bv = beta_vals(b.beta_table[k < b.beta_len ? k : b.beta_len - 1]);
    const BatchItem w = const_ref(b.queue[Q_ROWG] + off + blockIdx.x);
    const auto& a = const_ref(&b.scenes[w.scene].update);
    const auto& f = const_ref(&b.scenes[w.scene].fuse);
    row_update_mann<NX, ROW_UPDATE>(a, f, w.b, row_blocks(a.s), L, bv, ups, keep);
}

// Column pass over the segment [off, off + count) of the column queue, whose
// items all have column length NY.
template <int NY, bool FWD>
__global__ __launch_bounds__(kBlock) void kb_col(BatchLaunch b, int off, int count) {
    __shared__ float2 tw[NY];
    __shared__ float2 tile[NY * col_tile_cols(NY)];
    const BatchItem* q = b.queue[Q_COL] + off;
    if constexpr (FWD) {
        // every item of the segment has column length NY: one twiddle table,
        // and the next item's band rows load during the current FFTs
        for (int i = threadIdx.x; i < NY; i += kBlock) tw[i] = b.scenes[q[0].scene].cfwd.s.tw_y[i];
        __syncthreads();
        const SceneBatch* scenes = b.scenes;
        col_fwd_stream<NY>(blockIdx.x, count, gridDim.x, [scenes, q](int pos) {
            const BatchItem w = const_ref(q + pos);
            return ColItemConst{&const_ref(&scenes[w.scene].cfwd), w.a};
        }, tw, tile);
    } else {
        int prev = -1;
        for (int it = blockIdx.x; it < count; it += gridDim.x) {
            const BatchItem w = const_ref(q + it);
            const bool load = w.scene != prev;
            prev = w.scene;
            col_inv_item<NY>(const_ref(&b.scenes[w.scene].cinv), w.a, tw, tile, load);
        }
    }
}

__global__ __launch_bounds__(kBlock) void kb_gamma(BatchLaunch b) {
    const BatchItem* q = b.queue[Q_LOOK];
    for (int it = blockIdx.x; it < b.count[Q_LOOK]; it += gridDim.x) {
        const BatchItem w = q[it];
        const GammaArgs g = load_uniform(&b.scenes[w.scene].gam);
        gamma_item(w.a, g);
    }
}

__global__ __launch_bounds__(kBlock) void kb_resid(BatchLaunch b) {
    const BatchItem* q = b.queue[Q_RESID];
    for (int it = blockIdx.x; it < b.count[Q_RESID]; it += gridDim.x) {
        const BatchItem w = q[it];
        const ResidArgs r = load_uniform(&b.scenes[w.scene].res);
        const float g = (float)r.diag[(size_t)w.a * kDiag];
        const float f = resid_range(r.resid + r.per_look * w.a, r.dfd + r.per_look * w.a, g, (size_t)w.b * kBlock,
                                    r.per_look, (size_t)r.chunks * kBlock);
        double acc[1] = {f};
        block_sum_store<1>(acc, r.part + (size_t)w.a * r.chunks + w.b);
    }
}

__global__ __launch_bounds__(kBlock) void kb_diag(BatchLaunch b) {
    const BatchItem* q = b.queue[Q_LOOK];
    for (int it = blockIdx.x; it < b.count[Q_LOOK]; it += gridDim.x) {
        const BatchItem w = q[it];
        const DiagArgs d = load_uniform(&b.scenes[w.scene].dia);
        diag_after_item(w.a, d);
    }
}

// Mann step: one voxel per thread, agents held in registers (at most 40).
__global__ __launch_bounds__(kBlock) void kb_mace(BatchLaunch b) {
    const BatchItem* q = b.queue[Q_VOX];
    for (int it = blockIdx.x; it < b.count[Q_VOX]; it += gridDim.x) {
        const BatchItem w = q[it];
        const MaceArgs& mg = b.scenes[w.scene].mace;
        MaceArgs m;  // everything but the weights, in scalar registers
        m.n = __builtin_amdgcn_readfirstlane((int)mg.n);
        m.n_agents = __builtin_amdgcn_readfirstlane(mg.n_agents);
        m.two_rho = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(mg.two_rho)));
        m.w = load_uniform(&mg.w);
        m.r = load_uniform(&mg.r);
        m.wbar = load_uniform(&mg.wbar);
        m.part = load_uniform(&mg.part);
        float ups[40];
#pragma unroll
        for (int j = 0; j < 40; ++j) ups[j] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(mg.ups[j])));
        const unsigned n = (unsigned)m.n;
        const unsigned stride = (unsigned)__builtin_amdgcn_readfirstlane(b.scenes[w.scene].mace_chunks) * kBlock;
        double num = 0.0, den = 0.0;
        switch ((m.n_agents + 7) / 8) {
#define CASE(K)                                                                      \
    case K:                                                                          \
        for (unsigned i = (unsigned)w.b * kBlock + threadIdx.x; i < n; i += stride)  \
            mace_voxel<8 * K>(m, ups, n, i, num, den);                               \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5)
#undef CASE
            default:
                break;
        }
        double v[2] = {num, den};
        block_sum_store<2>(v, m.part + (size_t)w.b * 2);
    }
}

__global__ __launch_bounds__(kBlock) void kb_mace_final(BatchLaunch b) {
    const BatchItem* q = b.queue[Q_SCENE];
    for (int it = blockIdx.x; it < b.count[Q_SCENE]; it += gridDim.x) {
        const SceneBatch& sb = b.scenes[q[it].scene];
        double v[2] = {0.0, 0.0};
        strided_sums<2>(sb.mace.part, sb.mace_chunks, 2, v);
        __shared__ double tot[2];
        block_sum_store<2>(v, tot);
        if (threadIdx.x == 0) sb.conv[0] = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : 0.0;
    }
}

__global__ void kb_set_iter(int* iter, int value, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) iter[0] = add ? iter[0] + value : value;
}

// Gaussian prior agents: one block per output tile (scene, tile) of the
// scenes whose nx is a multiple of TX (gauss3d_tile).
template <int TX>
__global__ __launch_bounds__(kBlock) void kb_gauss3d(BatchLaunch b) {
    __shared__ float tin[gauss_in_floats<TX>()];
    __shared__ float txf[gauss_xf_floats<TX>()];
    const BatchItem w = const_ref(b.queue[TX == 64 ? Q_PRIOR64 : Q_PRIOR32] + blockIdx.x);
    gauss3d_tile<TX>(const_ref(&b.scenes[w.scene].prior), w.b, tin, txf);
}

hipError_t batch_set_iter(int* iter, int value, hipStream_t st) {
    hipLaunchKernelGGL(kb_set_iter, dim3(1), dim3(64), 0, st, iter, value, 0);
    return hipGetLastError();
}

template <int MODE>
static void launch_row_segments(const BatchLaunch& b, hipStream_t st) {
    for (int g = 0; g < b.nseg[0]; ++g) {
        const dim3 grid(b.seg_grid[0][g]);
        const int off = b.seg_off[0][g], cnt = b.seg_count[0][g];
        const bool per_item = b.seg_grid[0][g] >= cnt;
        switch (b.seg_len[0][g]) {
#define CASE(N)                                                                                   \
    case N:                                                                                       \
        if (per_item)                                                                             \
            hipLaunchKernelGGL((kb_row<N, MODE, false>), dim3(cnt), dim3(kBlock), 0, st, b, off, cnt); \
        else                                                                                      \
            hipLaunchKernelGGL((kb_row<N, MODE, true>), grid, dim3(kBlock), 0, st, b, off, cnt);   \
        break;
            CLAMP_SIZES(CASE)
#undef CASE
            default:
                break;
        }
    }
}

static void launch_rowg_segments(const BatchLaunch& b, hipStream_t st) {
    for (int g = 0; g < b.nseg[2]; ++g) {
        const int off = b.seg_off[2][g], cnt = b.seg_count[2][g];
        switch (b.seg_len[2][g]) {
#define CASE(N)                                                                            \
    case N:                                                                                \
        hipLaunchKernelGGL((kb_row_mann<N>), dim3(cnt), dim3(kBlock), 0, st, b, off);      \
        break;
            CLAMP_SIZES(CASE)
#undef CASE
            default:
                break;
        }
    }
}

template <bool FWD>
static void launch_col_segments(const BatchLaunch& b, hipStream_t st) {
    for (int g = 0; g < b.nseg[1]; ++g) {
        const dim3 grid(b.seg_grid[1][g]);
        const int off = b.seg_off[1][g], cnt = b.seg_count[1][g];
        switch (b.seg_len[1][g]) {
#define CASE(N)                                                                       \
    case N:                                                                           \
        hipLaunchKernelGGL((kb_col<N, FWD>), grid, dim3(kBlock), 0, st, b, off, cnt); \
        break;
            CLAMP_SIZES(CASE)
#undef CASE
            default:
                break;
        }
    }
}

hipError_t batch_stage(int stage, const BatchLaunch& b, hipStream_t st) {
    auto go = [&](int qi, auto kernel) {
        if (b.count[qi] > 0) hipLaunchKernelGGL(kernel, dim3(b.grid[qi]), dim3(kBlock), 0, st, b);
    };
    switch (stage) {
        case BS_COL_INV: launch_col_segments<false>(b, st); break;
        case BS_ROW_GRAD: launch_row_segments<ROW_GRAD>(b, st); break;
        case BS_COL_FWD: launch_col_segments<true>(b, st); break;
        case BS_GAMMA: go(Q_LOOK, kb_gamma); break;
        case BS_ROW_UPDATE: launch_row_segments<ROW_UPDATE>(b, st); break;
        case BS_RESID: go(Q_RESID, kb_resid); break;
        case BS_DIAG: go(Q_LOOK, kb_diag); break;
        case BS_PRIOR:
            go(Q_PRIOR64, kb_gauss3d<64>);
            go(Q_PRIOR32, kb_gauss3d<32>);
            break;
        case BS_ROW_UPDATE_MANN: launch_rowg_segments(b, st); break;
        case BS_MACE: go(Q_VOX, kb_mace); break;
        case BS_MACE_FINAL: go(Q_SCENE, kb_mace_final); break;
        case BS_NEXT_ITER: hipLaunchKernelGGL(kb_set_iter, dim3(1), dim3(64), 0, st, b.iter, 1, 1); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace clampk
