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

__host__ __device__ inline size_t strided_units(int len, size_t outer) {
    const int ch = len >= 32 ? 32 : 8;
    return outer * (size_t)((len + ch - 1) / ch);
}
int prior_strided_units(int len, size_t outer) { return (int)strided_units(len, outer); }

// Row pass over the segment [off, off + count) of the row queue, whose items
// all have row length NX.
template <int NX, int MODE>
__global__ __launch_bounds__(kBlock) void kb_row(BatchLaunch b, int off, int count) {
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
    int prev = -1;
    for (int it = blockIdx.x; it < count; it += gridDim.x) {
        const BatchItem w = q[it];
        // a private copy: the item's stores cannot alias its arguments
        const RowArgs a = load_uniform((MODE == ROW_GRAD) ? &b.scenes[w.scene].grad : &b.scenes[w.scene].update);
        const bool load = w.scene != prev;
        prev = w.scene;
        row_item<NX, MODE>(a, w.a, w.b, (size_t)w.a * row_blocks(a.s) + w.b, L, load, bv);
    }
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
            const BatchItem w = q[pos];
            return ColItemVal{load_uniform(&scenes[w.scene].cfwd), w.a};
        }, tw, tile);
    } else {
        int prev = -1;
        for (int it = blockIdx.x; it < count; it += gridDim.x) {
            const BatchItem w = q[it];
            const bool load = w.scene != prev;
            prev = w.scene;
            const ColArgs a = load_uniform(&b.scenes[w.scene].cinv);
            col_inv_item<NY>(a, w.a, tw, tile, load);
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

template <int AXIS>
__global__ __launch_bounds__(kBlock) void kb_prior(BatchLaunch b) {
    constexpr int Q = AXIS == 0 ? Q_PRIOR_X : AXIS == 1 ? Q_PRIOR_Y : Q_PRIOR_Z;
    const BatchItem* q = b.queue[Q];
    for (int it = blockIdx.x; it < b.count[Q]; it += gridDim.x) {
        const BatchItem w = q[it];
        const PriorArgs p = load_uniform(&b.scenes[w.scene].prior);
        const size_t n = (size_t)p.nx * p.ny * p.nz;
        const size_t begin = (size_t)w.b * kPriorChunk;
        if constexpr (AXIS == 0) {
            const size_t end = begin + kPriorChunk < n ? begin + kPriorChunk : n;
            for (size_t i = begin + threadIdx.x; i < end; i += kBlock) p.tmp0[i] = gauss_x_voxel(p.nx, p.g, p.in, i);
        } else {
            const int len = AXIS == 1 ? p.ny : p.nz;
            const size_t inner = AXIS == 1 ? (size_t)p.nx : (size_t)p.nx * p.ny;
            const size_t outer = AXIS == 1 ? (size_t)p.nz * p.nx : (size_t)p.nx * p.ny;
            const float* in = AXIS == 1 ? p.tmp0 : p.tmp1;
            float* out = AXIS == 1 ? p.tmp1 : p.out;
            const size_t units = strided_units(len, outer);
            const size_t end = begin + kPriorChunk < units ? begin + kPriorChunk : units;
            for (size_t u = begin + threadIdx.x; u < end; u += kBlock) {
                if (len >= 32)
                    gauss_strided_unit<32>(len, inner, outer, p.g, in, out, u);
                else
                    gauss_strided_unit<8>(len, inner, outer, p.g, in, out, u);
            }
        }
    }
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
        switch (b.seg_len[0][g]) {
#define CASE(N)                                                                        \
    case N:                                                                            \
        hipLaunchKernelGGL((kb_row<N, MODE>), grid, dim3(kBlock), 0, st, b, off, cnt); \
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
            go(Q_PRIOR_X, kb_prior<0>);
            go(Q_PRIOR_Y, kb_prior<1>);
            go(Q_PRIOR_Z, kb_prior<2>);
            break;
        case BS_MACE: go(Q_VOX, kb_mace); break;
        case BS_MACE_FINAL: go(Q_SCENE, kb_mace_final); break;
        case BS_NEXT_ITER: hipLaunchKernelGGL(kb_set_iter, dim3(1), dim3(64), 0, st, b.iter, 1, 1); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace clampk
