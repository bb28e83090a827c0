// Kernels of the CLAMP forward-model agent, prior and consensus step.
//
// Data flow of one forward-agent application (all looks in every launch):
//   1. column pass, inverse:  resid (compact pupil) -> band rows T
//      (inverse DFT of each band column; only band columns are non-zero)
//   2. row pass "grad":       T -> A^H resid (inverse row DFT), then
//      d = A^H resid / sigma_w^2 - omega mu, then the forward row DFT of d,
//      keeping band columns -> T2; partial sums of ||d||^2, sum omega|d|^2,
//      sum omega|mu|^2
//   3. column pass, forward:  T2 -> D(a) F d (compact); partial ||A d||^2
//   4. gamma:                 exact step size per look, kept on the device
//   5. row pass "update":     recompute d from T, mu += gamma d, and the
//      quadratic-surrogate r-update per voxel
//   6. resid -= gamma D(a) F d on the pupil samples
// Recomputing d in step 5 costs two row FFTs but saves writing and reading
// d (16 bytes per voxel-look); T is only half a slice wide at R = N/4.
#include <math.h>

#include <mutex>

#include "passes.hpp"

namespace clampk {

static int grid_cap(size_t work, int cap) {
    size_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (int)(b < (size_t)cap ? b : (size_t)cap);
}
int resid_blocks(const SceneTables& s) { return grid_cap((size_t)s.nz * s.P, 1 << 20); }
int mace_blocks(size_t n) { return grid_cap(n / 2, 1 << 22); }
int resid_chunks(const SceneTables& s) { return grid_cap((size_t)s.nz * s.P, 512); }

// ---------------------------------------------------------------------------
// Column passes.  A work item is a tile of TC band columns of one slice of one
// look.  The compact pupil layout is column-major (band column by band
// column, rows increasing), so a tile's pupil samples are TC contiguous runs.
//
// Inverse pass from the compact layout: one item per block.
template <int NY>
__global__ __launch_bounds__(kBlock) void k_col_inv_compact(ColArgs a) {
    __shared__ float2 tw[NY];
    __shared__ float2 tile[NY * col_tile_cols(NY)];
    col_inv_item<NY>(a, blockIdx.x, tw, tile, true);
}

// Inverse column passes from full grids (initialisation and the operator's
// adjoint).  Blocks are persistent and walk the items with a stride of the
// grid size; each thread keeps the next item's inputs in registers, loaded
// while the current item's column FFTs run.  Thread (tid / TC, tid % TC)
// loads rows y = tid / TC + k * TPC of column tid % TC; only pupil samples
// are read.
template <int NY, int MODE>
__device__ __forceinline__ void col_dense_inv(const ColArgs& a, float2* tw, float2* tile) {
    constexpr int TC = col_tile_cols(NY);
    constexpr int TPC = kBlock / TC;       // threads per column
    constexpr int PT = NY / TPC;           // values per thread per item
    static_assert(NY % TPC == 0, "column length must be a multiple of the threads per column");
    const SceneTables& s = a.s;
    const int tid = threadIdx.x;
    const int items = a.looks * s.nz * s.tiles;
    for (int i = tid; i < NY; i += kBlock) tw[i] = s.tw_y[i];

    float2 pre[PT];
    double acc_in = 0.0;  // sum |input|^2 of the prefetched item (init loads)

    auto load_item = [&](int item) {
        const int tile_i = item % s.tiles;
        const int zl = item / s.tiles;
        const int c = tid % TC, bc = tile_i * TC + c;
        float f = 0.f;
        const int v = bc < s.B ? s.band_cols[bc] : 0;
        const float2* src = a.full_in + (size_t)zl * s.ny * s.nx;
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int y = tid / TC + k * TPC;
            float2 val = make_float2(0.f, 0.f);
            if (bc < s.B) {
                const int pi = s.pidx[y * s.nx + v];
                if (pi >= 0) {
                    val = src[(size_t)y * s.nx + v];
                    if constexpr (MODE == COL_INV_INIT) {
                        a.cmp_out[(size_t)zl * s.P + pi] = cscale(val, a.init_keep);
                        if (a.cmp_keep != nullptr) a.cmp_keep[(size_t)zl * s.P + pi] = val;
                        f += cabs2(val);
                    }
                }
            }
            pre[k] = val;
        }
        acc_in = f;
    };

    int item = blockIdx.x;
    if (item < items) load_item(item);
    for (; item < items; item += gridDim.x) {
        const int tile_i = item % s.tiles;
        const int zl = item / s.tiles;
        const int c0 = tile_i * TC;
        double acc[1] = {acc_in};
        __syncthreads();  // the previous item's readers of `tile` are done
#pragma unroll
        for (int k = 0; k < PT; ++k) tile[(tid / TC + k * TPC) * TC + tid % TC] = pre[k];
        const int next = item + gridDim.x;
        if (next < items) load_item(next);
        fft_lds<NY, TPC, +1>(tile + tid % TC, TC, tid / TC, tw);
        const int c = tid % TC, bc = c0 + c;
        if (bc < s.B) {
            float2* dst = a.band_out + (size_t)zl * s.ny * s.Bs + (size_t)tile_i * s.ny * TC + c;  // the tile's block
            for (int y = tid / TC; y < NY; y += TPC) dst[(size_t)y * TC] = cscale(tile[y * TC + c], a.scale);
        }
        // item index = (look * nz + z) * tiles + tile = look * col_blocks + z * tiles + tile
        if (a.part != nullptr) block_sum_store<1>(acc, a.part + item);
    }
}

// Persistent dense column passes: the inverse passes from full grids.
template <int NY, int MODE>
__global__ __launch_bounds__(kBlock) void k_col(ColArgs a) {
    __shared__ float2 tw[NY];
    __shared__ float2 tile[NY * col_tile_cols(NY)];
    col_dense_inv<NY, MODE>(a, tw, tile);
}

// Persistent forward column pass from band rows, items pipelined by
// col_fwd_stream.  Three waves per SIMD: the LDS tile allows three or four
// blocks per CU, and the prefetched band rows plus the item's pupil rows
// would otherwise take the register count just past the three-wave limit.
// At 512 (16-column tiles of 64 KB, two blocks per CU) each thread holds 32
// values of an item, and two waves per SIMD is what fits.
template <int NY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NY == 512 ? 2 : 3))) void k_col_fwd(
    ColArgs a) {
    __shared__ float2 tw[NY];
    __shared__ float2 tile[NY * col_tile_cols(NY)];
    for (int i = threadIdx.x; i < NY; i += kBlock) tw[i] = a.s.tw_y[i];
    __syncthreads();
    const ColArgs* ap = &a;
    col_fwd_stream<NY>(blockIdx.x, a.looks * a.s.nz * a.s.tiles, gridDim.x,
                       [ap](int pos) { return ColItemRef{ap, pos}; }, tw, tile);
}

// ---------------------------------------------------------------------------
// Row pass: RPB rows of length NX per block, TR threads per row; block
// (x, y) = (row group, look).
template <int NX, int MODE>
__global__ __launch_bounds__(kBlock) void k_row(RowArgs a) {
    __shared__ float2 tw[NX];
    __shared__ int bpos[NX];
    __shared__ int bcol[NX];
    __shared__ float2 buf[row_lds_floats2<NX>()];
    const RowLds L{tw, bpos, bcol, buf};
    const BetaVals bv{a.beta, a.inv_beta, a.k_up, a.k_dn};
    row_item<NX, MODE>(a, blockIdx.y, blockIdx.x, (size_t)blockIdx.y * gridDim.x + blockIdx.x, L, true, bv);
}

// The gradient row pass as its own kernel, held to six waves per SIMD (its
// LDS allows seven blocks per CU; the register count otherwise allows five).
template <int NX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_row_grad(RowArgs a) {
    __shared__ float2 tw[NX];
    __shared__ int bpos[NX];
    __shared__ int bcol[NX];
    __shared__ float2 buf[row_lds_floats2<NX>()];
    const RowLds L{tw, bpos, bcol, buf};
    const BetaVals bv{a.beta, a.inv_beta, a.k_up, a.k_dn};
    row_item<NX, ROW_GRAD>(a, blockIdx.y, blockIdx.x, (size_t)blockIdx.y * gridDim.x + blockIdx.x, L, true, bv);
}

// The update pass with the Mann step fused in: one block per row group,
// walking every look (row_update_mann).  Held to three waves per SIMD (168
// registers): the per-voxel sums across looks come on top of the update
// pass's registers, and at four waves (128) the compiler spills 25 of them
// to scratch inside the look loop.
template <int NX, int MODE>
__device__ __forceinline__ void row_upd_mann_block(const RowArgs& a, const FuseArgs& f) {
    __shared__ float2 tw[NX];
    __shared__ int bpos[NX];
    __shared__ int bcol[NX];
    __shared__ float2 buf[row_lds_floats2<NX>()];
    __shared__ float ups[64];
    __shared__ float keep[mann_lds_floats<NX>()];
    const RowLds L{tw, bpos, bcol, buf};
    const BetaVals bv{a.beta, a.inv_beta, a.k_up, a.k_dn};
    row_update_mann<NX, MODE>(a, f, blockIdx.x, gridDim.x, L, bv, ups, keep);
}
template <int NX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_row_upd_mann(RowArgs a,
                                                                                                FuseArgs f) {
    row_upd_mann_block<NX, ROW_UPDATE>(a, f);
}
// The exact surrogate prox's float64 root solve needs more registers: two
// waves per SIMD.
template <int NX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_row_upd_mann_exact(
    RowArgs a, FuseArgs f) {
    row_upd_mann_block<NX, ROW_UPDATE_EXACT>(a, f);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_scatter_full(SceneTables s, size_t total,
                                                         const float2* cmp, float2* full) {
    const size_t per = (size_t)s.ny * s.nx;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
        const size_t zl = i / per, pos = i - zl * per;
        const int p = s.pidx[pos];
        full[i] = p >= 0 ? cmp[zl * s.P + p] : make_float2(0.f, 0.f);
    }
}

__global__ __launch_bounds__(kBlock) void k_gamma(GammaArgs a) { gamma_item(blockIdx.x, a); }

__global__ __launch_bounds__(kBlock) void k_resid(size_t per_look, float2* resid, const float2* dfd,
                                                  const double* diag, double* part) {
    const int look = blockIdx.y;
    const float g = (float)diag[(size_t)look * kDiag];
    const float f = resid_range(resid + per_look * look, dfd + per_look * look, g, (size_t)blockIdx.x * kBlock,
                                per_look, (size_t)gridDim.x * kBlock);
    double acc[1] = {f};
    block_sum_store<1>(acc, part + (size_t)look * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_diag_after(DiagArgs a) { diag_after_item(blockIdx.x, a); }

__global__ __launch_bounds__(kBlock) void k_csub(size_t count, const float2* a, const float2* b, float2* out) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock) {
        const float2 x = a[i], y = b[i];
        out[i] = make_float2(x.x - y.x, x.y - y.y);
    }
}

__global__ __launch_bounds__(kBlock) void k_init_r0(size_t n, int looks, float2* mu, float s_mu,
                                                    float* r0, double* part) {
    const float inv_l = 1.f / (float)looks;
    double f = 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        float acc = 0.f;
        for (int l = 0; l < looks; ++l) {
            const float2 b = mu[(size_t)l * n + i];
            acc += cabs2(b);
            mu[(size_t)l * n + i] = cscale(b, s_mu);
        }
        const float r = acc * inv_l;
        r0[i] = r;
        f += r;
    }
    double v[1] = {f};
    block_sum_store<1>(v, part + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_sum(const double* part, int count, double scale, double* out) {
    const int look = blockIdx.x;
    double v[1] = {0.0};
    strided_sums<1>(part + (size_t)look * count, count, 1, v);
    __shared__ double tot[1];
    block_sum_store<1>(v, tot);
    if (threadIdx.x == 0) out[look] = tot[0] * scale;
}

__global__ __launch_bounds__(kBlock) void k_init_floor(size_t n, int n_agents, const double* mean_r0,
                                                       float* r, float* w) {
    const float fl = (float)(1e-12 * mean_r0[0]);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const float v = fmaxf(r[i], fl);
        for (int j = 0; j < n_agents; ++j) {
            r[(size_t)j * n + i] = v;
            w[(size_t)j * n + i] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Mann step: two adjacent voxels per thread, every agent's w and r held in
// registers (NA >= n_agents, a multiple of 4).  Every load is unconditional so
// that all 2 NA of them are in flight at once: the NA - n_agents padding
// agents re-read the last agent, with weight 0 in the averages, and store
// nothing.
template <int NA>
__global__ __launch_bounds__(kBlock) void k_mace(MaceArgs a) {
    const unsigned n = (unsigned)a.n;
    const unsigned n2 = n / 2;
    const int na = a.n_agents;
    double num = 0.0, den = 0.0;
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < n2; i += gridDim.x * kBlock) {
        float2 wv[NA], rv[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const size_t base = (size_t)(j < na ? j : na - 1) * n;
            wv[j] = ld_stream(reinterpret_cast<const float2*>(a.w + base) + i);
            rv[j] = ld_stream(reinterpret_cast<const float2*>(a.r + base) + i);
        }
        float2 wb = make_float2(0.f, 0.f), rb = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const float u = a.ups[j];
            wb.x += u * wv[j].x;
            wb.y += u * wv[j].y;
            rb.x += u * rv[j].x;
            rb.y += u * rv[j].y;
        }
        const float2 xb = make_float2(2.f * rb.x - wb.x, 2.f * rb.y - wb.y);
        float2 wbn = make_float2(0.f, 0.f);
        float nm = 0.f;
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            if (j < na) {
                const float dx = rv[j].x - wb.x, dy = rv[j].y - wb.y;
                nm += dx * dx + dy * dy;
                const float2 wn = make_float2(wv[j].x + a.two_rho * (xb.x - rv[j].x),
                                              wv[j].y + a.two_rho * (xb.y - rv[j].y));
                st_stream(reinterpret_cast<float2*>(a.w + (size_t)j * n) + i, wn);
                const float u = a.ups[j];
                wbn.x += u * wn.x;
                wbn.y += u * wn.y;
            }
        }
        st_stream(reinterpret_cast<float2*>(a.wbar) + i, wbn);
        num += nm;
        den += (double)na * ((double)wb.x * wb.x + (double)wb.y * wb.y);
    }
    double v[2] = {num, den};
    block_sum_store<2>(v, a.part + (size_t)blockIdx.x * 2);
}

// Mann state from the fused pass's representation: out_l = u_l + 2 rho xbar
// for the looks, out_L = w_L (the prior agent's, kept whole).
__global__ __launch_bounds__(kBlock) void k_mann_state(size_t n, int looks, int n_agents, float two_rho,
                                                       const float* u, const float* xbar, float* out) {
    const size_t total = n * (size_t)n_agents;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
        const size_t j = i / n, v = i - j * n;
        out[i] = (int)j < looks ? u[i] + two_rho * xbar[v] : u[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_mace_final(const double* part, int blocks, double* conv) {
    double v[2] = {0.0, 0.0};
    strided_sums<2>(part, blocks, 2, v);
    __shared__ double tot[2];
    block_sum_store<2>(v, tot);
    if (threadIdx.x == 0) conv[0] = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : 0.0;
}

// ---------------------------------------------------------------------------
// The periodic separable 7-tap smoothing of a volume in one pass, one block
// per output tile (gauss3d_tile).  Each input element is fetched about
// (GTY + 6)(TX + 6)/(GTY TX) (GCZ + 6)/GCZ times and the output written
// once, where three separate passes read and write the volume three times.
// (Dealing the tiles to the eight XCDs in contiguous runs, so that
// neighbouring tiles share an L2, measured 1-2 us slower at 256x256x64.)
template <int TX>
__global__ __launch_bounds__(kBlock) void k_gauss3d(PriorArgs p) {
    __shared__ float tin[gauss_in_floats<TX>()];
    __shared__ float txf[gauss_xf_floats<TX>()];
    gauss3d_tile<TX>(p, blockIdx.x, tin, txf);
}

// ---------------------------------------------------------------------------
// Launchers
#define CLAMP_SIZES(X) X(32) X(64) X(128) X(192) X(256) X(384) X(512)

static int g_col_grid_cap = 0;

// Persistent grid of the column pass: enough blocks for every CU to hold as
// many items as its LDS allows, never more blocks than items.
static int col_grid(size_t items) {
    if (g_col_grid_cap == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g_col_grid_cap = cus * 8;
    }
    return (int)(items < (size_t)g_col_grid_cap ? items : (size_t)g_col_grid_cap);
}

template <int MODE>
static hipError_t col_dispatch(const ColArgs& a, hipStream_t st) {
    const size_t items = (size_t)a.looks * a.s.nz * a.s.tiles;
    const dim3 grid((unsigned)(MODE == COL_INV_COMPACT ? items : col_grid(items)));
    switch (a.s.ny) {
#define CASE(N)                                                                          \
    case N:                                                                              \
        if constexpr (MODE == COL_INV_COMPACT)                                           \
            hipLaunchKernelGGL((k_col_inv_compact<N>), grid, dim3(kBlock), 0, st, a);    \
        else if constexpr (MODE == COL_FWD_COMPACT)                                      \
            hipLaunchKernelGGL((k_col_fwd<N>), grid, dim3(kBlock), 0, st, a);            \
        else                                                                             \
            hipLaunchKernelGGL((k_col<N, MODE>), grid, dim3(kBlock), 0, st, a);          \
        break;
        CLAMP_SIZES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_col(int mode, const ColArgs& a, hipStream_t st) {
    if (a.looks <= 0) return hipSuccess;
    switch (mode) {
        case COL_INV_COMPACT: return col_dispatch<COL_INV_COMPACT>(a, st);
        case COL_INV_FULL: return col_dispatch<COL_INV_FULL>(a, st);
        case COL_INV_INIT: return col_dispatch<COL_INV_INIT>(a, st);
        case COL_FWD_COMPACT: return col_dispatch<COL_FWD_COMPACT>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t row_dispatch(const RowArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)row_blocks(a.s), (unsigned)a.looks);
    switch (a.s.nx) {
#define CASE(N)                                                                  \
    case N:                                                                      \
        if constexpr (MODE == ROW_GRAD)                                          \
            hipLaunchKernelGGL((k_row_grad<N>), grid, dim3(kBlock), 0, st, a);   \
        else                                                                     \
            hipLaunchKernelGGL((k_row<N, MODE>), grid, dim3(kBlock), 0, st, a);  \
        break;
        CLAMP_SIZES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row(int mode, const RowArgs& a, hipStream_t st) {
    if (a.looks <= 0) return hipSuccess;
    switch (mode) {
        case ROW_INV: return row_dispatch<ROW_INV>(a, st);
        case ROW_FWD: return row_dispatch<ROW_FWD>(a, st);
        case ROW_GRAD: return row_dispatch<ROW_GRAD>(a, st);
        case ROW_UPDATE: return row_dispatch<ROW_UPDATE>(a, st);
        case ROW_UPDATE_EXACT: return row_dispatch<ROW_UPDATE_EXACT>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t row_update_mann_dispatch(const RowArgs& a, const FuseArgs& f, hipStream_t st) {
    const dim3 grid((unsigned)row_blocks(a.s));
    switch (a.s.nx) {
#define CASE(N)                                                                          \
    case N:                                                                              \
        if constexpr (MODE == ROW_UPDATE_EXACT)                                          \
            hipLaunchKernelGGL((k_row_upd_mann_exact<N>), grid, dim3(kBlock), 0, st, a, f); \
        else                                                                             \
            hipLaunchKernelGGL((k_row_upd_mann<N>), grid, dim3(kBlock), 0, st, a, f);    \
        break;
        CLAMP_SIZES(CASE)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row_update_mann(int mode, const RowArgs& a, const FuseArgs& f, hipStream_t st) {
    if (a.looks <= 0) return hipSuccess;
    switch (mode) {
        case ROW_UPDATE: return row_update_mann_dispatch<ROW_UPDATE>(a, f, st);
        case ROW_UPDATE_EXACT: return row_update_mann_dispatch<ROW_UPDATE_EXACT>(a, f, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scatter_full(const SceneTables& s, int looks, const float2* cmp, float2* full,
                               hipStream_t st) {
    const size_t total = (size_t)looks * s.nz * s.ny * s.nx;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_full, dim3(grid_cap(total, 8192)), dim3(kBlock), 0, st, s, total, cmp, full);
    return hipGetLastError();
}

hipError_t launch_gamma(const SceneTables& s, int looks, const double* part_row, const double* part_colfwd,
                          const double* part_colinv, double inv_s2w, double* diag, uint32_t* fault,
                          unsigned* counter, hipStream_t st) {
    // with the 3D operator the column-side sums come from the range passes
    const int ncol = s.K > 0 ? zpass_blocks(s) : col_blocks(s);
    const GammaArgs a{row_blocks(s), ncol, part_row, part_colfwd, part_colinv, inv_s2w, diag, fault, counter};
    hipLaunchKernelGGL(k_gamma, dim3(looks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_resid_update(const SceneTables& s, int looks, float2* resid, const float2* dfd,
                               const double* diag, double* part, hipStream_t st) {
    const size_t per_look = (size_t)(s.K > 0 ? s.K : s.nz) * s.P;  // box [K][P] with the 3D operator
    hipLaunchKernelGGL(k_resid, dim3(resid_blocks(s), looks), dim3(kBlock), 0, st, per_look, resid, dfd, diag,
                       part);
    return hipGetLastError();
}

hipError_t launch_diag_after(const SceneTables& s, int looks, const double* pupd, const double* pres,
                             double s2w, const double* ahy2, double* diag, unsigned* counter, hipStream_t st) {
    const DiagArgs a{row_blocks(s), resid_blocks(s), looks, pupd, pres, s2w, ahy2, diag, counter};
    hipLaunchKernelGGL(k_diag_after, dim3(looks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_csub(size_t count, const float2* a, const float2* b, float2* out, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_csub, dim3(grid_cap(count, 8192)), dim3(kBlock), 0, st, count, a, b, out);
    return hipGetLastError();
}

hipError_t launch_init_r0(size_t n, int looks, float2* mu, float s_mu, float* r0, double* part,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_init_r0, dim3(mace_blocks(n)), dim3(kBlock), 0, st, n, looks, mu, s_mu, r0, part);
    return hipGetLastError();
}

hipError_t launch_sum(const double* part, int count, int looks, double scale, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum, dim3(looks), dim3(kBlock), 0, st, part, count, scale, out);
    return hipGetLastError();
}

hipError_t launch_init_floor(size_t n, int n_agents, const double* mean_r0, float* r, float* w,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_init_floor, dim3(mace_blocks(n)), dim3(kBlock), 0, st, n, n_agents, mean_r0, r, w);
    return hipGetLastError();
}

hipError_t launch_mace(const MaceArgs& a, hipStream_t st) {
    if (a.n % 2 != 0 || a.n_agents < 1) return hipErrorInvalidValue;
    const dim3 grid(mace_blocks(a.n));
    switch ((a.n_agents + 3) / 4) {
#define CASE(K)                                                              \
    case K:                                                                  \
        hipLaunchKernelGGL(k_mace<4 * K>, grid, dim3(kBlock), 0, st, a);     \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mann_state(size_t n, int looks, int n_agents, float two_rho, const float* u, const float* xbar,
                             float* out, hipStream_t st) {
    const size_t total = n * (size_t)n_agents;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mann_state, dim3(grid_cap(total, 8192)), dim3(kBlock), 0, st, n, looks, n_agents, two_rho,
                       u, xbar, out);
    return hipGetLastError();
}

hipError_t launch_mace_final(const double* part, int blocks, double* conv_err, hipStream_t st) {
    hipLaunchKernelGGL(k_mace_final, dim3(1), dim3(kBlock), 0, st, part, blocks, conv_err);
    return hipGetLastError();
}

// Scratch of the Mann step's entry point that allocates nothing: the block
// partial sums of the convergence error, two doubles per block, in a
// file-scope device array that every device holding the library keeps until
// the process ends.  Host code never passes the array's name to a kernel:
// its device address is resolved once per device with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kMaceScratchDoubles];

hipError_t mace_scratch(int device, double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static double* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (addr[device] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_gauss(int nx, int ny, int nz, const float* taps7, const float* in, float* out, hipStream_t st) {
    PriorArgs p{};
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    for (int k = 0; k < 7; ++k) p.g[k] = taps7[k];
    p.in = in;
    p.out = out;
    if (ny % kGaussTY != 0 || nx % 32 != 0) return hipErrorInvalidValue;
    if (nx % 64 == 0)
        hipLaunchKernelGGL(k_gauss3d<64>, dim3(gauss_tiles<64>(nx, ny, nz)), dim3(kBlock), 0, st, p);
    else
        hipLaunchKernelGGL(k_gauss3d<32>, dim3(gauss_tiles<32>(nx, ny, nz)), dim3(kBlock), 0, st, p);
    return hipGetLastError();
}

}  // namespace clampk
