// Internal interface between the C ABI layer (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace clampk {

constexpr int kBlock = 256;      // threads per block for every kernel

// Band columns per column tile: 16, except 8 for 384-row columns, where a
// 16-column tile takes the forward column pass past its registers (spills).
// At 512, 16 columns give the row passes 128-byte runs per tile row (8 gave
// 64-byte runs, 3-7% slower update and gradient passes), while the column
// passes hold two blocks per CU instead of four at about the same time.
__host__ __device__ constexpr int col_tile_cols(int ny) { return ny == 384 ? 8 : 16; }

// Band buffers (the column transforms of a slice kept only on its B band
// columns) hold each (look, slice) as ny Bs values, Bs = tiles TC with
// TC = col_tile_cols(ny): column tile after column tile, each tile row-major
// (TC values per row), so that a column pass moves a tile as one contiguous
// block and a row pass touches TC consecutive values per tile.  In-slice
// offsets of band column b and of row y (TC is 8 or 16: shifts):
__host__ __device__ inline int band_col_off(int b, int ny) {
    const int sh = col_tile_cols(ny) == 8 ? 3 : 4;
    return ((b >> sh) * ny << sh) + (b & ((1 << sh) - 1));
}
__host__ __device__ inline int band_row_off(int y, int ny) { return y * col_tile_cols(ny); }
constexpr int kDiag = 8;         // doubles of diagnostics per look (and of the summary row)
// diag[l][.] of look l: gamma, ||d||^2, ||A d||^2, h before, h after,
// mu-residual of the look, sum omega |d|^2, ||resid||^2 after; summary row
// diag[L][.]: mu-residual averaged over looks, sum of h before, sum of h after.
enum DiagSlot { DG_GAMMA = 0, DG_DD, DG_AD, DG_H0, DG_H1, DG_MURES, DG_WD, DG_R2 };

// Device tables of one scene (owned by the plan).
struct SceneTables {
    int nx, ny, nz;
    int P;       // pupil samples per slice
    int B;       // band columns (columns holding pupil samples)
    int Bs;      // band-buffer values per slice row: tiles * col_tile_cols(ny)
    int tiles;   // ceil(B / col_tile_cols(ny))
    const float2* tw_x;     // [nx] exp(-2 pi i m / nx)
    const float2* tw_y;     // [ny]
    const int* band_cols;   // [B] natural column index of each band column
    const int* band_pos;    // [nx] in-slice band-buffer offset of a column's band sample (band_col_off), -1 outside the band
    const int* col_off;     // [B + 1] compact offset of each band column
    const int* row_idx;     // [P] row of each compact entry
    const int* pidx;        // [ny * nx] compact index of a sample, -1 off-pupil
    const int* pidxb;       // [ny * Bs] compact index of row y of band column b at y * Bs + b, -1 off-pupil
    int K;                  // range frequencies of the 3D aperture (0: per-slice 2D operator)
    const float2* tw_z;     // [nz] (3D operator only)
    const int* cpos;        // [P] u * nx + v of each compact entry (3D operator only)
};

// Range lengths of the 3D operator's range pass.
#define CLAMP_RANGE_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256)
__host__ __device__ constexpr bool range_size_ok(int n) {
    return n == 16 || n == 32 || n == 48 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256;
}

// Range pass of the 3D operator (range.hip): dir +1 inverse (box [K][P] ->
// [nz][P], part = sum |in|^2), -1 forward ([nz][P] -> box, part = sum |out|^2);
// part has zpass_blocks(s) entries per look.
struct ZArgs {
    SceneTables s;
    int looks;
    const float2* in;
    float2* out;
    double* part;
};
int zpass_blocks(const SceneTables& s);
int gather_blocks(const SceneTables& s);
hipError_t launch_zpass(int dir, const ZArgs& a, hipStream_t st);
// out[l][k][p] = y[l][w_k][pupil position p] (and keep times that into
// out_keep if non-null); part has gather_blocks(s) entries per look.
hipError_t launch_range_gather(const SceneTables& s, int looks, const float2* y, float2* out, float2* out_keep,
                               float keep, double* part, hipStream_t st);
// Full 3D frequency grids from box data (zero off the support).
hipError_t launch_range_scatter(const SceneTables& s, int looks, const float2* cmp, float2* full, hipStream_t st);

// Threads per row of a row-pass block (the power of two >= n/8) and rows per
// block.
__host__ __device__ constexpr int row_threads(int n) {
    int t = 4;
    while (t * 8 < n) t *= 2;
    return t;
}
__host__ __device__ constexpr int rows_per_block(int n) { return kBlock / row_threads(n); }

// Number of partial-sum blocks per look of each pass.
__host__ __device__ inline int row_blocks(const SceneTables& s) {
    const int rpb = rows_per_block(s.nx);
    return (s.nz * s.ny + rpb - 1) / rpb;
}
__host__ __device__ inline int col_blocks(const SceneTables& s) { return s.nz * s.tiles; }
// Launches of the residual update and the Mann step take one element (pair)
// per thread: many short blocks stream HBM faster on this chip than a capped
// grid that loops.  The batched Mann step uses the same work items; the
// batched residual update keeps fewer, longer ones (resid_chunks <=
// resid_blocks, which sizes the partial-sum workspace), measured faster there.
int resid_blocks(const SceneTables& s);
int mace_blocks(size_t n);
int resid_chunks(const SceneTables& s);

enum ColMode { COL_INV_COMPACT = 0, COL_INV_FULL = 1, COL_INV_INIT = 2, COL_FWD_COMPACT = 3 };
enum RowMode { ROW_INV = 0, ROW_FWD = 1, ROW_GRAD = 2, ROW_UPDATE = 3, ROW_UPDATE_EXACT = 4 };

struct ColArgs {
    SceneTables s;
    int looks;                 // looks in this launch
    const float2* cmp_in;      // compact [looks][nz][P]      (COL_INV_COMPACT)
    const float2* full_in;     // full grids [looks][nz][ny][nx] (COL_INV_FULL/INIT)
    const float2* band_in;     // band buffers [looks][nz][ny * Bs] (COL_FWD_COMPACT)
    float2* band_out;          // band rows                      (COL_INV_*)
    float2* cmp_out;           // compact out: D(a)F x (FWD), (1 - s) D(a) y (INIT)
    float2* cmp_keep;          // compact out: D(a) y (INIT, optional)
    double* part;              // [looks][col_blocks] sum of |input or output|^2
    float scale;               // 1/sqrt(ny)
    float init_keep;           // 1 - s_mu (COL_INV_INIT)
};

struct RowArgs {
    SceneTables s;
    int looks;
    const float2* band_in;     // band rows in (INV, GRAD, UPDATE)
    float2* band_out;          // band rows out (FWD, GRAD)
    const float2* img_in;      // images in (FWD)
    float2* img_out;           // images out (INV)
    float2* mu;                // [looks][n]
    float* r;                  // [looks][n] anchors in, outputs out (UPDATE)
    const float* w;            // [looks][n] (UPDATE)
    const double* diag;        // [looks][8], gamma in slot 0 (UPDATE)
    double* part;              // GRAD: 3 per block, UPDATE: 1 per block
    uint32_t* fault;
    float scale;               // 1/sqrt(nx)
    float inv_s2w;             // 1/sigma_w^2
    float s2w;                 // sigma_w^2
    float floor_w;             // sigma_w^2/alpha
    float alpha;
    float sigma2;
    float inv_sigma2;
    float beta, inv_beta;
    float k_up;                // (1 + beta)/beta^2      (xi = beta r')
    float k_dn;                // beta (1 + beta)        (xi = r'/beta)
};

// The Mann step fused into the update pass (one block walks every look of
// its rows).  The forward agents' Mann state is kept as u_l = w_l - 2 rho
// xbar with xbar the reflected average x_bar of the previous step, so that
// the pass never re-reads a look: it forms v = u_l + 2 rho xbar_old, writes
// u_l' = v - 2 rho r_l, and after the last look xbar_new, w_bar and the prior
// agent's w (kept whole).
struct FuseArgs {
    float* u;             // [looks][n] in: u_l, out: u_l'
    float* wprior;        // [n] the prior agent's w, in and out (NULL without a prior)
    const float* rprior;  // [n] the prior agent's output H(w) (NULL without a prior)
    float* xbar;          // [n] in: x_bar of the previous step, out: this step's
    float* wbar;          // [n] out: sum_j upsilon_j w_j after the step
    double* part;         // [row_blocks][2] partial sums of the convergence error
    float ups[64];
    float two_rho;
    int n_agents;
};
hipError_t launch_col(int mode, const ColArgs& a, hipStream_t st);
hipError_t launch_row(int mode, const RowArgs& a, hipStream_t st);
// mode ROW_UPDATE or ROW_UPDATE_EXACT; a.w is unused (the fused pass forms v
// from f.u and f.xbar); a.part gets one partial sum per (look, row block)
hipError_t launch_row_update_mann(int mode, const RowArgs& a, const FuseArgs& f, hipStream_t st);
hipError_t launch_scatter_full(const SceneTables& s, int looks, const float2* cmp,
                               float2* full, hipStream_t st);
hipError_t launch_gamma(const SceneTables& s, int looks, const double* part_row,
                        const double* part_colfwd, const double* part_colinv,
                        double inv_s2w, double* diag, uint32_t* fault, unsigned* counter, hipStream_t st);
hipError_t launch_resid_update(const SceneTables& s, int looks, float2* resid,
                               const float2* dfd, const double* diag, double* part,
                               hipStream_t st);
// h after, mu-residual and ||resid||^2 per look, then (last look done) the
// summary row diag[looks]; ahy2 may be NULL (mu-residuals 0).
hipError_t launch_diag_after(const SceneTables& s, int looks, const double* part_upd,
                             const double* part_resid, double s2w, const double* ahy2, double* diag,
                             unsigned* counter, hipStream_t st);
// out[i] = a[i] - b[i] over count complex values
hipError_t launch_csub(size_t count, const float2* a, const float2* b, float2* out, hipStream_t st);
hipError_t launch_init_r0(size_t n, int looks, float2* mu, float s_mu, float* r0,
                          double* part, hipStream_t st);
// out[l] = scale * sum_i part[l * count + i] for l < looks
hipError_t launch_sum(const double* part, int count, int looks, double scale, double* out,
                      hipStream_t st);
hipError_t launch_init_floor(size_t n, int n_agents, const double* mean_r0, float* r,
                             float* w, hipStream_t st);

struct MaceArgs {
    size_t n;
    int n_agents;
    float ups[64];
    float two_rho;
    float* w;
    const float* r;
    float* wbar;
    double* part;   // [mace_blocks][2]
};
hipError_t launch_mace(const MaceArgs& a, hipStream_t st);
hipError_t launch_mace_final(const double* part, int blocks, double* conv_err, hipStream_t st);
// out = the Mann state of the fused representation (see FuseArgs)
hipError_t launch_mann_state(size_t n, int looks, int n_agents, float two_rho, const float* u, const float* xbar,
                             float* out, hipStream_t st);
// Device address, on `device` (which must be current), of the static scratch
// of clamp_mace_step_noalloc: kMaceScratchDoubles doubles (1 MiB), enough for
// the partial sums of mace_blocks(n) blocks up to n = 2^25 voxels.
constexpr size_t kMaceScratchDoubles = 131072;
hipError_t mace_scratch(int device, double** out);

// Comparison regularizers (regularizers.hip): the l_{2,1} proximal map
// (part: nz * l21_chunks(nx, ny) doubles) and the TV proximal map by
// Chambolle's iteration (p: 3 n floats, u: n floats of scratch).
int l21_chunks(int nx, int ny);
hipError_t launch_prior_l21(int nx, int ny, int nz, float tau, const float* in, float* out, double* part,
                            hipStream_t st);
hipError_t launch_prior_tv(int nx, int ny, int nz, float lam, int iters, const float* in, float* out, float* p,
                           float* u, hipStream_t st);

hipError_t launch_gauss(int nx, int ny, int nz, const float* taps7, const float* in, float* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched passes over many scenes.  Each stage is one persistent launch that
// walks a device queue of work items of every scene.

struct BatchItem {
    int scene;
    int a;  // look, or column-pass item (look * nz + z) * tiles + tile
    int b;  // row group, or chunk
    int pad;
};

struct GammaArgs {
    int nrow, ncol;
    const double* prow;
    const double* pcf;
    const double* pci;
    double inv_s2w;
    double* diag;
    uint32_t* fault;
    unsigned* counter;   // looks done by the diagnostics pass (zeroed here)
};

struct ResidArgs {
    size_t per_look;
    int chunks;
    float2* resid;
    const float2* dfd;
    const double* diag;
    double* part;
};

struct DiagArgs {
    int nrow, nres, looks;
    const double* pupd;
    const double* pres;
    double s2w;
    const double* ahy2;  // [looks] ||A^H y_l||^2, or NULL
    double* diag;
    unsigned* counter;
};

// The Gaussian prior agent of one volume (gauss3d_tile): output tiles of
// kGaussTY rows by 64 or 32 x-voxels over kGaussCZ range slices.
constexpr int kGaussTY = 8, kGaussCZ = 8;
template <int TX>
__host__ __device__ inline int gauss_tiles(int nx, int ny, int nz) {
    return (nx / TX) * (ny / kGaussTY) * ((nz + kGaussCZ - 1) / kGaussCZ);
}
struct PriorArgs {
    int nx, ny, nz;
    float g[7];
    const float* in;
    float* out;
};

// Everything the batched stages need to know about one scene.
struct SceneBatch {
    RowArgs grad, update;
    ColArgs cinv, cfwd;
    GammaArgs gam;
    ResidArgs res;
    DiagArgs dia;
    MaceArgs mace;         // the Mann step as its own pass (mace.part also holds the fused form's partials)
    FuseArgs fuse;         // the Mann step fused into the update pass
    PriorArgs prior;
    int mace_chunks;       // partial-sum slots of the scene's convergence error
    int with_prior;
    double* conv;
};

// Work queues: column tiles, row groups of a look, row groups walking every
// look (the fused update pass), looks, residual chunks, Mann-step chunks,
// Gaussian-prior tiles of 64 and 32 x-voxels, scenes.
enum BatchQueue { Q_COL = 0, Q_ROW, Q_ROWG, Q_LOOK, Q_RESID, Q_VOX, Q_PRIOR64, Q_PRIOR32, Q_SCENE, Q_COUNT };

constexpr int kSizeClasses = 7;  // supported FFT lengths

struct BatchLaunch {
    const SceneBatch* scenes;   // device [nscenes]
    const BatchItem* queue[Q_COUNT];
    int count[Q_COUNT];
    int grid[Q_COUNT];          // persistent grid size of each stage
    // The row, column and fused row-group queues (segment sides 0, 1, 2) are
    // ordered by FFT length (nx for rows, ny for columns); each length class
    // is a segment with its own launch.
    int seg_len[3][kSizeClasses];
    int seg_off[3][kSizeClasses];
    int seg_count[3][kSizeClasses];
    int seg_grid[3][kSizeClasses];
    int nseg[3];
    const float* beta_table;    // device [beta_len]
    int beta_len;
    int* iter;                  // device iteration counter (iterations done)
    uint32_t* fault;
};

hipError_t batch_stage(int stage, const BatchLaunch& b, hipStream_t st);
hipError_t batch_set_iter(int* iter, int value, hipStream_t st);
enum BatchStage {
    BS_COL_INV = 0, BS_ROW_GRAD, BS_COL_FWD, BS_GAMMA, BS_ROW_UPDATE, BS_RESID, BS_DIAG,
    BS_PRIOR, BS_MACE, BS_MACE_FINAL, BS_NEXT_ITER, BS_ROW_UPDATE_MANN
};

}  // namespace clampk
