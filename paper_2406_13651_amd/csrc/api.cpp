// C ABI of the CLAMP forward-model library: argument validation, plan
// tables, workspace layout and the launch sequences of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/clamp.h"
#include "internal.h"

using clampk::ColArgs;
using clampk::RowArgs;
using clampk::SceneTables;

namespace {

thread_local std::string g_err;

clamp_status fail(clamp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

clamp_status ok() {
    return CLAMP_OK;
}

}  // namespace

namespace clampk {
clamp_status set_error(clamp_status st, const char* msg) {
    g_err = msg;
    return st;
}
}  // namespace clampk

namespace {

clamp_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return CLAMP_OK;
    return fail(CLAMP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool size_supported(int n) {
    switch (n) {
        case 32: case 64: case 128: case 192: case 256: case 384: case 512: return true;
        default: return false;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t T, T2, dfd, prow, pcf, pci, pupd, pres, pmace, scal, cnt, tvu, tvp, pl21;
    size_t dfdb, pzi, pzf;  // 3D operator: box data [L][K][P], range-pass partial sums
    size_t total;
};

struct Scene {
    clamp_scene sc{};
    int P = 0, B = 0, Bs = 0, tiles = 0, K = 0;
    double alpha = 0.0;
    std::vector<int> band_cols, band_pos, col_off, row_idx, pidx, pidxb;
    std::vector<void*> dev;  // device allocations owned by this scene
    SceneTables tab{};
    Layout ws{};
    size_t n() const { return (size_t)sc.nx * sc.ny * sc.nz; }
};

}  // namespace

// Timing stages; the names are returned by clamp_stage_name.
enum Stage {
    ST_COL_INV = 0, ST_ROW_GRAD, ST_COL_FWD, ST_GAMMA, ST_ROW_UPDATE, ST_RESID, ST_DIAG,
    ST_PRIOR, ST_MACE, ST_INIT, ST_OPERATOR, ST_OTHER, ST_RANGE_INV, ST_RANGE_FWD, ST_ROW_UPDATE_MANN
};
const char* const kStageNames[CLAMP_STAGES] = {
    "col_inv", "row_grad", "col_fwd", "gamma", "row_update", "resid_update", "diag_after",
    "prior_gauss", "mace_step", "init", "aperture_op", "other", "range_inv", "range_fwd", "row_update_mann"};

struct TimingRecord {
    int stage;
    hipEvent_t start, stop;
};

struct clamp_plan {
    int device = 0;
    std::vector<Scene> scenes;
    size_t ws_bytes = 0;
    uint32_t timing = 0u;  // bit s: record events around stage s
    std::vector<TimingRecord> records;
    std::vector<hipEvent_t> pool;
};

namespace {

void free_scene(Scene& s) {
    for (void* p : s.dev) (void)hipFree(p);
    s.dev.clear();
}

template <typename T>
clamp_status upload(Scene& s, const std::vector<T>& h, const T** out) {
    void* p = nullptr;
    const size_t bytes = h.size() * sizeof(T) > 0 ? h.size() * sizeof(T) : sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) return fail(CLAMP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
        return fail(CLAMP_EDEVICE, "hipMalloc: %s", hipGetErrorString(e));
    }
    s.dev.push_back(p);
    if (!h.empty()) {
        e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(CLAMP_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    }
    *out = static_cast<const T*>(p);
    return CLAMP_OK;
}

std::vector<float2> twiddles(int n) {
    std::vector<float2> t(n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < n; ++m) {
        const double ang = -two_pi * (double)m / (double)n;
        t[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    return t;
}

clamp_status build_scene(const clamp_scene& in, Scene& s) {
    s.sc = in;
    s.sc.pupil_mask = nullptr;
    const int nx = in.nx, ny = in.ny;
    std::vector<uint8_t> mask((size_t)nx * ny, 0);
    if (in.pupil_mask != nullptr) {
        for (size_t i = 0; i < mask.size(); ++i) mask[i] = in.pupil_mask[i] ? 1 : 0;
    } else {
        const double r2 = (double)in.pupil_radius * (double)in.pupil_radius;
        for (int u = 0; u < ny; ++u) {
            const long su = (2 * u >= ny) ? u - ny : u;
            for (int v = 0; v < nx; ++v) {
                const long sv = (2 * v >= nx) ? v - nx : v;
                mask[(size_t)u * nx + v] = (double)(su * su + sv * sv) <= r2 ? 1 : 0;
            }
        }
    }
    s.band_pos.assign(nx, -1);
    s.pidx.assign((size_t)nx * ny, -1);
    s.col_off.clear();
    s.row_idx.clear();
    s.band_cols.clear();
    // compact layout: pupil samples band column by band column (v
    // increasing), rows u increasing inside a column
    for (int v = 0; v < nx; ++v) {
        bool any = false;
        for (int u = 0; u < ny; ++u) any = any || mask[(size_t)u * nx + v];
        if (!any) continue;
        s.band_pos[v] = (int)s.band_cols.size();
        s.band_cols.push_back(v);
        s.col_off.push_back((int)s.row_idx.size());
        for (int u = 0; u < ny; ++u)
            if (mask[(size_t)u * nx + v]) {
                s.pidx[(size_t)u * nx + v] = (int)s.row_idx.size();
                s.row_idx.push_back(u);
            }
    }
    s.col_off.push_back((int)s.row_idx.size());
    s.P = (int)s.row_idx.size();
    s.B = (int)s.band_cols.size();
    if (s.P == 0) return fail(CLAMP_EINVAL, "pupil passes no DFT sample");
    s.tiles = (s.B + clampk::col_tile_cols(ny) - 1) / clampk::col_tile_cols(ny);
    s.Bs = s.tiles * clampk::col_tile_cols(ny);
    s.pidxb.assign((size_t)ny * s.Bs, -1);
    for (int u = 0; u < ny; ++u)
        for (int b = 0; b < s.B; ++b) s.pidxb[(size_t)u * s.Bs + b] = s.pidx[(size_t)u * nx + s.band_cols[b]];
    // the row passes' gather table: in-slice offsets of each column's band sample
    for (int v = 0; v < nx; ++v)
        if (s.band_pos[v] >= 0) s.band_pos[v] = clampk::band_col_off(s.band_pos[v], ny);
    s.K = in.range_support;
    s.alpha = s.K > 0 ? (double)s.P * s.K / ((double)nx * ny * in.nz) : (double)s.P / ((double)nx * ny);
    return CLAMP_OK;
}

clamp_status upload_scene(Scene& s) {
    SceneTables& t = s.tab;
    t.nx = s.sc.nx;
    t.ny = s.sc.ny;
    t.nz = s.sc.nz;
    t.P = s.P;
    t.B = s.B;
    t.Bs = s.Bs;
    t.tiles = s.tiles;
    clamp_status st;
    if ((st = upload(s, twiddles(s.sc.nx), &t.tw_x)) != CLAMP_OK) return st;
    if ((st = upload(s, twiddles(s.sc.ny), &t.tw_y)) != CLAMP_OK) return st;
    if ((st = upload(s, s.band_cols, &t.band_cols)) != CLAMP_OK) return st;
    if ((st = upload(s, s.band_pos, &t.band_pos)) != CLAMP_OK) return st;
    if ((st = upload(s, s.col_off, &t.col_off)) != CLAMP_OK) return st;
    if ((st = upload(s, s.row_idx, &t.row_idx)) != CLAMP_OK) return st;
    if ((st = upload(s, s.pidx, &t.pidx)) != CLAMP_OK) return st;
    if ((st = upload(s, s.pidxb, &t.pidxb)) != CLAMP_OK) return st;
    t.K = s.K;
    t.tw_z = nullptr;
    t.cpos = nullptr;
    if (s.K > 0) {
        std::vector<int> cpos(s.P);
        for (int c = 0; c < s.B; ++c)
            for (int p = s.col_off[c]; p < s.col_off[c + 1]; ++p) cpos[p] = s.row_idx[p] * s.sc.nx + s.band_cols[c];
        if ((st = upload(s, twiddles(s.sc.nz), &t.tw_z)) != CLAMP_OK) return st;
        if ((st = upload(s, cpos, &t.cpos)) != CLAMP_OK) return st;
    }
    return CLAMP_OK;
}

void layout_scene(Scene& s) {
    const size_t L = (size_t)s.sc.looks;
    const size_t band = L * s.sc.nz * s.sc.ny * (size_t)s.Bs * sizeof(float2);
    Layout& w = s.ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    w.T = take(band);
    w.T2 = take(band);
    w.dfd = take(L * s.sc.nz * (size_t)s.P * sizeof(float2));
    w.prow = take(L * clampk::row_blocks(s.tab) * 3 * sizeof(double));
    w.pcf = take(L * clampk::col_blocks(s.tab) * sizeof(double));
    w.pci = take(L * clampk::col_blocks(s.tab) * sizeof(double));
    w.pupd = take(L * clampk::row_blocks(s.tab) * sizeof(double));
    w.pres = take(L * clampk::resid_blocks(s.tab) * sizeof(double));
    w.pmace = take((size_t)std::max(clampk::mace_blocks(s.n()), clampk::row_blocks(s.tab)) * 2 * sizeof(double));
    w.scal = take(64 * sizeof(double));
    w.cnt = take(64 * sizeof(unsigned));
    w.tvu = take(s.n() * sizeof(float));
    w.tvp = take(3 * s.n() * sizeof(float));
    w.pl21 = take((size_t)s.sc.nz * clampk::l21_chunks(s.sc.nx, s.sc.ny) * sizeof(double));
    if (s.K > 0) {
        const size_t nz_blocks = (size_t)std::max(clampk::zpass_blocks(s.tab), clampk::gather_blocks(s.tab));
        w.dfdb = take(L * s.K * (size_t)s.P * sizeof(float2));
        w.pzi = take(L * nz_blocks * sizeof(double));
        w.pzf = take(L * nz_blocks * sizeof(double));
    }
    w.total = o;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

clamp_status check_plan_scene(const clamp_plan* plan, int32_t scene) {
    if (plan == nullptr) return fail(CLAMP_EINVAL, "plan is NULL");
    if (scene < 0 || scene >= (int32_t)plan->scenes.size())
        return fail(CLAMP_EINVAL, "scene index %d out of range [0, %zu)", scene, plan->scenes.size());
    return CLAMP_OK;
}

clamp_status check_ws(const void* ws) {
    if (ws == nullptr) return fail(CLAMP_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(CLAMP_EINVAL, "workspace is not 256-byte aligned");
    return CLAMP_OK;
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

clamp_status check_params(const Scene& s, const clamp_params* p, bool need_prox) {
    if (p == nullptr) return fail(CLAMP_EINVAL, "params is NULL");
    if (!finite_pos(p->sigma_w2)) return fail(CLAMP_EINVAL, "sigma_w2 must be finite and > 0");
    if (need_prox) {
        if (!finite_pos(p->sigma2)) return fail(CLAMP_EINVAL, "sigma2 must be finite and > 0");
        if (!(std::isfinite(p->beta) && p->beta > 1.f)) return fail(CLAMP_EINVAL, "beta must be finite and > 1");
    }
    if (!(p->rho > 0.f && p->rho < 1.f)) return fail(CLAMP_EINVAL, "rho must lie in (0, 1)");
    if (!finite_pos(p->mu_init_scale)) return fail(CLAMP_EINVAL, "mu_init_scale must be finite and > 0");
    if (p->r_update != CLAMP_R_QUADRATIC && p->r_update != CLAMP_R_EXACT)
        return fail(CLAMP_EINVAL, "r_update must be CLAMP_R_QUADRATIC or CLAMP_R_EXACT");
    const int L = s.sc.looks;
    if (p->n_agents != L && p->n_agents != L + 1)
        return fail(CLAMP_EINVAL, "n_agents must be looks (%d) or looks + 1", L);
    if (p->n_agents > 64) return fail(CLAMP_EINVAL, "at most 64 agents");
    if (s.n() >= ((size_t)1 << 31)) return fail(CLAMP_ESHAPE, "a look must hold fewer than 2^31 voxels");
    if (p->upsilon == nullptr) return fail(CLAMP_EINVAL, "upsilon is NULL");
    double sum = 0.0;
    for (int j = 0; j < p->n_agents; ++j) {
        if (!(std::isfinite(p->upsilon[j]) && p->upsilon[j] >= 0.f))
            return fail(CLAMP_EINVAL, "upsilon[%d] must be finite and >= 0", j);
        sum += p->upsilon[j];
    }
    if (std::fabs(sum - 1.0) > 1e-6) return fail(CLAMP_EINVAL, "upsilon sums to %.9g, not 1", sum);
    return CLAMP_OK;
}

hipEvent_t take_event(clamp_plan* p) {
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` (returning hipError_t) with timing events around it when the
// plan's timing is on.  Events go back to the pool unless both were recorded,
// so a record always refers to two recorded events.
template <typename F>
hipError_t timed(const clamp_plan* cplan, int stage, hipStream_t st, F&& launch) {
    clamp_plan* p = const_cast<clamp_plan*>(cplan);
    if (((p->timing >> stage) & 1u) == 0u) return launch();
    TimingRecord rec{stage, take_event(p), take_event(p)};
    if (rec.start == nullptr || rec.stop == nullptr) {
        if (rec.start != nullptr) p->pool.push_back(rec.start);
        if (rec.stop != nullptr) p->pool.push_back(rec.stop);
        return hipErrorOutOfMemory;
    }
    hipError_t e = hipEventRecord(rec.start, st);
    if (e != hipSuccess) {
        p->pool.push_back(rec.start);
        p->pool.push_back(rec.stop);
        return e;
    }
    e = launch();
    const hipError_t es = hipEventRecord(rec.stop, st);
    if (es == hipSuccess) {
        p->records.push_back(rec);
    } else {
        p->pool.push_back(rec.start);
        p->pool.push_back(rec.stop);
    }
    return e != hipSuccess ? e : es;
}

ColArgs col_args(const Scene& s, int looks) {
    ColArgs a{};
    a.s = s.tab;
    a.looks = looks;
    a.scale = (float)(1.0 / std::sqrt((double)s.sc.ny));
    return a;
}

RowArgs row_args(const Scene& s, int looks) {
    RowArgs a{};
    a.s = s.tab;
    a.looks = looks;
    a.scale = (float)(1.0 / std::sqrt((double)s.sc.nx));
    return a;
}

}  // namespace

extern "C" {

const char* clamp_last_error(void) { return g_err.c_str(); }

clamp_status clamp_plan_create(const clamp_scene* scenes, int32_t nscenes, clamp_plan** out) {
    if (out == nullptr) return fail(CLAMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (scenes == nullptr || nscenes <= 0) return fail(CLAMP_EINVAL, "need at least one scene");
    for (int i = 0; i < nscenes; ++i) {
        const clamp_scene& c = scenes[i];
        if (c.nx <= 0 || c.ny <= 0 || c.nz <= 0 || c.looks <= 0)
            return fail(CLAMP_EINVAL, "scene %d: sizes and looks must be positive", i);
        if (!size_supported(c.nx) || !size_supported(c.ny))
            return fail(CLAMP_EUNSUPPORTED, "scene %d: nx=%d ny=%d; supported: 32 64 128 192 256 384 512", i,
                        c.nx, c.ny);
        if (c.pupil_mask == nullptr && !(std::isfinite(c.pupil_radius) && c.pupil_radius > 0.f))
            return fail(CLAMP_EINVAL, "scene %d: pupil_radius must be > 0 without a mask", i);
        if (c.range_support < 0 || c.range_support > c.nz)
            return fail(CLAMP_EINVAL, "scene %d: range_support must lie in [0, nz]", i);
        if (c.range_support > 0 && !clampk::range_size_ok(c.nz))
            return fail(CLAMP_EUNSUPPORTED, "scene %d: the 3D operator needs nz in 16 32 48 64 96 128 192 256", i);
        if ((size_t)c.nx * c.ny * c.nz * (size_t)c.looks > ((size_t)1 << 40))
            return fail(CLAMP_ESHAPE, "scene %d too large", i);
    }
    int dev = 0;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(CLAMP_EDEVICE, "no HIP device available");
    if (hipGetDevice(&dev) != hipSuccess) return fail(CLAMP_EDEVICE, "hipGetDevice failed");
    clamp_plan* plan = new (std::nothrow) clamp_plan();
    if (plan == nullptr) return fail(CLAMP_ENOMEM, "host allocation failed");
    plan->device = dev;
    plan->scenes.resize(nscenes);
    for (int i = 0; i < nscenes; ++i) {
        clamp_status st = build_scene(scenes[i], plan->scenes[i]);
        if (st == CLAMP_OK) st = upload_scene(plan->scenes[i]);
        if (st != CLAMP_OK) {
            clamp_plan_destroy(plan);
            return st;
        }
        layout_scene(plan->scenes[i]);
        if (plan->scenes[i].ws.total > plan->ws_bytes) plan->ws_bytes = plan->scenes[i].ws.total;
    }
    *out = plan;
    return ok();
}

clamp_status clamp_plan_destroy(clamp_plan* plan) {
    if (plan == nullptr) return CLAMP_OK;
    for (TimingRecord& r : plan->records) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : plan->pool) (void)hipEventDestroy(e);
    for (Scene& s : plan->scenes) free_scene(s);
    delete plan;
    return CLAMP_OK;
}

clamp_status clamp_plan_workspace_size(const clamp_plan* plan, size_t* bytes) {
    if (plan == nullptr || bytes == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    *bytes = plan->ws_bytes;
    return CLAMP_OK;
}

clamp_status clamp_plan_pupil_info(const clamp_plan* plan, int32_t scene, int32_t* P, int32_t* B,
                                   double* alpha) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if (P) *P = s.P;
    if (B) *B = s.B;
    if (alpha) *alpha = s.alpha;
    return CLAMP_OK;
}

clamp_status clamp_plan_pupil_index(const clamp_plan* plan, int32_t scene, int32_t* idx) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    if (idx == nullptr) return fail(CLAMP_EINVAL, "idx is NULL");
    const Scene& s = plan->scenes[scene];
    for (int c = 0; c < s.B; ++c)
        for (int p = s.col_off[c]; p < s.col_off[c + 1]; ++p) idx[p] = s.row_idx[p] * s.sc.nx + s.band_cols[c];
    return CLAMP_OK;
}

clamp_status clamp_aperture_op(const clamp_plan* plan, int32_t scene, int32_t dir, const void* in, void* out,
                               int32_t nbatch, void* workspace, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    if (dir != CLAMP_FWD && dir != CLAMP_ADJ && dir != CLAMP_NORMAL) return fail(CLAMP_EINVAL, "bad direction %d", dir);
    if (nbatch < 0) return fail(CLAMP_EINVAL, "nbatch must be >= 0");
    if (nbatch == 0) return CLAMP_OK;
    if (in == nullptr || out == nullptr) return fail(CLAMP_EINVAL, "in/out is NULL");
    if ((st = check_ws(workspace)) != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    const size_t n = s.n();
    if ((const char*)in < (const char*)out + n * nbatch * sizeof(float2) &&
        (const char*)out < (const char*)in + n * nbatch * sizeof(float2))
        return fail(CLAMP_EINVAL, "in and out overlap");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    float2* T = at<float2>(workspace, s.ws.T);
    float2* T2 = at<float2>(workspace, s.ws.T2);
    float2* dfd = at<float2>(workspace, s.ws.dfd);
    const float2* src = static_cast<const float2*>(in);
    float2* dst = static_cast<float2*>(out);
    const bool range = s.K > 0;
    for (int b0 = 0; b0 < nbatch; b0 += s.sc.looks) {
        const int nb = (nbatch - b0 < s.sc.looks) ? nbatch - b0 : s.sc.looks;
        const float2* x = src + (size_t)b0 * n;
        float2* y = dst + (size_t)b0 * n;
        hipError_t e = hipSuccess;
        if (range) {
            // 3D operator: per-slice passes plus range passes on the pupil samples
            float2* box = at<float2>(workspace, s.ws.dfdb);
            double* pz = at<double>(workspace, s.ws.pzi);
            if (dir == CLAMP_FWD || dir == CLAMP_NORMAL) {
                RowArgs ra = row_args(s, nb);
                ra.img_in = x;
                ra.band_out = T2;
                e = clampk::launch_row(clampk::ROW_FWD, ra, stream);
                if (e == hipSuccess) {
                    ColArgs ca = col_args(s, nb);
                    ca.band_in = T2;
                    ca.cmp_out = dfd;
                    e = clampk::launch_col(clampk::COL_FWD_COMPACT, ca, stream);
                }
                clampk::ZArgs za{s.tab, nb, dfd, box, pz};
                if (e == hipSuccess) e = clampk::launch_zpass(-1, za, stream);
                if (e == hipSuccess && dir == CLAMP_FWD) e = clampk::launch_range_scatter(s.tab, nb, box, y, stream);
            }
            if (e == hipSuccess && (dir == CLAMP_ADJ || dir == CLAMP_NORMAL)) {
                if (dir == CLAMP_ADJ) e = clampk::launch_range_gather(s.tab, nb, x, box, nullptr, 1.f, pz, stream);
                clampk::ZArgs za{s.tab, nb, box, dfd, pz};
                if (e == hipSuccess) e = clampk::launch_zpass(+1, za, stream);
                ColArgs ca = col_args(s, nb);
                ca.cmp_in = dfd;
                ca.band_out = T;
                if (e == hipSuccess) e = clampk::launch_col(clampk::COL_INV_COMPACT, ca, stream);
                if (e == hipSuccess) {
                    RowArgs ra = row_args(s, nb);
                    ra.band_in = T;
                    ra.img_out = y;
                    e = clampk::launch_row(clampk::ROW_INV, ra, stream);
                }
            }
            if ((st = hip_check(e, "clamp_aperture_op launch")) != CLAMP_OK) return st;
            continue;
        }
        if (dir == CLAMP_FWD || dir == CLAMP_NORMAL) {
            RowArgs ra = row_args(s, nb);
            ra.img_in = x;
            ra.band_out = T2;
            e = clampk::launch_row(clampk::ROW_FWD, ra, stream);
            if (e == hipSuccess) {
                ColArgs ca = col_args(s, nb);
                ca.band_in = T2;
                ca.cmp_out = dfd;
                e = clampk::launch_col(clampk::COL_FWD_COMPACT, ca, stream);
            }
            if (e == hipSuccess && dir == CLAMP_FWD) e = clampk::launch_scatter_full(s.tab, nb, dfd, y, stream);
        }
        if (e == hipSuccess && (dir == CLAMP_ADJ || dir == CLAMP_NORMAL)) {
            ColArgs ca = col_args(s, nb);
            if (dir == CLAMP_ADJ) {
                ca.full_in = x;
                ca.band_out = T;
                e = clampk::launch_col(clampk::COL_INV_FULL, ca, stream);
            } else {
                ca.cmp_in = dfd;
                ca.band_out = T;
                e = clampk::launch_col(clampk::COL_INV_COMPACT, ca, stream);
            }
            if (e == hipSuccess) {
                RowArgs ra = row_args(s, nb);
                ra.band_in = T;
                ra.img_out = y;
                e = clampk::launch_row(clampk::ROW_INV, ra, stream);
            }
        }
        if ((st = hip_check(e, "clamp_aperture_op launch")) != CLAMP_OK) return st;
    }
    return CLAMP_OK;
}

clamp_status clamp_fwd_init(const clamp_plan* plan, int32_t scene, const clamp_params* params, const void* y_full,
                            clamp_fwd_state* state, float* w, void* workspace, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if ((st = check_params(s, params, false)) != CLAMP_OK) return st;
    if (y_full == nullptr || state == nullptr || w == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    if (state->mu == nullptr || state->resid == nullptr || state->r == nullptr)
        return fail(CLAMP_EINVAL, "state has a NULL array");
    if ((st = check_ws(workspace)) != CLAMP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int L = s.sc.looks;
    const size_t n = s.n();
    float2* T = at<float2>(workspace, s.ws.T);
    double* pci = at<double>(workspace, s.ws.pci);
    double* pm = at<double>(workspace, s.ws.pmace);
    double* scal = at<double>(workspace, s.ws.scal);
    float2* mu = static_cast<float2*>(state->mu);
    float2* ypup = static_cast<float2*>(state->y_pupil);

    hipError_t e = hipSuccess;
    if (s.K > 0) {
        // 3D operator: D(a) y on the cylinder (kept as y_pupil when given),
        // then A^H y = F2^H F_z^H (zero-filled box)
        float2* box = ypup != nullptr ? ypup : at<float2>(workspace, s.ws.dfdb);
        double* pg = at<double>(workspace, s.ws.pzi);
        e = clampk::launch_range_gather(s.tab, L, static_cast<const float2*>(y_full), box,
                                        static_cast<float2*>(state->resid), 1.f - params->mu_init_scale, pg, stream);
        if (e == hipSuccess && state->ahy2 != nullptr)
            e = clampk::launch_sum(pg, clampk::gather_blocks(s.tab), L, 1.0, state->ahy2, stream);
        clampk::ZArgs za{s.tab, L, box, at<float2>(workspace, s.ws.dfd), at<double>(workspace, s.ws.pzf)};
        if (e == hipSuccess) e = clampk::launch_zpass(+1, za, stream);
        ColArgs ca = col_args(s, L);
        ca.cmp_in = at<float2>(workspace, s.ws.dfd);
        ca.band_out = T;
        ca.part = pci;
        if (e == hipSuccess) e = clampk::launch_col(clampk::COL_INV_COMPACT, ca, stream);
    } else {
        ColArgs ca = col_args(s, L);
        ca.full_in = static_cast<const float2*>(y_full);
        ca.band_out = T;
        ca.cmp_out = static_cast<float2*>(state->resid);
        ca.cmp_keep = ypup;
        ca.part = pci;
        ca.init_keep = 1.f - params->mu_init_scale;
        e = clampk::launch_col(clampk::COL_INV_INIT, ca, stream);
    }
    if (e == hipSuccess) {
        RowArgs ra = row_args(s, L);
        ra.band_in = T;
        ra.img_out = mu;
        e = clampk::launch_row(clampk::ROW_INV, ra, stream);
    }
    if (e == hipSuccess && s.K == 0 && state->ahy2 != nullptr)
        e = clampk::launch_sum(pci, clampk::col_blocks(s.tab), L, 1.0, state->ahy2, stream);
    if (e == hipSuccess) e = clampk::launch_init_r0(n, L, mu, params->mu_init_scale, state->r, pm, stream);
    if (e == hipSuccess) e = clampk::launch_sum(pm, clampk::mace_blocks(n), 1, 1.0 / (double)n, scal, stream);
    if (e == hipSuccess) e = clampk::launch_init_floor(n, params->n_agents, scal, state->r, w, stream);
    return hip_check(e, "clamp_fwd_init launch");
}

clamp_status clamp_fwd_refresh(const clamp_plan* plan, int32_t scene, clamp_fwd_state* state, void* workspace,
                               void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if (state == nullptr || state->mu == nullptr || state->resid == nullptr)
        return fail(CLAMP_EINVAL, "state or one of its mu/resid arrays is NULL");
    if (state->y_pupil == nullptr) return fail(CLAMP_EINVAL, "state->y_pupil is NULL: nothing to refresh from");
    if ((st = check_ws(workspace)) != CLAMP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int L = s.sc.looks;
    float2* T2 = at<float2>(workspace, s.ws.T2);
    float2* dfd = at<float2>(workspace, s.ws.dfd);
    // D(a) F mu on the pupil (and the range box), then resid = D(a) y - that
    RowArgs ra = row_args(s, L);
    ra.img_in = static_cast<const float2*>(state->mu);
    ra.band_out = T2;
    hipError_t e = clampk::launch_row(clampk::ROW_FWD, ra, stream);
    ColArgs ca = col_args(s, L);
    ca.band_in = T2;
    ca.cmp_out = dfd;
    if (e == hipSuccess) e = clampk::launch_col(clampk::COL_FWD_COMPACT, ca, stream);
    const float2* amu = dfd;
    if (e == hipSuccess && s.K > 0) {
        float2* box = at<float2>(workspace, s.ws.dfdb);
        clampk::ZArgs za{s.tab, L, dfd, box, at<double>(workspace, s.ws.pzf)};
        e = clampk::launch_zpass(-1, za, stream);
        amu = box;
    }
    const size_t count = (size_t)L * (s.K > 0 ? s.K : s.sc.nz) * s.P;
    if (e == hipSuccess)
        e = clampk::launch_csub(count, static_cast<const float2*>(state->y_pupil), amu,
                                static_cast<float2*>(state->resid), stream);
    return hip_check(e, "clamp_fwd_refresh launch");
}

}  // extern "C"

namespace {

// Launches of one forward-agent application shared by clamp_fwd_agent and
// clamp_fwd_agent_mace: everything up to the step size (range pass, inverse
// column pass, gradient row pass, forward column pass, range pass, gamma),
// then `update` (the update row pass, plain or with the Mann step), then the
// residual update and the diagnostics.
struct AgentRun {
    const clamp_plan* plan;
    const Scene& s;
    const clamp_params* params;
    clamp_fwd_state* state;
    double* diag;
    uint32_t* fault;
    void* workspace;
    hipStream_t stream;
};

RowArgs agent_row_args(const AgentRun& r, const float* w) {
    const Scene& s = r.s;
    const double s2w = r.params->sigma_w2;
    const double beta = r.params->beta;
    RowArgs ra = row_args(s, s.sc.looks);
    ra.mu = static_cast<float2*>(r.state->mu);
    ra.r = r.state->r;
    ra.w = w;
    ra.diag = r.diag;
    ra.fault = r.fault;
    ra.inv_s2w = (float)(1.0 / s2w);
    ra.s2w = (float)s2w;
    ra.floor_w = (float)(s2w / s.alpha);
    ra.alpha = (float)s.alpha;
    ra.sigma2 = r.params->sigma2;
    ra.inv_sigma2 = (float)(1.0 / (double)r.params->sigma2);
    ra.beta = (float)beta;
    ra.inv_beta = (float)(1.0 / beta);
    ra.k_up = (float)((1.0 + beta) / (beta * beta));
    ra.k_dn = (float)(beta * (1.0 + beta));
    return ra;
}

template <typename Update>
hipError_t agent_launches(const AgentRun& r, const RowArgs& ra, Update&& update) {
    const Scene& s = r.s;
    const clamp_plan* plan = r.plan;
    void* workspace = r.workspace;
    hipStream_t stream = r.stream;
    const int L = s.sc.looks;
    const double s2w = r.params->sigma_w2;
    float2* T = at<float2>(workspace, s.ws.T);
    float2* T2 = at<float2>(workspace, s.ws.T2);
    float2* dfd = at<float2>(workspace, s.ws.dfd);
    double* prow = at<double>(workspace, s.ws.prow);
    double* pcf = at<double>(workspace, s.ws.pcf);
    double* pci = at<double>(workspace, s.ws.pci);
    double* pupd = at<double>(workspace, s.ws.pupd);
    double* pres = at<double>(workspace, s.ws.pres);
    float2* resid = static_cast<float2*>(r.state->resid);

    // 3D operator: the residual lives on the cylinder [K][P]; a range pass
    // spreads it over every slice first, and one after the forward column
    // pass crops A d back to the box.  The gamma and residual sums then come
    // from the range passes.
    const bool range = s.K > 0;
    float2* dfd_box = range ? at<float2>(workspace, s.ws.dfdb) : dfd;
    double* pz_inv = range ? at<double>(workspace, s.ws.pzi) : pci;
    double* pz_fwd = range ? at<double>(workspace, s.ws.pzf) : pcf;
    hipError_t e = hipSuccess;
    if (range) {
        clampk::ZArgs za{s.tab, L, resid, dfd, pz_inv};
        e = timed(plan, ST_RANGE_INV, stream, [&] { return clampk::launch_zpass(+1, za, stream); });
    }
    ColArgs ci = col_args(s, L);
    ci.cmp_in = range ? dfd : resid;
    ci.band_out = T;
    ci.part = pci;
    if (e == hipSuccess)
        e = timed(plan, ST_COL_INV, stream, [&] { return clampk::launch_col(clampk::COL_INV_COMPACT, ci, stream); });
    if (e == hipSuccess) {
        RowArgs g = ra;
        g.band_in = T;
        g.band_out = T2;
        g.part = prow;
        e = timed(plan, ST_ROW_GRAD, stream, [&] { return clampk::launch_row(clampk::ROW_GRAD, g, stream); });
    }
    if (e == hipSuccess) {
        ColArgs cf = col_args(s, L);
        cf.band_in = T2;
        cf.cmp_out = dfd;
        cf.part = pcf;
        e = timed(plan, ST_COL_FWD, stream, [&] { return clampk::launch_col(clampk::COL_FWD_COMPACT, cf, stream); });
    }
    if (e == hipSuccess && range) {
        clampk::ZArgs za{s.tab, L, dfd, dfd_box, pz_fwd};
        e = timed(plan, ST_RANGE_FWD, stream, [&] { return clampk::launch_zpass(-1, za, stream); });
    }
    unsigned* counter = at<unsigned>(workspace, s.ws.cnt);
    if (e == hipSuccess)
        e = timed(plan, ST_GAMMA, stream, [&] {
            return clampk::launch_gamma(s.tab, L, prow, pz_fwd, pz_inv, 1.0 / s2w, r.diag, r.fault, counter, stream);
        });
    if (e == hipSuccess) {
        RowArgs u = ra;
        u.band_in = T;
        u.part = pupd;
        e = update(u);
    }
    if (e == hipSuccess)
        e = timed(plan, ST_RESID, stream,
                  [&] { return clampk::launch_resid_update(s.tab, L, resid, dfd_box, r.diag, pres, stream); });
    if (e == hipSuccess)
        e = timed(plan, ST_DIAG, stream, [&] {
            return clampk::launch_diag_after(s.tab, L, pupd, pres, s2w, r.state->ahy2, r.diag, counter, stream);
        });
    return e;
}

clamp_status check_agent_args(const clamp_plan* plan, int32_t scene, const clamp_params* params,
                              const clamp_fwd_state* state, const void* w, const double* diag, const uint32_t* fault,
                              const void* workspace) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if ((st = check_params(s, params, true)) != CLAMP_OK) return st;
    if (state == nullptr || w == nullptr || diag == nullptr || fault == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    if (state->mu == nullptr || state->resid == nullptr || state->r == nullptr)
        return fail(CLAMP_EINVAL, "state has a NULL array");
    return check_ws(workspace);
}

}  // namespace

extern "C" {

clamp_status clamp_fwd_agent(const clamp_plan* plan, int32_t scene, const clamp_params* params,
                             clamp_fwd_state* state, const float* w, double* diag, uint32_t* fault,
                             void* workspace, void* hip_stream) {
    clamp_status st = check_agent_args(plan, scene, params, state, w, diag, fault, workspace);
    if (st != CLAMP_OK) return st;
    const AgentRun run{plan, plan->scenes[scene], params, state, diag, fault, workspace,
                       static_cast<hipStream_t>(hip_stream)};
    const int mode = params->r_update == CLAMP_R_EXACT ? clampk::ROW_UPDATE_EXACT : clampk::ROW_UPDATE;
    const hipError_t e = agent_launches(run, agent_row_args(run, w), [&](const RowArgs& u) {
        return timed(plan, ST_ROW_UPDATE, run.stream, [&] { return clampk::launch_row(mode, u, run.stream); });
    });
    return hip_check(e, "clamp_fwd_agent launch");
}

clamp_status clamp_fwd_agent_mace(const clamp_plan* plan, int32_t scene, const clamp_params* params,
                                  clamp_fwd_state* state, float* w, float* xbar, float* wbar, double* diag,
                                  double* conv_err, uint32_t* fault, void* workspace, void* hip_stream) {
    clamp_status st = check_agent_args(plan, scene, params, state, w, diag, fault, workspace);
    if (st != CLAMP_OK) return st;
    if (xbar == nullptr || wbar == nullptr || conv_err == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    const Scene& s = plan->scenes[scene];
    const AgentRun run{plan, s, params, state, diag, fault, workspace, static_cast<hipStream_t>(hip_stream)};
    const int L = s.sc.looks;
    const size_t n = s.n();
    clampk::FuseArgs f{};
    f.u = w;
    const bool prior = params->n_agents == L + 1;
    f.wprior = prior ? w + (size_t)L * n : nullptr;
    f.rprior = prior ? state->r + (size_t)L * n : nullptr;
    f.xbar = xbar;
    f.wbar = wbar;
    f.part = at<double>(workspace, s.ws.pmace);
    for (int j = 0; j < params->n_agents; ++j) f.ups[j] = params->upsilon[j];
    f.two_rho = 2.f * params->rho;
    f.n_agents = params->n_agents;
    const int mode = params->r_update == CLAMP_R_EXACT ? clampk::ROW_UPDATE_EXACT : clampk::ROW_UPDATE;
    hipError_t e = agent_launches(run, agent_row_args(run, w), [&](const RowArgs& u) {
        return timed(plan, ST_ROW_UPDATE_MANN, run.stream,
                     [&] { return clampk::launch_row_update_mann(mode, u, f, run.stream); });
    });
    if (e == hipSuccess)
        e = timed(plan, ST_MACE, run.stream, [&] {
            return clampk::launch_mace_final(f.part, clampk::row_blocks(s.tab), conv_err, run.stream);
        });
    return hip_check(e, "clamp_fwd_agent_mace launch");
}

clamp_status clamp_prior_gauss(const clamp_plan* plan, int32_t scene, float sigma_vox, const float* in, float* out,
                               void* workspace, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    if (!finite_pos(sigma_vox)) return fail(CLAMP_EINVAL, "sigma_vox must be finite and > 0");
    if (in == nullptr || out == nullptr) return fail(CLAMP_EINVAL, "in/out is NULL");
    if (in == out) return fail(CLAMP_EINVAL, "in and out must not overlap");
    if (reinterpret_cast<uintptr_t>(in) % 16 != 0) return fail(CLAMP_EINVAL, "in must be 16-byte aligned");
    if ((st = check_ws(workspace)) != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    double g[7], sum = 0.0;
    for (int k = 0; k < 7; ++k) {
        const double x = (k - 3) / (double)sigma_vox;
        g[k] = std::exp(-0.5 * x * x);
        sum += g[k];
    }
    float taps[7];
    for (int k = 0; k < 7; ++k) taps[k] = (float)(g[k] / sum);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = timed(plan, ST_PRIOR, stream, [&] {
        return clampk::launch_gauss(s.sc.nx, s.sc.ny, s.sc.nz, taps, in, out, stream);
    });
    return hip_check(e, "clamp_prior_gauss launch");
}

static clamp_status check_prior_io(const clamp_plan* plan, int32_t scene, const float* in, float* out,
                                   const void* workspace) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    if (in == nullptr || out == nullptr) return fail(CLAMP_EINVAL, "in/out is NULL");
    const size_t n = plan->scenes[scene].n();
    if (in < out + n && out < in + n) return fail(CLAMP_EINVAL, "in and out must not overlap");
    return check_ws(workspace);
}

clamp_status clamp_prior_l21(const clamp_plan* plan, int32_t scene, float tau, const float* in, float* out,
                             void* workspace, void* hip_stream) {
    clamp_status st = check_prior_io(plan, scene, in, out, workspace);
    if (st != CLAMP_OK) return st;
    if (!(std::isfinite(tau) && tau >= 0.f)) return fail(CLAMP_EINVAL, "tau must be finite and >= 0");
    const Scene& s = plan->scenes[scene];
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hipError_t e = timed(plan, ST_PRIOR, stream, [&] {
        return clampk::launch_prior_l21(s.sc.nx, s.sc.ny, s.sc.nz, tau, in, out, at<double>(workspace, s.ws.pl21),
                                        stream);
    });
    return hip_check(e, "clamp_prior_l21 launch");
}

clamp_status clamp_prior_tv(const clamp_plan* plan, int32_t scene, float lam, int32_t iters, const float* in,
                            float* out, void* workspace, void* hip_stream) {
    clamp_status st = check_prior_io(plan, scene, in, out, workspace);
    if (st != CLAMP_OK) return st;
    if (!finite_pos(lam)) return fail(CLAMP_EINVAL, "lam must be finite and > 0");
    if (iters < 0 || iters > 100000) return fail(CLAMP_EINVAL, "iters must lie in [0, 100000]");
    const Scene& s = plan->scenes[scene];
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hipError_t e = timed(plan, ST_PRIOR, stream, [&] {
        return clampk::launch_prior_tv(s.sc.nx, s.sc.ny, s.sc.nz, lam, iters, in, out, at<float>(workspace, s.ws.tvp),
                                       at<float>(workspace, s.ws.tvu), stream);
    });
    return hip_check(e, "clamp_prior_tv launch");
}

clamp_status clamp_mace_step(const clamp_plan* plan, int32_t scene, const clamp_params* params, float* w,
                             const float* r, float* wbar, double* conv_err, void* workspace, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if ((st = check_params(s, params, false)) != CLAMP_OK) return st;
    if (w == nullptr || r == nullptr || wbar == nullptr || conv_err == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    if ((st = check_ws(workspace)) != CLAMP_OK) return st;
    clampk::MaceArgs a{};
    a.n = s.n();
    a.n_agents = params->n_agents;
    for (int j = 0; j < params->n_agents; ++j) a.ups[j] = params->upsilon[j];
    a.two_rho = 2.f * params->rho;
    a.w = w;
    a.r = r;
    a.wbar = wbar;
    a.part = at<double>(workspace, s.ws.pmace);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = timed(plan, ST_MACE, stream, [&] {
        hipError_t x = clampk::launch_mace(a, stream);
        if (x == hipSuccess) x = clampk::launch_mace_final(a.part, clampk::mace_blocks(a.n), conv_err, stream);
        return x;
    });
    return hip_check(e, "clamp_mace_step launch");
}

clamp_status clamp_mace_state(const clamp_plan* plan, int32_t scene, const clamp_params* params, const float* w,
                              const float* xbar, float* out, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if ((st = check_params(s, params, false)) != CLAMP_OK) return st;
    if (w == nullptr || xbar == nullptr || out == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    const size_t n = s.n();
    const size_t total = n * (size_t)params->n_agents;
    if ((const char*)out < (const char*)(w + total) && (const char*)w < (const char*)(out + total))
        return fail(CLAMP_EINVAL, "w and out overlap");
    const hipError_t e = clampk::launch_mann_state(n, s.sc.looks, params->n_agents, 2.f * params->rho, w, xbar,
                                                   out, static_cast<hipStream_t>(hip_stream));
    return hip_check(e, "clamp_mace_state launch");
}

clamp_status clamp_mace_step_noalloc(const clamp_plan* plan, int32_t scene, const clamp_params* params, float* w,
                                     const float* r, float* wbar, double* conv_err, void* hip_stream) {
    clamp_status st = check_plan_scene(plan, scene);
    if (st != CLAMP_OK) return st;
    const Scene& s = plan->scenes[scene];
    if ((st = check_params(s, params, false)) != CLAMP_OK) return st;
    if (w == nullptr || r == nullptr || wbar == nullptr || conv_err == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    const size_t n = s.n();
    if (n % 2 != 0) return fail(CLAMP_ESHAPE, "the Mann step needs an even voxel count");
    const int blocks = clampk::mace_blocks(n);
    if ((size_t)blocks * 2 > clampk::kMaceScratchDoubles)
        return fail(CLAMP_ESHAPE,
                    "volume of %zu voxels needs %zu bytes of scratch; clamp_mace_step_noalloc holds %zu "
                    "(volumes up to 2^25 voxels); use clamp_mace_step with a workspace",
                    n, (size_t)blocks * 2 * sizeof(double), clampk::kMaceScratchDoubles * sizeof(double));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "hipGetDevice");
    if (dev != plan->device)
        return fail(CLAMP_EDEVICE, "current device %d is not the plan's device %d", dev, plan->device);
    double* part = nullptr;
    if ((e = clampk::mace_scratch(dev, &part)) != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    clampk::MaceArgs a{};
    a.n = n;
    a.n_agents = params->n_agents;
    for (int j = 0; j < params->n_agents; ++j) a.ups[j] = params->upsilon[j];
    a.two_rho = 2.f * params->rho;
    a.w = w;
    a.r = r;
    a.wbar = wbar;
    a.part = part;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    e = clampk::launch_mace(a, stream);
    if (e == hipSuccess) e = clampk::launch_mace_final(part, blocks, conv_err, stream);
    return hip_check(e, "clamp_mace_step_noalloc launch");
}

clamp_status clamp_plan_set_timing(clamp_plan* plan, int32_t enable) {
    if (plan == nullptr) return fail(CLAMP_EINVAL, "plan is NULL");
    plan->timing = enable != 0 ? (1u << CLAMP_STAGES) - 1u : 0u;
    return CLAMP_OK;
}

clamp_status clamp_plan_set_timing_stages(clamp_plan* plan, uint32_t stage_mask) {
    if (plan == nullptr) return fail(CLAMP_EINVAL, "plan is NULL");
    if (stage_mask >> CLAMP_STAGES) return fail(CLAMP_EINVAL, "stage mask has bits at or past CLAMP_STAGES");
    plan->timing = stage_mask;
    return CLAMP_OK;
}

clamp_status clamp_plan_get_timing(clamp_plan* plan, double* total_ms, int32_t* launches) {
    if (plan == nullptr || total_ms == nullptr || launches == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    for (int i = 0; i < CLAMP_STAGES; ++i) {
        total_ms[i] = 0.0;
        launches[i] = 0;
    }
    clamp_status st = CLAMP_OK;
    for (TimingRecord& r : plan->records) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess && st == CLAMP_OK) st = hip_check(e, "clamp_plan_get_timing");
        total_ms[r.stage] += ms;
        launches[r.stage] += 1;
        plan->pool.push_back(r.start);
        plan->pool.push_back(r.stop);
    }
    plan->records.clear();
    return st;
}

const char* clamp_stage_name(int32_t stage) {
    if (stage < 0 || stage >= CLAMP_STAGES) return "";
    return kStageNames[stage];
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches
namespace {

constexpr int kBetaLen = 1 << 16;
const int kLengths[clampk::kSizeClasses] = {512, 384, 256, 192, 128, 64, 32};

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

}  // namespace

struct clamp_batch {
    const clamp_plan* plan = nullptr;
    clampk::BatchLaunch launch{};
    std::vector<void*> dev;
    int cus = 256;
    // persistent grid sizes in blocks per CU; 0 = one block per work item
    int row_per_cu = 0, col_per_cu = 4;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool fused = false;  // the Mann step inside the update pass (every scene has an xbar)
};

namespace {

void batch_free(clamp_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void* p : b->dev) (void)hipFree(p);
    b->dev.clear();
}

template <typename T>
clamp_status batch_upload(clamp_batch* b, const std::vector<T>& h, T** out) {
    void* p = nullptr;
    const size_t bytes = (h.empty() ? 1 : h.size()) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CLAMP_ENOMEM : CLAMP_EDEVICE, "hipMalloc: %s",
                                     hipGetErrorString(e));
    b->dev.push_back(p);
    if (!h.empty() && (e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(CLAMP_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    *out = static_cast<T*>(p);
    return CLAMP_OK;
}

void batch_grids(clamp_batch* b) {
    clampk::BatchLaunch& L = b->launch;
    auto cap = [&](int count, int per_cu) {
        return (per_cu <= 0 || count < b->cus * per_cu) ? count : b->cus * per_cu;
    };
    for (int g = 0; g < L.nseg[0]; ++g) L.seg_grid[0][g] = cap(L.seg_count[0][g], b->row_per_cu);
    for (int g = 0; g < L.nseg[1]; ++g) L.seg_grid[1][g] = cap(L.seg_count[1][g], b->col_per_cu);
    for (int g = 0; g < L.nseg[2]; ++g) L.seg_grid[2][g] = L.seg_count[2][g];
    L.grid[clampk::Q_LOOK] = L.count[clampk::Q_LOOK];
    L.grid[clampk::Q_SCENE] = L.count[clampk::Q_SCENE];
    for (int q : {clampk::Q_RESID, clampk::Q_VOX, clampk::Q_PRIOR64, clampk::Q_PRIOR32}) L.grid[q] = L.count[q];
}

hipError_t batch_run(clamp_batch* b, hipStream_t st) {
    using namespace clampk;
    const clamp_plan* p = b->plan;
    // Alg. 2's order; with the Mann step fused into the update pass the prior
    // agents (which read only their own w) run first
    const int plain[] = {BS_COL_INV, BS_ROW_GRAD, BS_COL_FWD, BS_GAMMA, BS_ROW_UPDATE, BS_RESID, BS_DIAG, BS_PRIOR};
    const int plain_t[] = {ST_COL_INV, ST_ROW_GRAD, ST_COL_FWD, ST_GAMMA, ST_ROW_UPDATE, ST_RESID, ST_DIAG, ST_PRIOR};
    const int fused[] = {BS_PRIOR, BS_COL_INV, BS_ROW_GRAD, BS_COL_FWD, BS_GAMMA, BS_ROW_UPDATE_MANN, BS_RESID,
                         BS_DIAG};
    const int fused_t[] = {ST_PRIOR, ST_COL_INV, ST_ROW_GRAD, ST_COL_FWD, ST_GAMMA, ST_ROW_UPDATE_MANN, ST_RESID,
                           ST_DIAG};
    const int* stages = b->fused ? fused : plain;
    const int* timing_stage = b->fused ? fused_t : plain_t;
    for (int i = 0; i < 8; ++i) {
        const hipError_t e = timed(p, timing_stage[i], st, [&] { return batch_stage(stages[i], b->launch, st); });
        if (e != hipSuccess) return e;
    }
    hipError_t e = timed(p, ST_MACE, st, [&] {
        hipError_t x = b->fused ? hipSuccess : batch_stage(BS_MACE, b->launch, st);
        if (x == hipSuccess) x = batch_stage(BS_MACE_FINAL, b->launch, st);
        return x;
    });
    if (e == hipSuccess) e = batch_stage(BS_NEXT_ITER, b->launch, st);
    return e;
}

}  // namespace

extern "C" {

clamp_status clamp_batch_workspace_size(const clamp_plan* plan, size_t* bytes) {
    if (plan == nullptr || bytes == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    size_t total = 0;
    for (const Scene& s : plan->scenes) total += align256(s.ws.total);
    *bytes = total;
    return CLAMP_OK;
}

clamp_status clamp_batch_create(const clamp_plan* plan, const clamp_batch_scene* scenes, uint32_t* fault,
                                double* conv_err, void* workspace, clamp_batch** out) {
    using namespace clampk;
    if (out == nullptr) return fail(CLAMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (plan == nullptr || scenes == nullptr || fault == nullptr || conv_err == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    clamp_status st = check_ws(workspace);
    if (st != CLAMP_OK) return st;
    const int ns = (int)plan->scenes.size();
    std::vector<SceneBatch> hb(ns);
    std::vector<BatchItem> q[Q_COUNT];
    // row and column items grouped by FFT length, longest first
    std::vector<BatchItem> rows_by_len[kSizeClasses], cols_by_len[kSizeClasses], rowg_by_len[kSizeClasses];
    int n_fused = 0;
    for (int i = 0; i < ns; ++i) n_fused += scenes[i].xbar != nullptr ? 1 : 0;
    if (n_fused != 0 && n_fused != ns)
        return fail(CLAMP_EINVAL, "either every scene of a batch has an xbar (the fused Mann step) or none has");
    const bool fused = n_fused == ns && ns > 0;
    size_t ws_off = 0;
    for (int i = 0; i < ns; ++i) {
        const Scene& s = plan->scenes[i];
        const clamp_batch_scene& bs = scenes[i];
        if ((st = check_params(s, &bs.params, true)) != CLAMP_OK) return fail(st, "scene %d: %s", i, g_err.c_str());
        if (bs.params.n_agents > 40) return fail(CLAMP_EUNSUPPORTED, "scene %d: a batch holds at most 40 agents", i);
        if (bs.params.r_update != CLAMP_R_QUADRATIC)
            return fail(CLAMP_EUNSUPPORTED, "scene %d: batches use the quadratic-surrogate r-update", i);
        if (s.K > 0) return fail(CLAMP_EUNSUPPORTED, "scene %d: batches use the per-slice operator", i);
        if (bs.state.mu == nullptr || bs.state.resid == nullptr || bs.state.r == nullptr || bs.w == nullptr ||
            bs.wbar == nullptr || bs.diag == nullptr)
            return fail(CLAMP_EINVAL, "scene %d: NULL array", i);
        const bool with_prior = bs.params.n_agents == s.sc.looks + 1;
        if (with_prior && !finite_pos(bs.prior_sigma))
            return fail(CLAMP_EINVAL, "scene %d: prior_sigma must be > 0", i);
        if (with_prior && (s.sc.ny % kGaussTY != 0 || s.sc.nx % 32 != 0))
            return fail(CLAMP_EUNSUPPORTED, "scene %d: the Gaussian prior needs ny a multiple of %d and nx of 32", i,
                        kGaussTY);
        void* w0 = static_cast<char*>(workspace) + ws_off;
        ws_off += align256(s.ws.total);
        const int L = s.sc.looks;
        const size_t n = s.n();
        SceneBatch& sb = hb[i];
        const double s2w = bs.params.sigma_w2;
        RowArgs ra = row_args(s, L);
        ra.mu = static_cast<float2*>(bs.state.mu);
        ra.r = bs.state.r;
        ra.w = bs.w;
        ra.diag = bs.diag;
        ra.fault = fault;
        ra.inv_s2w = (float)(1.0 / s2w);
        ra.s2w = (float)s2w;
        ra.floor_w = (float)(s2w / s.alpha);
        ra.alpha = (float)s.alpha;
        ra.sigma2 = bs.params.sigma2;
        ra.inv_sigma2 = (float)(1.0 / (double)bs.params.sigma2);
        sb.grad = ra;
        sb.grad.band_in = at<float2>(w0, s.ws.T);
        sb.grad.band_out = at<float2>(w0, s.ws.T2);
        sb.grad.part = at<double>(w0, s.ws.prow);
        sb.update = ra;
        sb.update.band_in = at<float2>(w0, s.ws.T);
        sb.update.part = at<double>(w0, s.ws.pupd);
        sb.cinv = col_args(s, L);
        sb.cinv.cmp_in = static_cast<const float2*>(bs.state.resid);
        sb.cinv.band_out = at<float2>(w0, s.ws.T);
        sb.cinv.part = at<double>(w0, s.ws.pci);
        sb.cfwd = col_args(s, L);
        sb.cfwd.band_in = at<float2>(w0, s.ws.T2);
        sb.cfwd.cmp_out = at<float2>(w0, s.ws.dfd);
        sb.cfwd.part = at<double>(w0, s.ws.pcf);
        sb.gam = GammaArgs{row_blocks(s.tab), col_blocks(s.tab), at<double>(w0, s.ws.prow), at<double>(w0, s.ws.pcf),
                           at<double>(w0, s.ws.pci), 1.0 / s2w, bs.diag, fault, at<unsigned>(w0, s.ws.cnt)};
        sb.res = ResidArgs{(size_t)s.sc.nz * s.P, resid_chunks(s.tab), static_cast<float2*>(bs.state.resid),
                           at<float2>(w0, s.ws.dfd), bs.diag, at<double>(w0, s.ws.pres)};
        sb.dia = DiagArgs{row_blocks(s.tab), resid_chunks(s.tab), L, at<double>(w0, s.ws.pupd),
                          at<double>(w0, s.ws.pres), s2w, bs.state.ahy2, bs.diag, at<unsigned>(w0, s.ws.cnt)};
        MaceArgs m{};
        m.n = n;
        m.n_agents = bs.params.n_agents;
        for (int j = 0; j < m.n_agents; ++j) m.ups[j] = bs.params.upsilon[j];
        m.two_rho = 2.f * bs.params.rho;
        m.w = bs.w;
        m.r = bs.state.r;
        m.wbar = bs.wbar;
        m.part = at<double>(w0, s.ws.pmace);
        sb.mace = m;
        sb.mace_chunks = fused ? row_blocks(s.tab) : mace_blocks(n);
        if (fused) {
            FuseArgs f{};
            f.u = bs.w;
            f.wprior = with_prior ? bs.w + (size_t)L * n : nullptr;
            f.rprior = with_prior ? bs.state.r + (size_t)L * n : nullptr;
            f.xbar = bs.xbar;
            f.wbar = bs.wbar;
            f.part = m.part;
            for (int j = 0; j < m.n_agents; ++j) f.ups[j] = m.ups[j];
            f.two_rho = m.two_rho;
            f.n_agents = m.n_agents;
            sb.fuse = f;
        }
        sb.with_prior = with_prior ? 1 : 0;
        sb.conv = conv_err + i;
        PriorArgs pr{};
        pr.nx = s.sc.nx;
        pr.ny = s.sc.ny;
        pr.nz = s.sc.nz;
        if (with_prior) {
            double g[7], sum = 0.0;
            for (int k = 0; k < 7; ++k) {
                const double x = (k - 3) / (double)bs.prior_sigma;
                g[k] = std::exp(-0.5 * x * x);
                sum += g[k];
            }
            for (int k = 0; k < 7; ++k) pr.g[k] = (float)(g[k] / sum);
            pr.in = bs.w + (size_t)L * n;
            pr.out = bs.state.r + (size_t)L * n;
        }
        sb.prior = pr;
        // work items
        int li = 0, ci = 0;
        for (int k = 0; k < kSizeClasses; ++k) {
            if (kLengths[k] == s.sc.nx) li = k;
            if (kLengths[k] == s.sc.ny) ci = k;
        }
        for (int l = 0; l < L; ++l)
            for (int g = 0; g < row_blocks(s.tab); ++g) rows_by_len[li].push_back(BatchItem{i, l, g, 0});
        if (fused)
            for (int g = 0; g < row_blocks(s.tab); ++g) rowg_by_len[li].push_back(BatchItem{i, 0, g, 0});
        for (int it = 0; it < L * s.sc.nz * s.tiles; ++it) cols_by_len[ci].push_back(BatchItem{i, it, 0, 0});
        for (int l = 0; l < L; ++l) {
            q[Q_LOOK].push_back(BatchItem{i, l, 0, 0});
            for (int c = 0; c < resid_chunks(s.tab); ++c) q[Q_RESID].push_back(BatchItem{i, l, c, 0});
        }
        if (!fused)
            for (int c = 0; c < sb.mace_chunks; ++c) q[Q_VOX].push_back(BatchItem{i, 0, c, 0});
        q[Q_SCENE].push_back(BatchItem{i, 0, 0, 0});
        if (with_prior) {
            // output tiles of the single-pass Gaussian (gauss3d_tile)
            const int tx = s.sc.nx % 64 == 0 ? 64 : 32;
            const int tiles = tx == 64 ? gauss_tiles<64>(s.sc.nx, s.sc.ny, s.sc.nz)
                                       : gauss_tiles<32>(s.sc.nx, s.sc.ny, s.sc.nz);
            for (int c = 0; c < tiles; ++c) q[tx == 64 ? Q_PRIOR64 : Q_PRIOR32].push_back(BatchItem{i, 0, c, 0});
        }
    }
    clamp_batch* b = new (std::nothrow) clamp_batch();
    if (b == nullptr) return fail(CLAMP_ENOMEM, "host allocation failed");
    b->plan = plan;
    b->cus = device_cus();
    b->fused = fused;
    BatchLaunch& L = b->launch;
    for (int side = 0; side < 3; ++side) {
        std::vector<BatchItem>* by = side == 0 ? rows_by_len : side == 1 ? cols_by_len : rowg_by_len;
        std::vector<BatchItem>& dst = q[side == 0 ? Q_ROW : side == 1 ? Q_COL : Q_ROWG];
        L.nseg[side] = 0;
        for (int k = 0; k < kSizeClasses; ++k) {
            if (by[k].empty()) continue;
            const int g = L.nseg[side]++;
            L.seg_len[side][g] = kLengths[k];
            L.seg_off[side][g] = (int)dst.size();
            L.seg_count[side][g] = (int)by[k].size();
            dst.insert(dst.end(), by[k].begin(), by[k].end());
        }
    }
    SceneBatch* d_scenes = nullptr;
    if ((st = batch_upload(b, hb, &d_scenes)) != CLAMP_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    L.scenes = d_scenes;
    for (int k = 0; k < Q_COUNT; ++k) {
        BatchItem* d = nullptr;
        if ((st = batch_upload(b, q[k], &d)) != CLAMP_OK) {
            batch_free(b);
            delete b;
            return st;
        }
        L.queue[k] = d;
        L.count[k] = (int)q[k].size();
    }
    std::vector<float> beta(kBetaLen);
    for (int k = 0; k < kBetaLen; ++k) beta[k] = (float)(1.0 + 2.0 / std::log((double)k + 2.0));
    float* d_beta = nullptr;
    std::vector<int> zero(1, 0);
    int* d_iter = nullptr;
    if ((st = batch_upload(b, beta, &d_beta)) != CLAMP_OK || (st = batch_upload(b, zero, &d_iter)) != CLAMP_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    L.beta_table = d_beta;
    L.beta_len = kBetaLen;
    L.iter = d_iter;
    L.fault = fault;
    batch_grids(b);
    *out = b;
    return CLAMP_OK;
}

clamp_status clamp_batch_destroy(clamp_batch* batch) {
    if (batch == nullptr) return CLAMP_OK;
    batch_free(batch);
    delete batch;
    return CLAMP_OK;
}

clamp_status clamp_batch_set_iteration(clamp_batch* batch, int32_t done, void* hip_stream) {
    if (batch == nullptr || done < 0) return fail(CLAMP_EINVAL, "bad argument");
    return hip_check(clampk::batch_set_iter(batch->launch.iter, done, static_cast<hipStream_t>(hip_stream)),
                     "clamp_batch_set_iteration");
}

clamp_status clamp_batch_step(clamp_batch* batch, void* hip_stream) {
    if (batch == nullptr) return fail(CLAMP_EINVAL, "batch is NULL");
    return hip_check(batch_run(batch, static_cast<hipStream_t>(hip_stream)), "clamp_batch_step launch");
}

clamp_status clamp_batch_set_tiles(clamp_batch* batch, int32_t row_blocks_per_cu, int32_t col_blocks_per_cu) {
    if (batch == nullptr || row_blocks_per_cu < 0 || col_blocks_per_cu < 0) return fail(CLAMP_EINVAL, "bad argument");
    batch->row_per_cu = row_blocks_per_cu;
    batch->col_per_cu = col_blocks_per_cu;
    batch_grids(batch);
    return CLAMP_OK;
}

clamp_status clamp_batch_autotune(clamp_batch* batch, void* hip_stream, int32_t* chosen) {
    using namespace clampk;
    if (batch == nullptr) return fail(CLAMP_EINVAL, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(CLAMP_EDEVICE, "hipEventCreate failed");
    }
    hipError_t err = hipSuccess;
    auto keep = [&](hipError_t x) {
        if (err == hipSuccess) err = x;
    };
    auto time_stages = [&](std::initializer_list<int> stages) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
            keep(hipEventRecord(e0, st));
            for (int sg : stages) keep(batch_stage(sg, batch->launch, st));
            keep(hipEventRecord(e1, st));
            keep(hipEventSynchronize(e1));
            float ms = 0.f;
            keep(hipEventElapsedTime(&ms, e0, e1));
            if (err == hipSuccess && ms < best) best = ms;
        }
        return best;
    };
    const int cands[] = {0, 2, 4, 8, 16};  // 0: one block per item
    int best_col = batch->col_per_cu, best_row = batch->row_per_cu;
    float tbest = 1e30f;
    for (int c : cands) {
        batch->col_per_cu = c;
        batch_grids(batch);
        const float t = time_stages({BS_COL_INV, BS_COL_FWD});
        if (t < tbest) { tbest = t; best_col = c; }
    }
    batch->col_per_cu = best_col;
    tbest = 1e30f;
    for (int c : cands) {
        batch->row_per_cu = c;
        batch_grids(batch);
        const float t = time_stages({BS_ROW_GRAD});
        if (t < tbest) { tbest = t; best_row = c; }
    }
    batch->row_per_cu = best_row;
    batch_grids(batch);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_check(err, "clamp_batch_autotune");
    if (chosen) {
        chosen[0] = best_row;
        chosen[1] = best_col;
    }
    return CLAMP_OK;
}

clamp_status clamp_batch_capture(clamp_batch* batch, void* hip_stream) {
    if (batch == nullptr) return fail(CLAMP_EINVAL, "batch is NULL");
    if (hip_stream == nullptr) return fail(CLAMP_EINVAL, "capture needs a non-NULL stream");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    clamp_plan* p = const_cast<clamp_plan*>(batch->plan);
    const uint32_t timing = p->timing;
    p->timing = 0u;  // no event records inside the graph
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
        const hipError_t run = batch_run(batch, st);
        e = hipStreamEndCapture(st, &g);
        if (e == hipSuccess) e = run;
    }
    p->timing = timing;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_check(e, "clamp_batch_capture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_check(e, "hipGraphInstantiate");
    }
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    batch->graph = g;
    batch->exec = x;
    return CLAMP_OK;
}

clamp_status clamp_batch_replay(clamp_batch* batch, int32_t iters, void* hip_stream) {
    if (batch == nullptr || iters < 0) return fail(CLAMP_EINVAL, "bad argument");
    if (batch->exec == nullptr) return fail(CLAMP_EINVAL, "nothing captured");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < iters; ++i) {
        const hipError_t e = hipGraphLaunch(batch->exec, st);
        if (e != hipSuccess) return hip_check(e, "hipGraphLaunch");
    }
    return CLAMP_OK;
}

}  // extern "C"
