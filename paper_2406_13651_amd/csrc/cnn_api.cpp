// C ABI of the learned prior agent (include/clamp.h, clamp_cnn_*): parameter
// storage, Adam state, BF16 weight copies, workspace layout and the launch
// sequences of the forward, backward and update passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/clamp.h"
#include "cnn.h"

namespace clampk {
// error reporting shared with api.cpp
clamp_status set_error(clamp_status st, const char* msg);
}

namespace {

using clampk::ConvArgs;
using clampk::WgradArgs;

constexpr int kLayers = 8;
constexpr int kWidth = 32;

int cin_of(int l) { return l == 0 ? 1 : kWidth; }
int cout_of(int l) { return l == kLayers - 1 ? 1 : kWidth; }
int cinp_of(int l) { return l == 0 ? 8 : kWidth; }    // stored channels of the layer input
int coutp_of(int l) { return l == kLayers - 1 ? 8 : kWidth; }  // stored channels of the layer output gradient

long w_offset(int l) {
    long o = 0;
    for (int i = 0; i < l; ++i) o += 27L * cin_of(i) * cout_of(i) + cout_of(i);
    return o;
}
long b_offset(int l) { return w_offset(l) + 27L * cin_of(l) * cout_of(l); }

clamp_status fail(clamp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return clampk::set_error(st, buf);
}

clamp_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return CLAMP_OK;
    return fail(CLAMP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t x8, act[kLayers], out, g8, ga, gb, mean, part, wpart, total;
};

Layout layout(long nvox, bool train) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    if (train) L.x8 = take(nvox * 16);  // evaluation reads the fp32 input in the first layer
    if (train) {
        for (int l = 1; l < kLayers; ++l) L.act[l] = take(nvox * 64);
        L.out = take(nvox * 4);
        L.g8 = take(nvox * 16);
        L.ga = take(nvox * 64);
        L.gb = take(nvox * 64);
        L.wpart = take(clampk::cnn_wgrad_part_bytes());
    } else {
        L.act[1] = take(nvox * 64);
        L.act[2] = take(nvox * 64);
    }
    L.mean = take(16);
    L.part = take((size_t)clampk::cnn_reduce_blocks(nvox) * 8);
    L.total = o;
    return L;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

clamp_status check_dims(int32_t nvol, int32_t nz, int32_t ny, int32_t nx) {
    if (nvol <= 0 || nz <= 0 || ny <= 0 || nx <= 0) return fail(CLAMP_EINVAL, "sizes must be positive");
    if (nx % 32 != 0) return fail(CLAMP_ESHAPE, "nx must be a multiple of 32");
    if ((long)nvol * nz * ny * nx >= (1L << 31)) return fail(CLAMP_ESHAPE, "at most 2^31 voxels per call");
    return CLAMP_OK;
}

}  // namespace

struct clamp_cnn {
    float* params = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    float* clip = nullptr;        // gradient-norm clipping state [2] + norm partial sums
    uint16_t* wq[kLayers] = {};   // forward weight fragments
    uint16_t* wqd[kLayers] = {};  // backward-data weight fragments
    uint16_t* wq1 = nullptr;      // first-layer fragments of the one-channel form (evaluation)
    float* bias32[kLayers] = {};
    int step = 0;
    std::vector<void*> dev;
};

namespace {

template <typename T>
clamp_status alloc(clamp_cnn* c, size_t count, T** out) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CLAMP_ENOMEM : CLAMP_EDEVICE, "hipMalloc: %s",
                                     hipGetErrorString(e));
    c->dev.push_back(p);
    *out = static_cast<T*>(p);
    return CLAMP_OK;
}

hipError_t prep_all(clamp_cnn* c, hipStream_t st) {
    for (int l = 0; l < kLayers; ++l) {
        const hipError_t e = clampk::cnn_prep(c->params + w_offset(l), c->params + b_offset(l), cin_of(l), cout_of(l),
                                              cinp_of(l), coutp_of(l), c->wq[l], l > 0 ? c->wqd[l] : nullptr,
                                              c->bias32[l], st);
        if (e != hipSuccess) return e;
    }
    return clampk::cnn_prep_first(c->params + w_offset(0), c->wq1, st);
}

ConvArgs conv_args(int32_t nvol, int32_t nz, int32_t ny, int32_t nx) {
    ConvArgs a{};
    a.nvol = nvol;
    a.nz = nz;
    a.ny = ny;
    a.nx = nx;
    return a;
}

// Forward pass; stores every activation when `acts` is non-null (training),
// else ping-pongs between two buffers.  Training packs the input into the
// 8-channel bf16 form (x8), which the first layer's weight gradient reads;
// evaluation runs the first layer straight from the fp32 volume.
hipError_t forward(clamp_cnn* c, const float* x, float* out, const float* scale, int32_t nvol, int32_t nz,
                   int32_t ny, int32_t nx, uint16_t* x8, uint16_t* const* acts, uint16_t* ping, uint16_t* pong,
                   hipStream_t st) {
    const long nvox = (long)nvol * nz * ny * nx;
    const bool packed = acts != nullptr;
    hipError_t e = packed ? clampk::cnn_pack(x, scale, nvox, x8, st) : hipSuccess;
    const uint16_t* in = x8;
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
        ConvArgs a = conv_args(nvol, nz, ny, nx);
        a.in = in;
        a.wq = c->wq[l];
        a.bias = c->bias32[l];
        if (l < kLayers - 1) {
            uint16_t* dst = acts ? acts[l + 1] : ((l % 2 == 0) ? ping : pong);
            a.out = dst;
            if (l == 0 && !packed) {
                a.in = nullptr;
                a.xin = x;
                a.scale = scale;
                a.wq = c->wq1;
                e = clampk::cnn_conv(1, clampk::EPI_RELU, a, st);
            } else {
                e = clampk::cnn_conv(cinp_of(l), clampk::EPI_RELU, a, st);
            }
            in = dst;
        } else {
            a.out_f32 = out;
            a.xin = x;
            a.scale = scale;
            e = clampk::cnn_conv(kWidth, clampk::EPI_FINAL, a, st);
        }
    }
    return e;
}

}  // namespace

extern "C" {

clamp_status clamp_cnn_create(clamp_cnn** out) {
    if (out == nullptr) return fail(CLAMP_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(CLAMP_EDEVICE, "no HIP device available");
    clamp_cnn* c = new clamp_cnn();
    clamp_status st = CLAMP_OK;
    if (st == CLAMP_OK) st = alloc(c, CLAMP_CNN_PARAMS, &c->params);
    if (st == CLAMP_OK) st = alloc(c, CLAMP_CNN_PARAMS, &c->m);
    if (st == CLAMP_OK) st = alloc(c, CLAMP_CNN_PARAMS, &c->v);
    if (st == CLAMP_OK) st = alloc(c, CLAMP_CNN_PARAMS, &c->grad);
    if (st == CLAMP_OK) st = alloc(c, clampk::kClipFloats, &c->clip);
    for (int l = 0; l < kLayers && st == CLAMP_OK; ++l) {
        st = alloc(c, clampk::cnn_wq_elems(cinp_of(l)), &c->wq[l]);
        if (st == CLAMP_OK) st = alloc(c, clampk::cnn_wq_elems(coutp_of(l)), &c->wqd[l]);
        if (st == CLAMP_OK) st = alloc(c, 32, &c->bias32[l]);
    }
    if (st == CLAMP_OK) st = alloc(c, 2 * 2 * 32 * 8, &c->wq1);
    if (st == CLAMP_OK) {
        std::vector<float> zero(CLAMP_CNN_PARAMS, 0.f);
        st = clamp_cnn_set_params(c, zero.data());
    }
    if (st != CLAMP_OK) {
        clamp_cnn_destroy(c);
        return st;
    }
    *out = c;
    return CLAMP_OK;
}

clamp_status clamp_cnn_destroy(clamp_cnn* cnn) {
    if (cnn == nullptr) return CLAMP_OK;
    for (void* p : cnn->dev) (void)hipFree(p);
    delete cnn;
    return CLAMP_OK;
}

clamp_status clamp_cnn_set_params(clamp_cnn* cnn, const float* params) {
    if (cnn == nullptr || params == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    for (long i = 0; i < CLAMP_CNN_PARAMS; ++i)
        if (!std::isfinite(params[i])) return fail(CLAMP_EINVAL, "parameter %ld is not finite", i);
    const size_t bytes = sizeof(float) * CLAMP_CNN_PARAMS;
    hipError_t e = hipMemcpy(cnn->params, params, bytes, hipMemcpyHostToDevice);
    std::vector<float> zero(CLAMP_CNN_PARAMS, 0.f);
    if (e == hipSuccess) e = hipMemcpy(cnn->m, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(cnn->v, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(cnn->grad, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(cnn->clip, zero.data(), 2 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = prep_all(cnn, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    cnn->step = 0;
    return hip_check(e, "clamp_cnn_set_params");
}

clamp_status clamp_cnn_get_params(const clamp_cnn* cnn, float* params) {
    if (cnn == nullptr || params == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    return hip_check(hipMemcpy(params, cnn->params, sizeof(float) * CLAMP_CNN_PARAMS, hipMemcpyDeviceToHost),
                     "clamp_cnn_get_params");
}

clamp_status clamp_cnn_workspace_size(int32_t nvol, int32_t nz, int32_t ny, int32_t nx, int32_t train,
                                      size_t* bytes) {
    if (bytes == nullptr) return fail(CLAMP_EINVAL, "bytes is NULL");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    *bytes = layout((long)nvol * nz * ny * nx, train != 0).total;
    return CLAMP_OK;
}

clamp_status clamp_cnn_apply(clamp_cnn* cnn, const float* x, float* out, int32_t nvol, int32_t nz, int32_t ny,
                             int32_t nx, int32_t normalize, void* workspace, void* hip_stream) {
    if (cnn == nullptr || x == nullptr || out == nullptr || workspace == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    if (x == out) return fail(CLAMP_EINVAL, "x and out must not overlap");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const long nvox = (long)nvol * nz * ny * nx;
    const Layout L = layout(nvox, false);
    float* mean = nullptr;
    hipError_t e = hipSuccess;
    if (normalize) {
        mean = at<float>(workspace, L.mean);
        e = clampk::cnn_mean(x, nvox, at<double>(workspace, L.part), mean, s);
    }
    if (e == hipSuccess)
        e = forward(cnn, x, out, mean, nvol, nz, ny, nx, nullptr, nullptr,
                    at<uint16_t>(workspace, L.act[1]), at<uint16_t>(workspace, L.act[2]), s);
    return hip_check(e, "clamp_cnn_apply launch");
}

clamp_status clamp_cnn_grad(clamp_cnn* cnn, const float* x, const float* target, int32_t nvol, int32_t nz,
                            int32_t ny, int32_t nx, double* loss, float* grad, void* workspace, void* hip_stream) {
    if (cnn == nullptr || x == nullptr || target == nullptr || loss == nullptr || workspace == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const long nvox = (long)nvol * nz * ny * nx;
    const Layout L = layout(nvox, true);
    uint16_t* acts[kLayers];
    acts[0] = at<uint16_t>(workspace, L.x8);
    for (int l = 1; l < kLayers; ++l) acts[l] = at<uint16_t>(workspace, L.act[l]);
    float* out = at<float>(workspace, L.out);
    float* g = grad != nullptr ? grad : cnn->grad;
    hipError_t e = forward(cnn, x, out, nullptr, nvol, nz, ny, nx, acts[0], acts, nullptr, nullptr, s);
    uint16_t* g8 = at<uint16_t>(workspace, L.g8);
    if (e == hipSuccess) e = clampk::cnn_loss(out, target, nvox, g8, at<double>(workspace, L.part), loss, s);
    // backward: g holds dL/dz_l with channels coutp_of(l) (8 for the last layer)
    const uint16_t* gl = g8;
    uint16_t* gbuf[2] = {at<uint16_t>(workspace, L.ga), at<uint16_t>(workspace, L.gb)};
    for (int l = kLayers - 1; l >= 0 && e == hipSuccess; --l) {
        WgradArgs wa{};
        wa.nvol = nvol;
        wa.nz = nz;
        wa.ny = ny;
        wa.nx = nx;
        wa.act = acts[l];
        wa.g = gl;
        wa.part = at<float>(workspace, L.wpart);
        e = clampk::cnn_wgrad(cinp_of(l), coutp_of(l), wa, cin_of(l), cout_of(l), g + w_offset(l), g + b_offset(l), s);
        if (e == hipSuccess && l > 0) {
            ConvArgs a = conv_args(nvol, nz, ny, nx);
            a.in = gl;
            a.wq = cnn->wqd[l];
            a.relu_src = acts[l];
            a.out = gbuf[l % 2];
            e = clampk::cnn_conv(coutp_of(l), clampk::EPI_DGRAD, a, s);
            gl = gbuf[l % 2];
        }
    }
    return hip_check(e, "clamp_cnn_grad launch");
}

clamp_status clamp_cnn_adam_step(clamp_cnn* cnn, float lr, void* hip_stream) {
    if (cnn == nullptr) return fail(CLAMP_EINVAL, "cnn is NULL");
    if (!(std::isfinite(lr) && lr > 0.f)) return fail(CLAMP_EINVAL, "lr must be finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    cnn->step += 1;
    hipError_t e =
        clampk::cnn_adam(cnn->params, cnn->m, cnn->v, cnn->grad, CLAMP_CNN_PARAMS, lr, cnn->step, cnn->clip, s);
    if (e == hipSuccess) e = prep_all(cnn, s);
    return hip_check(e, "clamp_cnn_adam_step launch");
}

}  // extern "C"
