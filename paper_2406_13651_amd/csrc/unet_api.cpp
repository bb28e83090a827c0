// C ABI of the U-Net prior agent (include/clamp.h, clamp_unet_*): parameter
// and running-statistics storage, the evaluation-mode weights (batch
// normalisation folded into the convolutions), workspace layout and the
// launch sequence of the forward pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "../../include/clamp.h"
#include "cnn.h"
#include "unet.h"

namespace clampk {
clamp_status set_error(clamp_status st, const char* msg);
}

namespace {

using clampk::ConvArgs;

constexpr int kWidth = 32;
constexpr int kLevels = 3;
constexpr int kConvs = 4 * kLevels;  // encoder blocks 1, 2, 3, then decoder blocks 3, 2, 1; two each

int cin_of(int l) { return l == 0 ? 1 : kWidth; }
int cinp_of(int l) { return l == 0 ? 8 : kWidth; }  // stored channels of the convolution input

// flat parameter layout: per convolution W [27][cin][32], gamma [32], beta
// [32]; per transposed convolution W [8][32][32], b [32]; final W [27][32][1], b [1]
long conv_w(int l) {
    long o = 0;
    for (int i = 0; i < l; ++i) o += 27L * cin_of(i) * kWidth + 2 * kWidth;
    return o;
}
long conv_gamma(int l) { return conv_w(l) + 27L * cin_of(l) * kWidth; }
long conv_beta(int l) { return conv_gamma(l) + kWidth; }
long up_w(int j) { return conv_w(kConvs) + j * (8L * kWidth * kWidth + kWidth); }
long up_b(int j) { return up_w(j) + 8L * kWidth * kWidth; }
long final_w() { return up_w(kLevels); }
long final_b() { return final_w() + 27L * kWidth; }

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

// Workspace of the evaluation pass (V voxels at level 0, V / 8^k at level k):
// levels 0, 1 and 2: e and two buffers; level 3: the pooled bottom (the
// first convolution reads the fp32 input itself).
struct Layout {
    size_t e[kLevels], t[kLevels][2], p3, mean, part, total;
};

Layout layout(long nvox) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    long v = nvox;
    for (int k = 0; k < kLevels; ++k, v /= 8) {
        L.e[k] = take(v * 64);
        L.t[k][0] = take(v * 64);
        L.t[k][1] = take(v * 64);
    }
    L.p3 = take(v * 64);
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
    if (nz % 8 != 0 || ny % 8 != 0) return fail(CLAMP_ESHAPE, "nz and ny must be multiples of 8");
    if (nx % 128 != 0) return fail(CLAMP_ESHAPE, "nx must be a multiple of 128");
    if ((long)nvol * nz * ny * nx >= (1L << 31)) return fail(CLAMP_ESHAPE, "at most 2^31 voxels per call");
    return CLAMP_OK;
}

}  // namespace

struct clamp_unet {
    float* params = nullptr;  // CLAMP_UNET_PARAMS
    float* stats = nullptr;   // CLAMP_UNET_STATS: per BN layer mean [32], variance [32]
    // evaluation-mode weights
    float* wfold = nullptr;             // fp32 scratch [27][32][32] of one folded convolution
    float* bfold = nullptr;             // fp32 scratch [32]
    uint16_t* wq[kConvs + 1] = {};      // forward fragments of the 12 convolutions and the final one
    uint16_t* wq1 = nullptr;            // the first convolution in the one-channel form (k_conv_first)
    float* bias32[kConvs + 1] = {};     // padded biases (folded for the 12)
    uint16_t* wup[kLevels] = {};        // transposed-convolution fragments (forward)
    bool eval_ready = false;
    // training
    float* m = nullptr;                 // Adam moments and gradient (CLAMP_UNET_PARAMS)
    float* v = nullptr;
    float* grad = nullptr;
    float* clip = nullptr;              // gradient-norm clipping state [2] + norm partial sums
    float* zero32 = nullptr;            // zero bias of the batch-normalised convolutions
    float* bscratch = nullptr;          // [32] bias gradients the bias-free convolutions discard
    uint16_t* wqt[kConvs] = {};         // forward fragments of the unfolded convolutions
    uint16_t* wqd[kConvs + 1] = {};     // backward-data fragments (and the final layer's)
    float* bias_t = nullptr;            // [32] padded zero bias of the unfolded convolutions
    uint16_t* wupt[kLevels] = {};       // transposed-convolution fragments (backward data)
    bool train_ready = false;
    int step = 0;
    std::vector<void*> dev;
};

namespace {

template <typename T>
clamp_status alloc(clamp_unet* u, size_t count, T** out) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? CLAMP_ENOMEM : CLAMP_EDEVICE, "hipMalloc: %s",
                                     hipGetErrorString(e));
    u->dev.push_back(p);
    *out = static_cast<T*>(p);
    return CLAMP_OK;
}

// Evaluation-mode weights from the parameters and running statistics.
hipError_t prep_eval(clamp_unet* u, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < kConvs && e == hipSuccess; ++l) {
        const float* mean = u->stats + l * 2 * kWidth;
        e = clampk::unet_fold_bn(u->params + conv_w(l), u->params + conv_gamma(l), u->params + conv_beta(l), mean,
                                 mean + kWidth, cin_of(l), u->wfold, u->bfold, st);
        if (e == hipSuccess)
            e = clampk::cnn_prep(u->wfold, u->bfold, cin_of(l), kWidth, cinp_of(l), kWidth, u->wq[l], nullptr,
                                 u->bias32[l], st);
        // the first convolution also in the one-channel form, before the
        // next fold overwrites the scratch
        if (e == hipSuccess && l == 0) e = clampk::cnn_prep_first(u->wfold, u->wq1, st);
    }
    for (int j = 0; j < kLevels && e == hipSuccess; ++j) e = clampk::unet_prep_up(u->params + up_w(j), 0, u->wup[j], st);
    if (e == hipSuccess)
        e = clampk::cnn_prep(u->params + final_w(), u->params + final_b(), kWidth, 1, kWidth, 8, u->wq[kConvs],
                             nullptr, u->bias32[kConvs], st);
    return e;
}

ConvArgs conv_args(int32_t nvol, int32_t nz, int32_t ny, int32_t nx) {
    ConvArgs a{};
    a.nvol = nvol;
    a.nz = nz;
    a.ny = ny;
    a.nx = nx;
    return a;
}

// Evaluation-mode forward pass.
hipError_t forward_eval(clamp_unet* u, const float* x, float* out, const float* scale, int32_t nvol, int32_t nz,
                        int32_t ny, int32_t nx, void* ws, const Layout& L, hipStream_t st) {
    int dz[kLevels + 1], dy[kLevels + 1], dx[kLevels + 1];
    for (int k = 0; k <= kLevels; ++k) {
        dz[k] = nz >> k;
        dy[k] = ny >> k;
        dx[k] = nx >> k;
    }
    auto conv = [&](int l, int k, const uint16_t* in, uint16_t* o) {
        ConvArgs a = conv_args(nvol, dz[k], dy[k], dx[k]);
        a.in = in;
        a.wq = u->wq[l];
        a.bias = u->bias32[l];
        a.out = o;
        return clampk::cnn_conv(cinp_of(l), clampk::EPI_RELU, a, st);
    };
    uint16_t* e_[kLevels];
    uint16_t* t[kLevels][2];
    for (int k = 0; k < kLevels; ++k) {
        e_[k] = at<uint16_t>(ws, L.e[k]);
        t[k][0] = at<uint16_t>(ws, L.t[k][0]);
        t[k][1] = at<uint16_t>(ws, L.t[k][1]);
    }
    uint16_t* p3 = at<uint16_t>(ws, L.p3);
    // encoder: block k reads the pooled output of block k - 1 (held in
    // t[k][1]); the first convolution reads the fp32 volume itself
    hipError_t e = hipSuccess;
    const uint16_t* in = nullptr;
    for (int k = 0; k < kLevels && e == hipSuccess; ++k) {
        if (k == 0) {
            ConvArgs a = conv_args(nvol, nz, ny, nx);
            a.xin = x;
            a.scale = scale;
            a.wq = u->wq1;
            a.bias = u->bias32[0];
            a.out = t[0][0];
            e = clampk::cnn_conv(1, clampk::EPI_RELU, a, st);
        } else {
            e = conv(2 * k, k, in, t[k][0]);
        }
        if (e == hipSuccess) e = conv(2 * k + 1, k, t[k][0], e_[k]);
        uint16_t* pooled = k + 1 < kLevels ? t[k + 1][1] : p3;
        if (e == hipSuccess) e = clampk::unet_pool(e_[k], pooled, nvol, dz[k], dy[k], dx[k], st);
        in = pooled;
    }
    // decoder: block of level k = 2, 1, 0 (transposed convolution j = 2 - k)
    for (int j = 0; j < kLevels && e == hipSuccess; ++j) {
        const int k = kLevels - 1 - j;
        clampk::UpArgs a{};
        a.nvol = nvol;
        a.nz = dz[k + 1];
        a.ny = dy[k + 1];
        a.nx = dx[k + 1];
        a.in = in;
        a.wf = u->wup[j];
        a.bias = u->params + up_b(j);
        a.skip = e_[k];
        a.out = t[k][0];
        e = clampk::unet_upconv(a, st);
        const int l = 2 * kLevels + 2 * j;
        if (e == hipSuccess) e = conv(l, k, t[k][0], t[k][1]);
        if (e == hipSuccess) e = conv(l + 1, k, t[k][1], t[k][0]);
        in = t[k][0];
    }
    if (e == hipSuccess) {
        ConvArgs a = conv_args(nvol, nz, ny, nx);
        a.in = in;
        a.wq = u->wq[kConvs];
        a.bias = u->bias32[kConvs];
        a.out_f32 = out;
        a.xin = x;
        a.scale = scale;
        e = clampk::cnn_conv(kWidth, clampk::EPI_FINAL, a, st);
    }
    return e;
}

// Training-mode weights: the unfolded convolutions and every backward-data
// fragment (the final layer's forward fragments are shared with evaluation).
hipError_t prep_train(clamp_unet* u, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < kConvs && e == hipSuccess; ++l)
        e = clampk::cnn_prep(u->params + conv_w(l), u->zero32, cin_of(l), kWidth, cinp_of(l), kWidth, u->wqt[l],
                             l > 0 ? u->wqd[l] : nullptr, u->bias_t, st);
    for (int j = 0; j < kLevels && e == hipSuccess; ++j) {
        e = clampk::unet_prep_up(u->params + up_w(j), 0, u->wup[j], st);
        if (e == hipSuccess) e = clampk::unet_prep_up(u->params + up_w(j), 1, u->wupt[j], st);
    }
    if (e == hipSuccess)
        e = clampk::cnn_prep(u->params + final_w(), u->params + final_b(), kWidth, 1, kWidth, 8, u->wq[kConvs],
                             u->wqd[kConvs], u->bias32[kConvs], st);
    return e;
}

int level_of(int l) { return l < 2 * kLevels ? l / 2 : (4 * kLevels - 1 - l) / 2; }

// Workspace of a training step: every tensor the backward pass reads.
struct TrainLayout {
    size_t x8, out, g8, z[kConvs], a[kConvs], p[kLevels + 1], s[kLevels], gs[kLevels], G[kLevels][3], gp3;
    size_t bn, coef, chanpart, uppart, wpart, part, total;
};

TrainLayout train_layout(long nvox) {
    TrainLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    long nv[kLevels + 1];
    for (int k = 0; k <= kLevels; ++k) nv[k] = nvox >> (3 * k);
    L.x8 = take(nvox * 16);
    L.out = take(nvox * 4);
    L.g8 = take(nvox * 16);
    for (int l = 0; l < kConvs; ++l) {
        L.z[l] = take(nv[level_of(l)] * 64);
        L.a[l] = take(nv[level_of(l)] * 64);
    }
    for (int k = 1; k <= kLevels; ++k) L.p[k] = take(nv[k] * 64);
    for (int k = 0; k < kLevels; ++k) {
        L.s[k] = take(nv[k] * 64);
        L.gs[k] = take(nv[k] * 64);
        for (int i = 0; i < 3; ++i) L.G[k][i] = take(nv[k] * 64);
    }
    L.gp3 = take(nv[kLevels] * 64);
    L.bn = take(kConvs * 4 * 32 * sizeof(float));  // per convolution: mean, rstd, A, B
    L.coef = take(3 * 32 * sizeof(float));
    L.chanpart = take(clampk::unet_chan_part_bytes());
    L.uppart = take(clampk::unet_upwgrad_part_bytes());
    L.wpart = take(clampk::cnn_wgrad_part_bytes());
    L.part = take((size_t)clampk::cnn_reduce_blocks(nvox) * 8);
    L.total = o;
    return L;
}

struct Trainer {
    clamp_unet* u;
    void* ws;
    const TrainLayout& L;
    int32_t nvol;
    int dz[kLevels + 1], dy[kLevels + 1], dx[kLevels + 1];
    float* g;  // gradient vector
    hipStream_t st;

    template <typename T>
    T* buf(size_t off) const { return at<T>(ws, off); }
    long nvox(int k) const { return (long)nvol * dz[k] * dy[k] * dx[k]; }
    float* bn(int l, int which) const { return buf<float>(L.bn) + (l * 4 + which) * 32; }

    ConvArgs conv(int k) const {
        ConvArgs a = conv_args(nvol, dz[k], dy[k], dx[k]);
        return a;
    }

    // z = W * in (no bias), batch statistics, a = ReLU(BN(z)); updates the running statistics
    hipError_t conv_bn(int l, const uint16_t* in) {
        const int k = level_of(l);
        ConvArgs a = conv(k);
        a.in = in;
        a.wq = u->wqt[l];
        a.out = buf<uint16_t>(L.z[l]);
        hipError_t e = clampk::cnn_conv(cinp_of(l), clampk::EPI_RAW, a, st);
        int blocks = 0;
        double* part = buf<double>(L.chanpart);
        if (e == hipSuccess) e = clampk::unet_chan_sums(0, a.out, nullptr, nullptr, nullptr, nvox(k), part, &blocks, st);
        float* rmean = u->stats + l * 2 * kWidth;
        if (e == hipSuccess)
            e = clampk::unet_chan_finalize(0, part, blocks, nvox(k), u->params + conv_gamma(l), u->params + conv_beta(l),
                                           bn(l, 0), bn(l, 1), bn(l, 2), bn(l, 3), nullptr, rmean, rmean + kWidth,
                                           nullptr, nullptr, st);
        if (e == hipSuccess)
            e = clampk::unet_affine(a.out, nullptr, bn(l, 2), nullptr, bn(l, 3), 1, nvox(k), buf<uint16_t>(L.a[l]), st);
        return e;
    }

    // Backward of batch normalisation and convolution l: gy (gradient at the
    // ReLU output, already masked) -> dz -> weight, gamma and beta gradients;
    // the input gradient into gin (masked by relu_src, or raw when NULL; not
    // formed when gin is NULL).
    hipError_t conv_bn_back(int l, const uint16_t* gy, uint16_t* dzb, const uint16_t* in, const uint16_t* relu_src,
                            uint16_t* gin) {
        const int k = level_of(l);
        int blocks = 0;
        double* part = buf<double>(L.chanpart);
        float* c = buf<float>(L.coef);
        const uint16_t* z = buf<uint16_t>(L.z[l]);
        hipError_t e = clampk::unet_chan_sums(1, gy, z, bn(l, 0), bn(l, 1), nvox(k), part, &blocks, st);
        if (e == hipSuccess)
            e = clampk::unet_chan_finalize(1, part, blocks, nvox(k), u->params + conv_gamma(l), nullptr, bn(l, 0),
                                           bn(l, 1), c, c + 32, c + 64, nullptr, nullptr, g + conv_gamma(l),
                                           g + conv_beta(l), st);
        if (e == hipSuccess) e = clampk::unet_affine(gy, z, c, c + 32, c + 64, 0, nvox(k), dzb, st);
        if (e == hipSuccess) {
            clampk::WgradArgs wa{};
            wa.nvol = nvol;
            wa.nz = dz[k];
            wa.ny = dy[k];
            wa.nx = dx[k];
            wa.act = in;
            wa.g = dzb;
            wa.part = buf<float>(L.wpart);
            e = clampk::cnn_wgrad(cinp_of(l), kWidth, wa, cin_of(l), kWidth, g + conv_w(l), u->bscratch, st);
        }
        if (e == hipSuccess && gin != nullptr) {
            ConvArgs a = conv(k);
            a.in = dzb;
            a.wq = u->wqd[l];
            a.relu_src = relu_src;
            a.out = gin;
            e = clampk::cnn_conv(kWidth, relu_src ? clampk::EPI_DGRAD : clampk::EPI_RAW, a, st);
        }
        return e;
    }
};

hipError_t train_step(clamp_unet* u, const float* x, const float* target, int32_t nvol, int32_t nz, int32_t ny,
                      int32_t nx, double* loss, float* g, void* ws, const TrainLayout& L, hipStream_t st) {
    Trainer T{u, ws, L, nvol, {}, {}, {}, g, st};
    for (int k = 0; k <= kLevels; ++k) {
        T.dz[k] = nz >> k;
        T.dy[k] = ny >> k;
        T.dx[k] = nx >> k;
    }
    auto B = [&](size_t off) { return T.buf<uint16_t>(off); };
    const long nvox = (long)nvol * nz * ny * nx;
    hipError_t e = clampk::cnn_pack(x, nullptr, nvox, B(L.x8), st);
    // forward, batch statistics
    const uint16_t* in = B(L.x8);
    for (int k = 0; k < kLevels && e == hipSuccess; ++k) {
        e = T.conv_bn(2 * k, in);
        if (e == hipSuccess) e = T.conv_bn(2 * k + 1, B(L.a[2 * k]));
        if (e == hipSuccess) e = clampk::unet_pool(B(L.a[2 * k + 1]), B(L.p[k + 1]), nvol, T.dz[k], T.dy[k], T.dx[k], st);
        in = B(L.p[k + 1]);
    }
    for (int j = 0; j < kLevels && e == hipSuccess; ++j) {
        const int k = kLevels - 1 - j;
        clampk::UpArgs a{};
        a.nvol = nvol;
        a.nz = T.dz[k + 1];
        a.ny = T.dy[k + 1];
        a.nx = T.dx[k + 1];
        a.in = in;
        a.wf = u->wup[j];
        a.bias = u->params + up_b(j);
        a.skip = B(L.a[2 * k + 1]);
        a.out = B(L.s[k]);
        e = clampk::unet_upconv(a, st);
        const int l = 2 * kLevels + 2 * j;
        if (e == hipSuccess) e = T.conv_bn(l, B(L.s[k]));
        if (e == hipSuccess) e = T.conv_bn(l + 1, B(L.a[l]));
        in = B(L.a[l + 1]);
    }
    float* out = T.buf<float>(L.out);
    if (e == hipSuccess) {
        ConvArgs a = T.conv(0);
        a.in = in;
        a.wq = u->wq[kConvs];
        a.bias = u->bias32[kConvs];
        a.out_f32 = out;
        a.xin = x;
        a.scale = nullptr;
        e = clampk::cnn_conv(kWidth, clampk::EPI_FINAL, a, st);
    }
    uint16_t* g8 = B(L.g8);
    if (e == hipSuccess) e = clampk::cnn_loss(out, target, nvox, g8, T.buf<double>(L.part), loss, st);
    // backward: final layer
    const uint16_t* d1 = B(L.a[4 * kLevels - 1]);
    if (e == hipSuccess) {
        clampk::WgradArgs wa{};
        wa.nvol = nvol;
        wa.nz = nz;
        wa.ny = ny;
        wa.nx = nx;
        wa.act = d1;
        wa.g = g8;
        wa.part = T.buf<float>(L.wpart);
        e = clampk::cnn_wgrad(kWidth, 8, wa, kWidth, 1, g + final_w(), g + final_b(), st);
    }
    uint16_t* gcur = B(L.G[0][0]);
    if (e == hipSuccess) {
        ConvArgs a = T.conv(0);
        a.in = g8;
        a.wq = u->wqd[kConvs];
        a.relu_src = d1;
        a.out = gcur;
        e = clampk::cnn_conv(8, clampk::EPI_DGRAD, a, st);
    }
    // decoder blocks 1, 2, 3 (j = 2, 1, 0), each: second convolution, first
    // convolution (its input gradient is the skip gradient gs), transposed
    // convolution (coarse input gradient, masked by the coarse input)
    for (int j = kLevels - 1; j >= 0 && e == hipSuccess; --j) {
        const int k = kLevels - 1 - j, l1 = 2 * kLevels + 2 * j, l2 = l1 + 1;
        uint16_t* G1 = B(L.G[k][1]);
        uint16_t* G2 = B(L.G[k][2]);
        e = T.conv_bn_back(l2, gcur, G1, B(L.a[l1]), B(L.a[l1]), G2);
        if (e == hipSuccess) e = T.conv_bn_back(l1, G2, G1, B(L.s[k]), nullptr, B(L.gs[k]));
        const uint16_t* xin = j == 0 ? B(L.p[kLevels]) : B(L.a[l1 - 1]);
        clampk::UpBwdArgs ub{};
        ub.nvol = nvol;
        ub.nz = T.dz[k + 1];
        ub.ny = T.dy[k + 1];
        ub.nx = T.dx[k + 1];
        ub.g = B(L.gs[k]);
        ub.wt = u->wupt[j];
        ub.relu_src = xin;
        ub.in = xin;
        ub.out = j == 0 ? B(L.gp3) : B(L.G[k + 1][0]);
        if (e == hipSuccess) e = clampk::unet_upconv_wgrad(ub, T.buf<float>(L.uppart), g + up_w(j), st);
        int blocks = 0;
        double* part = T.buf<double>(L.chanpart);
        if (e == hipSuccess) e = clampk::unet_chan_sums(0, B(L.gs[k]), nullptr, nullptr, nullptr, T.nvox(k), part, &blocks, st);
        if (e == hipSuccess)
            e = clampk::unet_chan_finalize(2, part, blocks, T.nvox(k), nullptr, nullptr, nullptr, nullptr, nullptr,
                                           nullptr, nullptr, nullptr, nullptr, g + up_b(j), nullptr, st);
        if (e == hipSuccess) e = clampk::unet_upconv_dgrad(ub, st);
        gcur = ub.out;
    }
    // encoder blocks 3, 2, 1: pooling backward with the skip gradient, then
    // the two convolutions (the first one's input gradient goes to the next
    // finer level's pooling backward)
    for (int k = kLevels - 1; k >= 0 && e == hipSuccess; --k) {
        uint16_t* G0 = B(L.G[k][0]);
        uint16_t* G1 = B(L.G[k][1]);
        uint16_t* G2 = B(L.G[k][2]);
        e = clampk::unet_pool_bwd(B(L.a[2 * k + 1]), gcur, B(L.gs[k]), G0, nvol, T.dz[k], T.dy[k], T.dx[k], st);
        if (e == hipSuccess) e = T.conv_bn_back(2 * k + 1, G0, G1, B(L.a[2 * k]), B(L.a[2 * k]), G2);
        const uint16_t* in0 = k == 0 ? B(L.x8) : B(L.p[k]);
        if (e == hipSuccess) e = T.conv_bn_back(2 * k, G2, G1, in0, nullptr, k == 0 ? nullptr : G0);
        gcur = G0;
    }
    return e;
}

}  // namespace

extern "C" {

clamp_status clamp_unet_create(clamp_unet** out) {
    if (out == nullptr) return fail(CLAMP_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(CLAMP_EDEVICE, "no HIP device available");
    clamp_unet* u = new clamp_unet();
    clamp_status st = alloc(u, CLAMP_UNET_PARAMS, &u->params);
    if (st == CLAMP_OK) st = alloc(u, CLAMP_UNET_STATS, &u->stats);
    if (st == CLAMP_OK) st = alloc(u, 27 * kWidth * kWidth, &u->wfold);
    if (st == CLAMP_OK) st = alloc(u, kWidth, &u->bfold);
    for (int l = 0; l <= kConvs && st == CLAMP_OK; ++l) {
        st = alloc(u, clampk::cnn_wq_elems(l == kConvs ? kWidth : cinp_of(l)), &u->wq[l]);
        if (st == CLAMP_OK) st = alloc(u, 32, &u->bias32[l]);
    }
    if (st == CLAMP_OK) st = alloc(u, 2 * 2 * 32 * 8, &u->wq1);
    for (int j = 0; j < kLevels && st == CLAMP_OK; ++j) st = alloc(u, 8 * 2 * 64 * 8, &u->wup[j]);
    if (st == CLAMP_OK) st = alloc(u, CLAMP_UNET_PARAMS, &u->m);
    if (st == CLAMP_OK) st = alloc(u, CLAMP_UNET_PARAMS, &u->v);
    if (st == CLAMP_OK) st = alloc(u, CLAMP_UNET_PARAMS, &u->grad);
    if (st == CLAMP_OK) st = alloc(u, clampk::kClipFloats, &u->clip);
    if (st == CLAMP_OK) st = alloc(u, 32, &u->zero32);
    if (st == CLAMP_OK) st = alloc(u, 32, &u->bscratch);
    if (st == CLAMP_OK) st = alloc(u, 32, &u->bias_t);
    for (int l = 0; l < kConvs && st == CLAMP_OK; ++l) {
        st = alloc(u, clampk::cnn_wq_elems(cinp_of(l)), &u->wqt[l]);
        if (st == CLAMP_OK && l > 0) st = alloc(u, clampk::cnn_wq_elems(kWidth), &u->wqd[l]);
    }
    if (st == CLAMP_OK) st = alloc(u, clampk::cnn_wq_elems(8), &u->wqd[kConvs]);
    for (int j = 0; j < kLevels && st == CLAMP_OK; ++j) st = alloc(u, 8 * 2 * 64 * 8, &u->wupt[j]);
    if (st == CLAMP_OK) {
        std::vector<float> zero(CLAMP_UNET_PARAMS, 0.f);
        st = clamp_unet_set_params(u, zero.data(), nullptr);
    }
    if (st != CLAMP_OK) {
        clamp_unet_destroy(u);
        return st;
    }
    *out = u;
    return CLAMP_OK;
}

clamp_status clamp_unet_destroy(clamp_unet* u) {
    if (u == nullptr) return CLAMP_OK;
    for (void* p : u->dev) (void)hipFree(p);
    delete u;
    return CLAMP_OK;
}

clamp_status clamp_unet_set_params(clamp_unet* u, const float* params, const float* stats) {
    if (u == nullptr || params == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    for (long i = 0; i < CLAMP_UNET_PARAMS; ++i)
        if (!std::isfinite(params[i])) return fail(CLAMP_EINVAL, "parameter %ld is not finite", i);
    std::vector<float> s(CLAMP_UNET_STATS);
    for (int l = 0; l < kConvs; ++l)
        for (int c = 0; c < kWidth; ++c) {
            const float m = stats ? stats[l * 2 * kWidth + c] : 0.f;
            const float v = stats ? stats[l * 2 * kWidth + kWidth + c] : 1.f;
            if (!std::isfinite(m) || !(v >= 0.f) || !std::isfinite(v))
                return fail(CLAMP_EINVAL, "running statistics of layer %d channel %d are invalid", l, c);
            s[l * 2 * kWidth + c] = m;
            s[l * 2 * kWidth + kWidth + c] = v;
        }
    const size_t bytes = sizeof(float) * CLAMP_UNET_PARAMS;
    std::vector<float> zero(CLAMP_UNET_PARAMS, 0.f);
    hipError_t e = hipMemcpy(u->params, params, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->stats, s.data(), sizeof(float) * CLAMP_UNET_STATS, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->m, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->v, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->grad, zero.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->clip, zero.data(), 2 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->zero32, zero.data(), 32 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = prep_eval(u, nullptr);
    if (e == hipSuccess) e = prep_train(u, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    u->eval_ready = u->train_ready = e == hipSuccess;
    u->step = 0;
    return hip_check(e, "clamp_unet_set_params");
}

clamp_status clamp_unet_get_params(const clamp_unet* u, float* params, float* stats) {
    if (u == nullptr) return fail(CLAMP_EINVAL, "NULL argument");
    hipError_t e = hipSuccess;
    if (params != nullptr) e = hipMemcpy(params, u->params, sizeof(float) * CLAMP_UNET_PARAMS, hipMemcpyDeviceToHost);
    if (e == hipSuccess && stats != nullptr)
        e = hipMemcpy(stats, u->stats, sizeof(float) * CLAMP_UNET_STATS, hipMemcpyDeviceToHost);
    return hip_check(e, "clamp_unet_get_params");
}

clamp_status clamp_unet_workspace_size(int32_t nvol, int32_t nz, int32_t ny, int32_t nx, int32_t train,
                                       size_t* bytes) {
    if (bytes == nullptr) return fail(CLAMP_EINVAL, "bytes is NULL");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    const long nvox = (long)nvol * nz * ny * nx;
    *bytes = train != 0 ? train_layout(nvox).total : layout(nvox).total;
    return CLAMP_OK;
}

clamp_status clamp_unet_apply(clamp_unet* u, const float* x, float* out, int32_t nvol, int32_t nz, int32_t ny,
                              int32_t nx, int32_t normalize, void* workspace, void* hip_stream) {
    if (u == nullptr || x == nullptr || out == nullptr || workspace == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    if (x == out) return fail(CLAMP_EINVAL, "x and out must not overlap");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const long nvox = (long)nvol * nz * ny * nx;
    const Layout L = layout(nvox);
    hipError_t e = hipSuccess;
    if (!u->eval_ready) {
        e = prep_eval(u, s);
        u->eval_ready = e == hipSuccess;
    }
    float* mean = nullptr;
    if (e == hipSuccess && normalize) {
        mean = at<float>(workspace, L.mean);
        e = clampk::cnn_mean(x, nvox, at<double>(workspace, L.part), mean, s);
    }
    if (e == hipSuccess) e = forward_eval(u, x, out, mean, nvol, nz, ny, nx, workspace, L, s);
    return hip_check(e, "clamp_unet_apply launch");
}

clamp_status clamp_unet_grad(clamp_unet* u, const float* x, const float* target, int32_t nvol, int32_t nz,
                             int32_t ny, int32_t nx, double* loss, float* grad, void* workspace, void* hip_stream) {
    if (u == nullptr || x == nullptr || target == nullptr || loss == nullptr || workspace == nullptr)
        return fail(CLAMP_EINVAL, "NULL argument");
    clamp_status st = check_dims(nvol, nz, ny, nx);
    if (st != CLAMP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const TrainLayout L = train_layout((long)nvol * nz * ny * nx);
    hipError_t e = hipSuccess;
    if (!u->train_ready) {
        e = prep_train(u, s);
        u->train_ready = e == hipSuccess;
    }
    if (e == hipSuccess)
        e = train_step(u, x, target, nvol, nz, ny, nx, loss, grad != nullptr ? grad : u->grad, workspace, L, s);
    u->eval_ready = false;  // the running statistics moved
    return hip_check(e, "clamp_unet_grad launch");
}

clamp_status clamp_unet_adam_step(clamp_unet* u, float lr, void* hip_stream) {
    if (u == nullptr) return fail(CLAMP_EINVAL, "unet is NULL");
    if (!(std::isfinite(lr) && lr > 0.f)) return fail(CLAMP_EINVAL, "lr must be finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    u->step += 1;
    hipError_t e = clampk::cnn_adam(u->params, u->m, u->v, u->grad, CLAMP_UNET_PARAMS, lr, u->step, u->clip, s);
    if (e == hipSuccess) e = prep_train(u, s);
    u->train_ready = e == hipSuccess;
    u->eval_ready = false;
    return hip_check(e, "clamp_unet_adam_step launch");
}

}  // extern "C"
