"""Float64 oracle of the 3D U-Net prior agent (Sec. III-C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Architecture as Sec. III-C describes it:
- three encoder blocks of two 3x3x3 convolutions, each followed by batch
  normalisation and ReLU, with a 2x2x2 max pooling after each block;
- three decoder blocks, each opening with a 2x2x2 stride-2 transposed
  convolution that doubles the resolution, then two convolutions with batch
  normalisation and ReLU;
- a final 3x3x3 convolution to one channel.

Where the paper's figure (not available as text) would decide, this oracle
reads:
- every level is 32 channels wide;
- the encoder output of a level joins the decoder of that level by addition
  (not concatenation), right after the transposed convolution;
- convolutions followed by batch normalisation have no bias; the transposed
  convolutions and the final convolution have one;
- the output is residual, H(x) = x + N(x), as for the CNN prior.

Batch normalisation: training mode normalises with the batch statistics over
(volume, z, y, x) per channel (biased variance, eps 1e-5) and updates running
statistics with momentum 0.1 (unbiased variance); evaluation mode uses the
running statistics, and folds into the preceding convolution (fold_bn).

Layouts as in cnn.py: a volume is [C, D, H, W], a batch [N, C, D, H, W]; a
convolution weight is [27, Cin, Cout]; a transposed-convolution weight is
[8, Cin, Cout] with sub-position s = 4 a + 2 b + c of the output voxel
(2z + a, 2y + b, 2x + c).

`act_round` rounds every stored tensor (pre-activations, activations, skip
sums, gradients) to bfloat16, where the GPU kernels store them.
"""

import numpy as np

from .cnn import bf16_round, conv3d, conv3d_input_grad, conv3d_weight_grad

WIDTH = 32
LEVELS = 3
CONVS = 4 * LEVELS  # two per encoder and two per decoder block
BN_EPS = 1e-5
BN_MOMENTUM = 0.1


def conv_shapes(width=WIDTH):
    """(Cin, Cout) of the 12 batch-normalised convolutions: encoder blocks
    1, 2, 3, then decoder blocks 3, 2, 1 (deepest first), two each."""
    return [(1, width)] + [(width, width)] * (CONVS - 1)


def init_params(rng, width=WIDTH, last_scale=0.0):
    """He-normal convolution weights, BN gamma 1 and beta 0, transposed
    convolutions He-normal with zero bias; the final layer scaled by
    last_scale so that the untrained network starts at H(x) = x."""
    p = {"conv": [], "gamma": [], "beta": [], "up_w": [], "up_b": []}
    for ci, co in conv_shapes(width):
        p["conv"].append(rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci)))
        p["gamma"].append(np.ones(co))
        p["beta"].append(np.zeros(co))
    for _ in range(LEVELS):
        p["up_w"].append(rng.standard_normal((8, width, width)) * np.sqrt(1.0 / width))
        p["up_b"].append(np.zeros(width))
    p["final_w"] = rng.standard_normal((27, width, 1)) * np.sqrt(2.0 / (27 * width)) * last_scale
    p["final_b"] = np.zeros(1)
    return p


def init_stats(width=WIDTH):
    """Running BN statistics: mean 0, variance 1."""
    return {"mean": [np.zeros(width) for _ in range(CONVS)], "var": [np.ones(width) for _ in range(CONVS)]}


def flatten(p):
    """The flat parameter vector in the order of the C interface: per
    convolution W, gamma, beta; per transposed convolution W, b (decoder
    blocks 3, 2, 1); the final W, b."""
    parts = []
    for w, g, b in zip(p["conv"], p["gamma"], p["beta"]):
        parts += [w.ravel(), g, b]
    for w, b in zip(p["up_w"], p["up_b"]):
        parts += [w.ravel(), b]
    parts += [p["final_w"].ravel(), p["final_b"]]
    return np.concatenate(parts)


def unflatten(v, width=WIDTH):
    """Inverse of flatten."""
    p = {"conv": [], "gamma": [], "beta": [], "up_w": [], "up_b": []}
    o = 0
    def take(n, shape):
        nonlocal o
        a = np.asarray(v[o:o + n], dtype=np.float64).reshape(shape)
        o += n
        return a
    for ci, co in conv_shapes(width):
        p["conv"].append(take(27 * ci * co, (27, ci, co)))
        p["gamma"].append(take(co, (co,)))
        p["beta"].append(take(co, (co,)))
    for _ in range(LEVELS):
        p["up_w"].append(take(8 * width * width, (8, width, width)))
        p["up_b"].append(take(width, (width,)))
    p["final_w"] = take(27 * width, (27, width, 1))
    p["final_b"] = take(1, (1,))
    assert o == len(v)
    return p


def param_count(width=WIDTH):
    return sum(27 * ci * co + 2 * co for ci, co in conv_shapes(width)) + LEVELS * (8 * width * width + width) \
        + 27 * width + 1


# ---------------------------------------------------------------------------
# pooling and transposed convolution (per volume, [C, D, H, W])

def maxpool2(x):
    """2x2x2 max pooling (D, H, W even)."""
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).max(axis=(2, 4, 6))


def maxpool2_argmax(x):
    """Sub-position s = 4 a + 2 b + c of the maximum of each window, the
    first one in s order among equal values."""
    C, D, H, W = x.shape
    w = x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).transpose(0, 1, 3, 5, 2, 4, 6).reshape(C, D // 2, H // 2, W // 2, 8)
    return np.argmax(w, axis=-1)


def maxpool2_grad(x, g):
    """Gradient of sum(g * maxpool2(x)) with respect to x: each window's
    gradient goes to its (first) maximum."""
    C, D, H, W = x.shape
    s = maxpool2_argmax(x)
    out = np.zeros((C, D // 2, H // 2, W // 2, 8))
    np.put_along_axis(out, s[..., None], g[..., None], axis=-1)
    return out.reshape(C, D // 2, H // 2, W // 2, 2, 2, 2).transpose(0, 1, 4, 2, 5, 3, 6).reshape(C, D, H, W)


def upconv(x, w, b):
    """out[co, 2z + a, 2y + b, 2x + c] = b[co] + sum_ci x[ci, z, y, x] w[4a + 2b + c, ci, co]."""
    C, D, H, W = x.shape
    out = np.zeros((w.shape[2], 2 * D, 2 * H, 2 * W))
    for s in range(8):
        a, bb, c = s >> 2, (s >> 1) & 1, s & 1
        out[:, a::2, bb::2, c::2] = np.einsum("cdhw,co->odhw", x, w[s])
    return out + b[:, None, None, None]


def upconv_input_grad(g, w):
    """Gradient of sum(g * upconv(x, w, b)) with respect to x."""
    dx = 0.0
    for s in range(8):
        a, bb, c = s >> 2, (s >> 1) & 1, s & 1
        dx = dx + np.einsum("odhw,co->cdhw", g[:, a::2, bb::2, c::2], w[s])
    return dx


def upconv_weight_grad(x, g):
    """Gradient of sum(g * upconv(x, w, b)) with respect to w and b."""
    dw = np.stack([np.einsum("cdhw,odhw->co", x, g[:, s >> 2::2, (s >> 1) & 1::2, s & 1::2]) for s in range(8)])
    return dw, g.sum(axis=(1, 2, 3))


# ---------------------------------------------------------------------------
# batch normalisation over a batch [N, C, D, H, W]

def bn_train(z, gamma, beta):
    """Training-mode batch normalisation; returns (y, xhat, rstd, mean,
    biased variance)."""
    mean = z.mean(axis=(0, 2, 3, 4))
    var = z.var(axis=(0, 2, 3, 4))
    rstd = 1.0 / np.sqrt(var + BN_EPS)
    xhat = (z - mean[None, :, None, None, None]) * rstd[None, :, None, None, None]
    return gamma[None, :, None, None, None] * xhat + beta[None, :, None, None, None], xhat, rstd, mean, var


def bn_train_grad(dy, xhat, gamma, rstd):
    """Gradients of sum(dy * bn_train(z)) with respect to z, gamma and beta."""
    m = dy.shape[0] * np.prod(dy.shape[2:])
    sdy = dy.sum(axis=(0, 2, 3, 4))
    sdyx = (dy * xhat).sum(axis=(0, 2, 3, 4))
    dz = (gamma * rstd)[None, :, None, None, None] * (
        dy - (sdy / m)[None, :, None, None, None] - xhat * (sdyx / m)[None, :, None, None, None])
    return dz, sdyx, sdy


def bn_eval(z, gamma, beta, mean, var):
    s = gamma / np.sqrt(var + BN_EPS)
    return z * s[None, :, None, None, None] + (beta - mean * s)[None, :, None, None, None]


def fold_bn(w, gamma, beta, mean, var):
    """A bias-free convolution followed by evaluation-mode batch
    normalisation, as one convolution: (w s, beta - mean s) with s = gamma /
    sqrt(var + eps) per output channel."""
    s = gamma / np.sqrt(var + BN_EPS)
    return w * s[None, None, :], beta - mean * s


# ---------------------------------------------------------------------------
# the network

def _batch(f, xs, *args):
    return np.stack([f(x, *args) for x in xs])


def forward(xs, p, train, stats=None, act_round=False):
    """H over a batch xs [N, D, H, W] (D, H, W divisible by 8).  train: BN
    with batch statistics (and stats, if given, updated in place); else BN
    with stats.  Returns (H, cache) with every stored tensor for backward."""
    rnd = bf16_round if act_round else (lambda a: a)
    N = xs.shape[0]
    cache = {"layers": [], "enc": [], "pool_in": [], "up_in": [], "skip": []}

    def block(h, idx):
        for k in range(2):
            i = idx + k
            z = rnd(_batch(conv3d, h, p["conv"][i], np.zeros(p["conv"][i].shape[2])))
            if train:
                y, xhat, rstd, mean, var = bn_train(z, p["gamma"][i], p["beta"][i])
                if stats is not None:
                    m = z.shape[0] * np.prod(z.shape[2:])
                    stats["mean"][i] = (1 - BN_MOMENTUM) * stats["mean"][i] + BN_MOMENTUM * mean
                    stats["var"][i] = (1 - BN_MOMENTUM) * stats["var"][i] + BN_MOMENTUM * var * m / (m - 1)
            else:
                y = bn_eval(z, p["gamma"][i], p["beta"][i], stats["mean"][i], stats["var"][i])
                xhat = rstd = None
            a = rnd(np.maximum(y, 0.0))
            cache["layers"].append({"in": h, "xhat": xhat, "rstd": rstd, "out": a})
            h = a
        return h

    h = rnd(xs[:, None])
    for lev in range(LEVELS):
        h = block(h, 2 * lev)
        cache["enc"].append(h)
        cache["pool_in"].append(h)
        h = _batch(maxpool2, h)
    for j in range(LEVELS):
        lev = LEVELS - 1 - j
        cache["up_in"].append(h)
        s = rnd(_batch(upconv, h, p["up_w"][j], p["up_b"][j]) + cache["enc"][lev])
        cache["skip"].append(s)
        h = block(s, 2 * LEVELS + 2 * j)
    cache["final_in"] = h
    n = _batch(conv3d, h, p["final_w"], p["final_b"])[:, 0]
    return xs + n, cache


def forward_folded(xs, fp, act_round=False):
    """Evaluation-mode H with batch normalisation folded into the
    convolutions (fp from fold_params): the form the GPU applies."""
    rnd = bf16_round if act_round else (lambda a: a)
    enc = []
    h = rnd(xs[:, None])

    def block(h, idx):
        for k in range(2):
            w, b = fp["conv"][idx + k]
            h = rnd(np.maximum(_batch(conv3d, h, w, b), 0.0))
        return h

    for lev in range(LEVELS):
        h = block(h, 2 * lev)
        enc.append(h)
        h = _batch(maxpool2, h)
    for j in range(LEVELS):
        h = rnd(_batch(upconv, h, fp["up_w"][j], fp["up_b"][j]) + enc[LEVELS - 1 - j])
        h = block(h, 2 * LEVELS + 2 * j)
    return xs + _batch(conv3d, h, fp["final_w"], fp["final_b"])[:, 0]


def fold_params(p, stats):
    """Convolutions with evaluation-mode BN folded in; other parameters as
    they are."""
    return {"conv": [fold_bn(w, g, b, m, v) for w, g, b, m, v in
                     zip(p["conv"], p["gamma"], p["beta"], stats["mean"], stats["var"])],
            "up_w": p["up_w"], "up_b": p["up_b"], "final_w": p["final_w"], "final_b": p["final_b"]}


def loss_and_grads(xs, ts, p, act_round=False):
    """Mean squared error of training-mode H over the batch and its gradient
    with respect to every parameter (backpropagation written out)."""
    rnd = bf16_round if act_round else (lambda a: a)
    out, c = forward(xs, p, True, act_round=act_round)
    r = out - ts
    n_vox = xs.size
    loss = float(np.sum(r * r)) / n_vox
    gr = {"conv": [None] * CONVS, "gamma": [None] * CONVS, "beta": [None] * CONVS,
          "up_w": [None] * LEVELS, "up_b": [None] * LEVELS}
    g = rnd((2.0 / n_vox) * r[:, None])
    h = c["final_in"]
    dws = [conv3d_weight_grad(a, gg) for a, gg in zip(h, g)]
    gr["final_w"] = sum(d[0] for d in dws)
    gr["final_b"] = sum(d[1] for d in dws)
    g = rnd(_batch(conv3d_input_grad, g, p["final_w"]) * (h > 0))

    def block_back(g, idx):
        """g: gradient at the block output (ReLU mask applied); returns the
        gradient at the block input (the second convolution's input is the
        first one's activation, so it takes that ReLU mask; the block input
        itself is a pooled activation or a skip sum and is masked by the
        caller where it is an activation)."""
        for k in (1, 0):
            i = idx + k
            L = c["layers"][i]
            dz, dgam, dbet = bn_train_grad(g, L["xhat"], p["gamma"][i], L["rstd"])
            dz = rnd(dz)
            gr["gamma"][i], gr["beta"][i] = dgam, dbet
            dws = [conv3d_weight_grad(a, gg) for a, gg in zip(L["in"], dz)]
            gr["conv"][i] = sum(d[0] for d in dws)
            gi = _batch(conv3d_input_grad, dz, p["conv"][i])
            if k == 1:
                gi = gi * (L["in"] > 0)
            g = rnd(gi)
        return g

    g_enc = [0.0] * LEVELS
    for j in range(LEVELS - 1, -1, -1):
        lev = LEVELS - 1 - j
        gs = block_back(g, 2 * LEVELS + 2 * j)  # block input: the skip sum
        g_enc[lev] = g_enc[lev] + gs
        x_in = c["up_in"][j]
        dws = [upconv_weight_grad(a, gg) for a, gg in zip(x_in, gs)]
        gr["up_w"][j] = sum(d[0] for d in dws)
        gr["up_b"][j] = sum(d[1] for d in dws)
        gu = _batch(upconv_input_grad, gs, p["up_w"][j])
        if j == 0:  # the deepest input is the pooled last encoder output
            g_enc[LEVELS - 1] = g_enc[LEVELS - 1] + np.stack(
                [maxpool2_grad(a, gg) for a, gg in zip(c["pool_in"][LEVELS - 1], rnd(gu))])
        else:  # the previous decoder block's output
            g = rnd(gu * (x_in > 0))
    for lev in range(LEVELS - 1, -1, -1):
        g = rnd(g_enc[lev] * (c["enc"][lev] > 0))
        gi = block_back(g, 2 * lev)
        if lev > 0:
            g_enc[lev - 1] = g_enc[lev - 1] + np.stack(
                [maxpool2_grad(a, gg) for a, gg in zip(c["pool_in"][lev - 1], gi)])
    return loss, gr


def denoise(x, p, stats, act_round=False):
    """The prior agent on a volume of any scale (evaluation mode, folded):
    H(x) = x + m N(x / m) with m the mean of x."""
    m = float(np.mean(x))
    fp = fold_params(p, stats)
    out = forward_folded((x / m)[None], fp, act_round)[0]
    return x + m * (out - x / m)
