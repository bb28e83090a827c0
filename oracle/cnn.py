"""Float64 oracle of the learned prior agent: a residual 3D CNN denoiser.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's prior agent is a 3D U-Net trained as an image denoiser (Sec.
III-C); the learned form here is a smaller residual network: 8 convolutions
of 3x3x3 taps (1 -> 32, six 32 -> 32, 32 -> 1) with biases, zero padding,
ReLU after the first seven, and output H(x) = x + N(x).  Training minimises
the mean squared error to the target (Sec. III-C), and the same Adam update
is written out here for reference, with the gradient-norm clipping the
library's optimiser adds to it.

Layouts: a volume is [C, D, H, W]; a weight is [27, Cin, Cout] with tap t =
9 (dz + 1) + 3 (dy + 1) + (dx + 1) for offsets dz, dy, dx in {-1, 0, 1}; the
layer computes y[co, v] = b[co] + sum_t sum_ci x[ci, v + off(t)] W[t, ci, co].

`act_round` rounds every stored activation and gradient to bfloat16 (round to
nearest even), the storage precision of the GPU kernels, so that the oracle
and the GPU take the same roundings; weights are rounded by the caller.
"""

import numpy as np

WIDTH = 32
LAYERS = 8
OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    nan = np.isnan(f)
    out = (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def layer_shapes(width=WIDTH, layers=LAYERS):
    """(Cin, Cout) of each layer."""
    return [(1, width)] + [(width, width)] * (layers - 2) + [(width, 1)]


def init_params(rng, width=WIDTH, layers=LAYERS, last_scale=0.0):
    """He-normal weights, zero biases; the last layer scaled by last_scale so
    that the untrained network starts at the identity H(x) = x."""
    params = []
    for i, (ci, co) in enumerate(layer_shapes(width, layers)):
        w = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        if i == layers - 1:
            w = w * last_scale
        params.append((w, np.zeros(co)))
    return params


def _shift(x, off):
    """x[:, v + off] with zeros outside the volume."""
    dz, dy, dx = off
    C, D, H, W = x.shape
    out = np.zeros_like(x)
    zs, ze = max(0, -dz), min(D, D - dz)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[:, zs:ze, ys:ye, xs:xe] = x[:, zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv3d(x, w, b):
    """y[co, v] = b[co] + sum_t sum_ci x[ci, v + off(t)] w[t, ci, co]."""
    y = np.zeros((w.shape[2],) + x.shape[1:])
    for t, off in enumerate(OFFSETS):
        y += np.einsum("cdhw,co->odhw", _shift(x, off), w[t])
    return y + b[:, None, None, None]


def conv3d_input_grad(g, w):
    """Gradient of sum(g * conv3d(x, w, b)) with respect to x."""
    dx = np.zeros((w.shape[1],) + g.shape[1:])
    for t, off in enumerate(OFFSETS):
        dx += _shift(np.einsum("odhw,co->cdhw", g, w[t]), tuple(-o for o in off))
    return dx


def conv3d_weight_grad(x, g):
    """Gradient of sum(g * conv3d(x, w, b)) with respect to w and b."""
    dw = np.stack([np.einsum("cdhw,odhw->co", _shift(x, off), g) for off in OFFSETS])
    return dw, g.sum(axis=(1, 2, 3))


def forward(x, params, act_round=False):
    """H(x) = x + N(x) for one volume x[D, H, W]; returns (H(x), activations)."""
    rnd = bf16_round if act_round else (lambda a: a)
    a = rnd(x[None])
    acts = [a]
    for i, (w, b) in enumerate(params):
        z = conv3d(a, w, b)
        if i < len(params) - 1:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
        else:
            out = x + z[0]
    return out, acts


def loss_and_grads(xs, ts, params, act_round=False):
    """Mean squared error of H over a batch (xs, ts: [N, D, H, W]) and its
    gradients with respect to every weight and bias (backpropagation written
    out layer by layer)."""
    rnd = bf16_round if act_round else (lambda a: a)
    n_vox = xs.size
    loss = 0.0
    grads = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for x, t in zip(xs, ts):
        out, acts = forward(x, params, act_round)
        r = out - t
        loss += float(np.sum(r * r))
        g = rnd((2.0 / n_vox) * r[None])
        for i in range(len(params) - 1, -1, -1):
            w, _ = params[i]
            dw, db = conv3d_weight_grad(acts[i], g)
            grads[i] = (grads[i][0] + dw, grads[i][1] + db)
            if i > 0:
                g = rnd(conv3d_input_grad(g, w) * (acts[i] > 0))
    return loss / n_vox, grads


def _adam_moments(params, grads, state, t, lr, b1, b2, eps):
    """Adam's moment updates and bias-corrected step at step count t."""
    new = []
    for i, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        upd = []
        for j, (p, g) in enumerate(((w, gw), (b, gb))):
            m = state.get(("m", i, j), np.zeros_like(p))
            v = state.get(("v", i, j), np.zeros_like(p))
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            state[("m", i, j)] = m
            state[("v", i, j)] = v
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            upd.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(upd))
    return new


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected first and second moments)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    return _adam_moments(params, grads, state, t, lr, b1, b2, eps)


def adam_step_clipped(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8, clip=3.0, avg_weight=0.05):
    """Adam with the training safeguards of the learned prior (not in the
    paper, which trains with plain Adam): the gradient of all parameters,
    taken as one vector, is scaled down to norm `clip` times a running
    average of the past (scaled) gradient norms when its norm exceeds that;
    the first step is not scaled and starts the average, which afterwards
    moves by `avg_weight` towards each step's scaled norm.  A gradient whose
    norm is not finite changes neither the parameters, the moments nor the
    average; the step count of the bias correction still advances."""
    t = state.get("t", 0) + 1
    state["t"] = t
    sq = 0.0
    for gw, gb in grads:
        sq += float(np.sum(gw * gw)) + float(np.sum(gb * gb))
    norm = np.sqrt(sq)
    if not np.isfinite(norm):
        return [(w.copy(), b.copy()) for w, b in params]
    run = state.get("run_norm", 0.0)
    if run == 0.0:
        scale = 1.0
        run = norm
    else:
        cap = clip * run
        scale = min(1.0, cap / norm) if norm > 0.0 else 1.0
        run = (1.0 - avg_weight) * run + avg_weight * min(norm, cap)
    state["run_norm"] = run
    scaled = [(scale * gw, scale * gb) for gw, gb in grads]
    return _adam_moments(params, scaled, state, t, lr, b1, b2, eps)


def denoise(x, params, act_round=False):
    """The prior agent on a volume of any scale: H(x) = x + m N(x / m) with m
    the mean of x, so the network sees inputs of unit mean."""
    m = float(np.mean(x))
    out, _ = forward(x / m, params, act_round)
    return x + m * (out - x / m)
