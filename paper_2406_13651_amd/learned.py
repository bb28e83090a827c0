"""The learned form of CLAMP: a CNN prior agent trained as a denoiser, used
in place of the fixed prior of Alg. 2.

Training (Sec. III-C trains its prior as an image denoiser on volumes with
10% additive white Gaussian noise, MSE loss, Adam, batch 24, learning rate
decayed by 0.975 every 300 batches, weights kept at the lowest validation
loss).  Here the clean volumes are seeded facet scenes r of the synthetic
recipe instead of rendered models.  The default input comes from the
forward model itself: L looks of r are simulated on the GPU through the
library's aperture operator (speckle and noise drawn there), and the input
is their speckle average (1/L) sum_l |A^H y_l|^2, the initial image of Alg. 2
("speckle").  "clamp" takes instead the consensus image of a
forward-agents-only CLAMP run on such looks after k iterations, k drawn from
{0, 2, 5, 10, 20, 40} (k = 0 is the speckle average) -- the kind of image the
prior agent is handed inside the loop; "awgn" follows the paper's recipe:
r plus white Gaussian noise of standard deviation U[0, 0.1] max(r).  Inputs and targets are scaled to unit mean, and as
a prior agent the network runs in the scale-free form H(w) = w + m N(w / m)
with m = mean(w).

Fallback: the forward-model-only reconstruction (forward agents alone)
replaces the learned form's result when the learned run raises a fault,
produces a non-finite value, or its consensus error rises at `patience`
consecutive checks (the consensus theory of Sec. IV covers proximal priors,
not a trained network).
"""

from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import _clamp as C
from .clamp import ClampGPU, beta_schedule

LAYER_SHAPES = [(1, 32)] + [(32, 32)] * 6 + [(32, 1)]


def init_params(seed=0, last_scale=0.0):
    """He-normal weights and zero biases as one flat float32 vector in the
    library's parameter order; the output layer is scaled by last_scale (0
    starts the network at the identity H(x) = x)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i, (ci, co) in enumerate(LAYER_SHAPES):
        w = rng.standard_normal((27, ci, co)) * math.sqrt(2.0 / (27 * ci))
        if i == len(LAYER_SHAPES) - 1:
            w = w * last_scale
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


class CnnPrior:
    """The trained network on the GPU, with workspaces cached per shape."""

    def __init__(self, params=None, device="cuda"):
        self.dev = torch.device(device)
        self.net = C.clamp_cnn_create()
        C.clamp_cnn_set_params(self.net, init_params() if params is None else params)
        self._ws = {}

    def params(self):
        return C.clamp_cnn_get_params(self.net)

    def set_params(self, p):
        C.clamp_cnn_set_params(self.net, p)

    def workspace(self, shape, train):
        key = (tuple(shape), bool(train))
        if key not in self._ws:
            self._ws[key] = torch.empty(max(C.clamp_cnn_workspace_size(*shape, train), 256), dtype=torch.uint8,
                                        device=self.dev)
        return self._ws[key]

    def apply(self, x, out, normalize=True):
        shape = tuple(x.shape) if x.dim() == 4 else (1,) + tuple(x.shape)
        C.clamp_cnn_apply(self.net, x, out, normalize, self.workspace(shape, False))

    def grad(self, x, t, loss, ws, grad=None):
        C.clamp_cnn_grad(self.net, x, t, loss, ws, grad=grad)

    def adam_step(self, lr):
        C.clamp_cnn_adam_step(self.net, lr)

    def val_loss(self, x, t, ws, vgrad):
        loss = torch.zeros(1, dtype=torch.float64, device=x.device)
        C.clamp_cnn_grad(self.net, x, t, loss, ws, grad=vgrad)
        return float(loss.item())

    n_params = C.CNN_PARAMS


class UnetPrior:
    """The U-Net prior (Sec. III-C's architecture) on the GPU, evaluation mode
    for apply, training mode (batch statistics) for grad; workspaces cached
    per shape.  params() and set_params() carry the parameters together with
    the running statistics of its batch normalisation."""

    n_params = C.UNET_PARAMS

    def __init__(self, params=None, device="cuda"):
        self.dev = torch.device(device)
        self.net = C.clamp_unet_create()
        C.clamp_unet_set_params(self.net, unet_init_params() if params is None else params)
        self._ws = {}

    def params(self):
        return C.clamp_unet_get_params(self.net)

    def set_params(self, p):
        params, stats = p if isinstance(p, tuple) else (p, None)
        C.clamp_unet_set_params(self.net, params, stats)

    def workspace(self, shape, train):
        key = (tuple(shape), bool(train))
        if key not in self._ws:
            self._ws[key] = torch.empty(max(C.clamp_unet_workspace_size(*shape, train), 256), dtype=torch.uint8,
                                        device=self.dev)
        return self._ws[key]

    def apply(self, x, out, normalize=True):
        shape = tuple(x.shape) if x.dim() == 4 else (1,) + tuple(x.shape)
        C.clamp_unet_apply(self.net, x, out, normalize, self.workspace(shape, False))

    def grad(self, x, t, loss, ws, grad=None):
        C.clamp_unet_grad(self.net, x, t, loss, ws, grad=grad)

    def adam_step(self, lr):
        C.clamp_unet_adam_step(self.net, lr)

    def val_loss(self, x, t, ws, vgrad):
        """Evaluation mode (running statistics; the training-mode gradient pass
        would move them): mean squared error of H(x)."""
        out = torch.empty_like(x)
        self.apply(x, out, normalize=False)
        return float(torch.mean((out.double() - t.double()) ** 2).item())


def unet_init_params(seed=0, last_scale=0.0, width=32, levels=3):
    """He-normal convolution and transposed-convolution weights, BN gamma 1
    and beta 0, zero biases, as one flat float32 vector in the library's
    parameter order; the output layer scaled by last_scale."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i in range(4 * levels):
        ci = 1 if i == 0 else width
        parts += [(rng.standard_normal((27, ci, width)) * math.sqrt(2.0 / (27 * ci))).ravel(), np.ones(width),
                  np.zeros(width)]
    for _ in range(levels):
        parts += [(rng.standard_normal((8, width, width)) * math.sqrt(1.0 / width)).ravel(), np.zeros(width)]
    parts += [(rng.standard_normal((27, width, 1)) * math.sqrt(2.0 / (27 * width)) * last_scale).ravel(), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


CLAMP_PAIR_ITERS = (0, 2, 5, 10, 20, 40)


def simulate_looks(g, r, s2, gen):
    """L looks y_l = A (sqrt(r) z_l) + eta_l (eq. forward-model) of the float32
    GPU volume r, simulated on the GPU through the library's aperture operator
    of g (a ClampGPU whose plan has L looks): speckle z_l ~ CN(0, I) (eq.
    g-given-r) and noise eta_l ~ CN(0, s2 I), drawn from the CUDA generator
    gen.  Returns complex64 [L, nz, ny, nx]."""
    L = g.L
    shape = (L,) + tuple(r.shape)
    field = torch.randn(shape, dtype=torch.complex64, device=r.device, generator=gen)
    field *= torch.sqrt(r)
    y = torch.empty_like(field)
    C.clamp_aperture_op(g.plan, 0, C.CLAMP_FWD, field, y, L, g.ws)
    y += math.sqrt(s2) * torch.randn(shape, dtype=torch.complex64, device=r.device, generator=gen)
    return y


def make_pairs(n, seed=0, nz=32, ny=64, nx=64, looks=(4, 8, 16), snr_db=10.0, mode="speckle", noise=0.1,
               device="cuda", sigma2=1e-3):
    """Training pairs (inputs, targets) as float32 [n, nz, ny, nx] GPU tensors,
    both scaled to unit mean.  The targets are seeded facet scenes (drawn on
    the host).  mode "speckle": the input is the speckle average of L looks
    that the forward model simulates on the GPU; "clamp": the consensus image
    of a forward-agents-only CLAMP run (proximal parameter sigma2) on such
    looks after CLAMP_PAIR_ITERS[i % 6] iterations; "awgn": the target plus
    white Gaussian noise of standard deviation U[0, noise] max(target)."""
    import synth
    X = torch.empty((n, nz, ny, nx), dtype=torch.float32, device=device)
    T = torch.empty_like(X)
    gpus = {}
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = None
    if mode in ("speckle", "clamp"):
        gen = torch.Generator(device=device)
        gen.manual_seed(2406_13651 + seed)
    for i in range(n):
        L = int(looks[i % len(looks)])
        facets = int(rng.integers(8, 33))
        spec = synth.SceneSpec("train%d" % i, nx, ny, nz, L, nx / 4.0, snr_db, facets, 0.05, 1, 5)
        r = synth.facet_scene(spec, np.random.Generator(np.random.PCG64(synth.seed_sequence(5, seed * 100_000 + i))))
        t = r / r.mean()
        if mode in ("speckle", "clamp"):
            s2 = synth.noise_variance(r, snr_db)
            if L not in gpus:
                gpus[L] = ClampGPU(nx, ny, nz, L, nx / 4.0, s2, sigma2, with_prior=False, device=device)
            g = gpus[L]
            g.sigma_w2 = s2
            rt = torch.from_numpy(r.astype(np.float32)).to(device)
            g.init(simulate_looks(g, rt, s2, gen))
            k = CLAMP_PAIR_ITERS[i % len(CLAMP_PAIR_ITERS)] if mode == "clamp" else 0
            g.run(k)
            img = g.wbar if k > 0 else g.r[0]
            X[i] = img / img.mean()
            T[i] = rt / rt.mean()
        else:
            sd = rng.uniform(0.0, noise) * t.max()
            x = t + sd * rng.standard_normal(t.shape)
            X[i] = torch.from_numpy(x.astype(np.float32)).to(device)
            T[i] = torch.from_numpy(t.astype(np.float32)).to(device)
    torch.cuda.synchronize()
    return X, T


def train(prior, X, T, epochs=10, batch=24, lr=1e-3, decay=0.975, decay_every=300, val_frac=0.1, seed=0,
          log=None):
    """Adam on the MSE, learning rate lr * decay^(step // decay_every); keeps
    the parameters of the lowest validation loss.  Returns a history dict."""
    n = X.shape[0]
    n_val = max(1, int(round(n * val_frac)))
    n_tr = n - n_val
    shape = (batch,) + tuple(X.shape[1:])
    ws = prior.workspace(shape, True)
    loss = torch.zeros(1, dtype=torch.float64, device=X.device)
    vgrad = torch.empty(prior.n_params, dtype=torch.float32, device=X.device)
    rng = np.random.Generator(np.random.PCG64(seed))
    best = (math.inf, prior.params())
    hist = {"train": [], "val": [], "seconds": 0.0, "steps": 0, "voxels": 0}
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(n_tr)
        tl = []
        for b0 in range(0, n_tr - batch + 1, batch):
            idx = torch.from_numpy(order[b0:b0 + batch]).to(X.device)
            xb, tb = X.index_select(0, idx).contiguous(), T.index_select(0, idx).contiguous()
            prior.grad(xb, tb, loss, ws)
            prior.adam_step(lr * decay ** (step // decay_every))
            step += 1
            tl.append(loss)
            loss = torch.zeros(1, dtype=torch.float64, device=X.device)
        vl = []
        for b0 in range(n_tr, n - batch + 1, batch):
            xb, tb = X[b0:b0 + batch].contiguous(), T[b0:b0 + batch].contiguous()
            vl.append(prior.val_loss(xb, tb, ws, vgrad))
        if not vl:  # fewer validation volumes than a batch: evaluate them padded with training volumes
            xb = torch.cat([X[n_tr:], X[:batch - n_val]]).contiguous()
            tb = torch.cat([T[n_tr:], T[:batch - n_val]]).contiguous()
            vl.append(prior.val_loss(xb, tb, ws, vgrad))
        tr = float(np.mean([x.item() for x in tl])) if tl else math.nan
        va = float(np.mean(vl))
        hist["train"].append(tr)
        hist["val"].append(va)
        if va < best[0]:
            best = (va, prior.params())
        if log:
            log("epoch %d train %.5f val %.5f" % (ep, tr, va))
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    hist["steps"] = step
    hist["voxels"] = step * batch * int(np.prod(X.shape[1:]))
    prior.set_params(best[1])
    hist["best_val"] = best[0]
    return hist


class LearnedClamp(ClampGPU):
    """CLAMP with the CNN prior agent (Alg. 2 with H = the trained network)."""

    def __init__(self, *args, prior=None, **kw):
        kw["with_prior"] = True
        super().__init__(*args, **kw)
        self.cnn = prior

    def prior(self):
        self.cnn.apply(self.w[self.L], self.r[self.L], normalize=True)


def nrmse(rhat, r_true):
    """Volumetric ||b rhat - r|| / ||r|| with the least-squares scale b (Sec. V-A)."""
    a = rhat.double().flatten()
    b = r_true.double().flatten()
    s = float(a @ b / (a @ a))
    return float(torch.linalg.norm(s * a - b) / torch.linalg.norm(b))


def run_with_fallback(make_learned, make_plain, y, iters, r_true=None, check_every=5, patience=3):
    """Run the learned form; on a fault, a non-finite value or a consensus
    error rising at `patience` consecutive checks, return the forward-only
    reconstruction instead.  Returns (wbar, info)."""
    g = make_learned()
    g.init(y)
    rising, last = 0, math.inf
    info = {"fallback": False, "conv": []}
    for k in range(1, iters + 1):
        g.iterate()
        if k % check_every == 0 or k == iters:
            ce = g.conv_err()
            info["conv"].append(ce)
            bad = int(g.fault.item()) != 0 or not math.isfinite(ce) or not bool(torch.isfinite(g.wbar).all())
            rising = rising + 1 if ce > last else 0
            last = ce
            if bad or rising >= patience:
                info["fallback"] = True
                info["reason"] = "fault" if bad else "consensus error rising"
                break
    if info["fallback"]:
        f = make_plain()
        f.init(y)
        f.run(iters)
        out = f.wbar
    else:
        out = g.wbar
    if r_true is not None:
        info["nrmse"] = nrmse(out, r_true)
    return out, info
