"""GPU parity of the learned prior's BF16 MFMA kernels (forward, weight and
input gradients) against the float64 oracle run with the same bfloat16
weights and the same bfloat16 rounding of stored activations and gradients."""

import numpy as np
import pytest

from oracle import cnn as ocnn
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch  # noqa: F401
    import paper_2406_13651_amd._clamp as C
    return C


def flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def bf16_params(params):
    """Weights rounded to bfloat16 as the GPU stores them; biases stay float32."""
    return [(ocnn.bf16_round(w), np.asarray(b, np.float32).astype(np.float64)) for w, b in params]


def _setup(C, seed=0, last_scale=0.5, shape=(2, 6, 8, 32)):
    import torch
    rng = np.random.default_rng(seed)
    params = ocnn.init_params(rng, last_scale=last_scale)
    for i, (w, b) in enumerate(params):
        if i < len(params) - 1 or last_scale != 0.0:
            b += 0.05 * rng.standard_normal(b.shape)
    params = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in params]
    net = C.clamp_cnn_create()
    C.clamp_cnn_set_params(net, flat(params))
    x = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    t = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    return net, params, x, t, torch


def test_param_count_and_round_trip(C):
    net, params, x, t, torch = _setup(C)
    assert flat(params).size == C.CNN_PARAMS
    np.testing.assert_array_equal(C.clamp_cnn_get_params(net), flat(params))


# shapes: one ragged row tile; several row and x tiles with ragged rows and
# a ragged last range chunk; a taller volume with full 8-slice range chunks
SHAPES = [(2, 6, 8, 32), (1, 11, 37, 64), (1, 20, 16, 32)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(C, shape):
    net, params, x, t, torch = _setup(C, shape=shape)
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_apply(net, xt, out, False, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    p16 = bf16_params(params)
    for i in range(x.shape[0]):
        ref, _ = ocnn.forward(x[i].astype(np.float64), p16, act_round=True)
        # compare the learned part N(x) = H(x) - x
        err = rel_l2(got[i] - x[i], ref - x[i])
        assert report("cnn forward N(x) %s volume %d" % (shape, i), err, 5e-3) <= 5e-3


def test_normalized_apply_matches_oracle_and_scales(C):
    net, params, x, t, torch = _setup(C, seed=1)
    xv = 0.03 * x[:1]
    xt = torch.from_numpy(xv).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(C.clamp_cnn_workspace_size(*xv.shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_apply(net, xt, out, True, ws)
    torch.cuda.synchronize()
    ref = ocnn.denoise(xv[0].astype(np.float64), bf16_params(params), act_round=True)
    err = rel_l2(out.cpu().numpy()[0] - xv[0], ref - xv[0])
    assert report("cnn normalized apply", err, 5e-3) <= 5e-3


def test_zero_output_layer_is_identity(C):
    net, params, x, t, torch = _setup(C, last_scale=0.0)
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_apply(net, xt, out, True, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), x)


@pytest.mark.parametrize("shape", [(2, 4, 8, 32), (1, 9, 21, 64)])
def test_gradients_match_oracle(C, shape):
    net, params, x, t, torch = _setup(C, seed=2, shape=shape)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(C.CNN_PARAMS, dtype=torch.float32, device="cuda")
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, True), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_grad(net, xt, tt, loss, ws, grad=grad)
    torch.cuda.synchronize()
    ref_loss, ref_grads = ocnn.loss_and_grads(x.astype(np.float64), t.astype(np.float64), bf16_params(params),
                                              act_round=True)
    assert abs(loss.item() - ref_loss) <= 1e-3 * ref_loss
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for l, (w, b) in enumerate(params):
        gw = g[off:off + w.size].reshape(w.shape)
        off += w.size
        gb = g[off:off + b.size]
        off += b.size
        ew = rel_l2(gw, ref_grads[l][0])
        eb = rel_l2(gb, ref_grads[l][1])
        report("cnn dW layer %d %s" % (l, shape), ew, 2e-2)
        report("cnn db layer %d %s" % (l, shape), eb, 2e-2)
        assert ew <= 2e-2 and eb <= 2e-2


def test_adam_steps_reduce_loss(C):
    net, params, x, t, torch = _setup(C, seed=3, last_scale=0.1, shape=(4, 4, 8, 32))
    # a target the output bias alone can reach: H(x) = x + 0.1
    t = x + 0.1
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t.astype(np.float32)).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, True), dtype=torch.uint8, device="cuda")
    losses = []
    for _ in range(30):
        C.clamp_cnn_grad(net, xt, tt, loss, ws)
        C.clamp_cnn_adam_step(net, 1e-2)
        torch.cuda.synchronize()
        losses.append(loss.item())
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]


def test_adam_gradient_clipping_matches_oracle(C):
    """Adam steps with gradient-norm clipping against the oracle's clipped
    rule (oracle.cnn.adam_step_clipped), fed with the gradients the library
    computes: five ordinary steps, one with the target scaled by 100 (its
    gradient norm far above 3 times the running norm: clipped), two more."""
    from oracle import cnn as ocnn
    net, params, x, t, torch = _setup(C, seed=5, shape=(2, 4, 8, 32))
    xt = torch.from_numpy(x).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, True), dtype=torch.uint8, device="cuda")
    g = torch.empty(C.CNN_PARAMS, dtype=torch.float32, device="cuda")
    p = [(C.clamp_cnn_get_params(net).astype(np.float64), np.zeros(0))]
    state, lr = {}, 1e-3
    clipped = []
    for k, sc in enumerate([1, 1, 1, 1, 1, 100, 1, 1], start=1):
        tt = torch.from_numpy((t * sc).astype(np.float32)).cuda()
        C.clamp_cnn_grad(net, xt, tt, loss, ws, grad=g)  # read out
        gk = g.cpu().numpy().astype(np.float64)
        C.clamp_cnn_grad(net, xt, tt, loss, ws)  # kept for the step
        C.clamp_cnn_adam_step(net, lr)
        run_before = state.get("run_norm", 0.0)
        p = ocnn.adam_step_clipped(p, [(gk, np.zeros(0))], state, lr)
        clipped.append(run_before > 0.0 and np.linalg.norm(gk) > 3.0 * run_before)
        np.testing.assert_allclose(C.clamp_cnn_get_params(net), p[0][0], rtol=1e-5, atol=1e-7)
    print("clipped steps", clipped)
    assert clipped[5]


def test_adam_skips_non_finite_gradient(C):
    """A gradient with a non-finite norm leaves the parameters unchanged; the
    next finite step updates them."""
    net, params, x, t, torch = _setup(C, seed=6, shape=(1, 4, 8, 32))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(C.clamp_cnn_workspace_size(*x.shape, True), dtype=torch.uint8, device="cuda")
    tt = torch.from_numpy(t).cuda()
    before = C.clamp_cnn_get_params(net)
    xn = x.copy()
    xn[0, 1, 2, 3] = np.nan
    C.clamp_cnn_grad(net, torch.from_numpy(xn).cuda(), tt, loss, ws)
    C.clamp_cnn_adam_step(net, 1e-3)
    np.testing.assert_array_equal(C.clamp_cnn_get_params(net), before)
    C.clamp_cnn_grad(net, torch.from_numpy(x).cuda(), tt, loss, ws)
    C.clamp_cnn_adam_step(net, 1e-3)
    after = C.clamp_cnn_get_params(net)
    assert np.all(np.isfinite(after)) and not np.array_equal(after, before)


def test_forward_full_size_sampled(C):
    """At the full evaluation size (64 x 256 x 256, the launch configuration of
    the learned-form benchmark) sampled outputs match the oracle run on the
    receptive field around each sample (8 layers: +-8 voxels, clipped at the
    volume boundary, where both sides pad with zeros)."""
    import torch
    shape = (1, 64, 256, 256)
    rng = np.random.default_rng(7)
    params = ocnn.init_params(rng, last_scale=0.5)
    for w, b in params:
        b += 0.05 * rng.standard_normal(b.shape)
    params = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in params]
    net = C.clamp_cnn_create()
    C.clamp_cnn_set_params(net, flat(params))
    x = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(C.clamp_cnn_workspace_size(*shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_apply(net, xt, out, False, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0].astype(np.float64)
    p16 = bf16_params(params)
    samples = [(31, 100, 77), (0, 0, 0), (63, 255, 255), (7, 16, 32), (40, 15, 31), (8, 200, 128), (32, 128, 128),
               (63, 0, 255), (1, 254, 1)]
    diffs, resid = [], []
    for c in samples:
        lo = [max(0, c[d] - 8) for d in range(3)]
        hi = [min(shape[1 + d], c[d] + 9) for d in range(3)]
        crop = x[0, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].astype(np.float64)
        ref, _ = ocnn.forward(crop, p16, act_round=True)
        r = ref[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]] - x[0][c]
        diffs.append(got[c] - x[0][c] - r)
        resid.append(r)
    # bf16 rounding flips move an output by a few 1e-4 whatever its size: the
    # error is taken against the RMS of the sampled residuals N(x)
    err = float(np.max(np.abs(diffs)) / np.sqrt(np.mean(np.square(resid))))
    assert report("cnn forward 64x256x256 sampled voxels", err, 2e-2) <= 2e-2
