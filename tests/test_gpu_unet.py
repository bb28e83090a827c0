"""GPU parity of the U-Net prior agent (clamp_unet_*) against the float64
oracle (oracle/unet.py) run with the same bf16 roundings: evaluation mode,
batch normalisation folded into the convolutions."""

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import unet as U
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    from paper_2406_13651_amd import _clamp as C
    return C


def _params(seed, last_scale=0.5):
    rng = np.random.default_rng(seed)
    p = U.init_params(rng, last_scale=last_scale)
    for i in range(U.CONVS):
        p["gamma"][i] = rng.uniform(0.5, 1.5, 32)
        p["beta"][i] = 0.1 * rng.standard_normal(32)
    for j in range(U.LEVELS):
        p["up_b"][j] = 0.05 * rng.standard_normal(32)
    p["final_b"] = np.array([0.02])
    stats = {"mean": [0.2 * rng.standard_normal(32) for _ in range(U.CONVS)],
             "var": [rng.uniform(0.5, 2.0, 32) for _ in range(U.CONVS)]}
    # parameters as the GPU holds them (float32)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    p = U.unflatten(f32(U.flatten(p)))
    stats = {k: [f32(a) for a in v] for k, v in stats.items()}
    return p, stats


def _stats_vector(stats):
    return np.concatenate([np.concatenate([m, v]) for m, v in zip(stats["mean"], stats["var"])]).astype(np.float32)


def _oracle_folded(p, stats):
    """The evaluation weights as the GPU forms them: folded in float32, then
    rounded to bf16 (biases stay float32)."""
    fp = U.fold_params(p, stats)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    fp["conv"] = [(ocnn.bf16_round(f32(w)), f32(b)) for w, b in fp["conv"]]
    fp["up_w"] = [ocnn.bf16_round(w) for w in fp["up_w"]]
    fp["final_w"] = ocnn.bf16_round(fp["final_w"])
    return fp


def _make(C, p, stats):
    net = C.clamp_unet_create()
    C.clamp_unet_set_params(net, U.flatten(p), _stats_vector(stats))
    return net


def _apply(C, net, x, normalize=False):
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    out = torch.empty_like(xt)
    ws = torch.empty(C.clamp_unet_workspace_size(*xt.shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_unet_apply(net, xt, out, normalize, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def test_round_trip_of_parameters_and_statistics(C):
    p, stats = _params(0)
    net = _make(C, p, stats)
    got_p, got_s = C.clamp_unet_get_params(net)
    np.testing.assert_array_equal(got_p, U.flatten(p).astype(np.float32))
    np.testing.assert_array_equal(got_s, _stats_vector(stats))


# shapes: the smallest (one tile per level, the bottom 1 x 1 x 16); ragged
# 16-row tiles at every level with two volumes; several x tiles per level
SHAPES = [(1, 8, 8, 128), (2, 16, 24, 128), (1, 8, 32, 256)]


def _check_against_budget(name, got, ref, ref64, x):
    """bf16 storage of the 17 tensors along the network's path (input, 13
    convolution outputs, 3 skip sums) puts the rounded oracle itself ~5e-3
    from the unrounded one; the kernels round at the same points but from
    fp32 sums, which flips some of those roundings.  So the GPU must be no
    farther from the unrounded oracle than 1.5 times the rounded oracle is
    (plus 1e-4), and within 1e-2 of the rounded oracle."""
    budget = rel_l2(ref - x, ref64 - x)
    err = rel_l2(got - x, ref - x)
    err64 = rel_l2(got - x, ref64 - x)
    assert report(name + " vs rounded oracle", err, 1e-2) <= 1e-2
    bound = 1.5 * budget + 1e-4
    assert report(name + " vs unrounded oracle", err64, bound) <= bound


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(C, shape):
    p, stats = _params(1)
    net = _make(C, p, stats)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.05, 1.0, shape)
    x32 = x.astype(np.float32).astype(np.float64)
    got = _apply(C, net, x32)
    fp = _oracle_folded(p, stats)
    ref = U.forward_folded(x32, fp, act_round=True)
    ref64 = U.forward_folded(x32, fp, act_round=False)
    for v in range(shape[0]):
        _check_against_budget("unet forward N(x) %s volume %d" % (shape, v), got[v], ref[v], ref64[v], x32[v])


def test_zero_output_layer_is_identity(C):
    p, stats = _params(3, last_scale=0.0)
    p["final_b"] = np.zeros(1)
    net = _make(C, p, stats)
    x = np.random.default_rng(4).uniform(0.05, 1.0, (1, 8, 16, 128)).astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(_apply(C, net, x), x)


def test_normalized_apply_matches_oracle(C):
    p, stats = _params(5)
    net = _make(C, p, stats)
    x = np.random.default_rng(6).uniform(0.5, 20.0, (1, 8, 16, 128)).astype(np.float32).astype(np.float64)
    got = _apply(C, net, x, normalize=True)
    m = float(np.float32(x.mean()))
    xs = (x / m).astype(np.float32).astype(np.float64)
    fp = _oracle_folded(p, stats)
    ref = m * U.forward_folded(xs, fp, act_round=True)
    ref64 = m * U.forward_folded(xs, fp, act_round=False)
    _check_against_budget("unet normalized apply", got, ref, ref64, x)


def test_full_size_properties(C):
    """At the evaluation size 64 x 256 x 256: a zero output layer returns x
    exactly; the scale-free form is equivariant to the input scale; the
    output is finite."""
    import torch
    shape = (1, 64, 256, 256)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(8)
    x = torch.rand(shape, device="cuda", generator=gen) * 0.95 + 0.05
    out = torch.empty_like(x)
    out2 = torch.empty_like(x)
    ws = torch.empty(C.clamp_unet_workspace_size(*shape, False), dtype=torch.uint8, device="cuda")
    p0, stats = _params(7, last_scale=0.0)
    p0["final_b"] = np.zeros(1)
    net = _make(C, p0, stats)
    C.clamp_unet_apply(net, x, out, True, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    p, stats = _params(7)
    net = _make(C, p, stats)
    C.clamp_unet_apply(net, x, out, True, ws)
    C.clamp_unet_apply(net, x * 4.0, out2, True, ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    err = float(torch.linalg.norm(out2 - 4.0 * out) / torch.linalg.norm(4.0 * out - 4.0 * x))
    assert report("unet full-size scale equivariance", err, 1e-5) <= 1e-5


def test_errors(C):
    import torch
    net = C.clamp_unet_create()
    x = torch.ones((1, 8, 16, 128), device="cuda")
    ws = torch.empty(C.clamp_unet_workspace_size(1, 8, 16, 128, False), dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        C.clamp_unet_apply(net, x, x, False, ws)
    with pytest.raises(RuntimeError):
        C.clamp_unet_workspace_size(1, 8, 16, 96, False)
    bad = U.flatten(U.init_params(np.random.default_rng(0)))
    bad[5] = np.nan
    with pytest.raises(RuntimeError):
        C.clamp_unet_set_params(net, bad)


def _grad_groups(v):
    """Gradient vector split by parameter group (flat layout of the oracle)."""
    q = U.unflatten(np.asarray(v, dtype=np.float64))
    out = {}
    for i in range(U.CONVS):
        out["conv%d" % i] = q["conv"][i]
        out["gamma%d" % i] = q["gamma"][i]
        out["beta%d" % i] = q["beta"][i]
    for j in range(U.LEVELS):
        out["up_w%d" % j] = q["up_w"][j]
        out["up_b%d" % j] = q["up_b"][j]
    out["final_w"] = q["final_w"]
    out["final_b"] = q["final_b"]
    return out


@pytest.mark.parametrize("shape", [(2, 8, 8, 128), (1, 16, 16, 128)])
def test_training_gradients_and_running_statistics(C, shape):
    """Training mode (batch statistics) against the oracle's backward pass
    with the same bf16 roundings: the loss, every parameter group's gradient,
    and the running statistics after the call."""
    import torch
    p, _ = _params(9, last_scale=1.0)
    p16 = U.unflatten(U.flatten(p))
    for i in range(U.CONVS):
        p16["conv"][i] = ocnn.bf16_round(p16["conv"][i])
    for j in range(U.LEVELS):
        p16["up_w"][j] = ocnn.bf16_round(p16["up_w"][j])
    p16["final_w"] = ocnn.bf16_round(p16["final_w"])
    net = C.clamp_unet_create()
    C.clamp_unet_set_params(net, U.flatten(p))
    rng = np.random.default_rng(10)
    x = rng.uniform(0.05, 1.0, shape).astype(np.float32).astype(np.float64)
    t = rng.uniform(0.05, 1.0, shape).astype(np.float32).astype(np.float64)
    xt, tt = torch.from_numpy(x.astype(np.float32)).cuda(), torch.from_numpy(t.astype(np.float32)).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(C.UNET_PARAMS, dtype=torch.float32, device="cuda")
    ws = torch.empty(C.clamp_unet_workspace_size(*shape, True), dtype=torch.uint8, device="cuda")
    C.clamp_unet_grad(net, xt, tt, loss, ws, grad=g)
    torch.cuda.synchronize()
    ref_loss, ref = U.loss_and_grads(x, t, p16, act_round=True)
    _, ref64 = U.loss_and_grads(x, t, p16, act_round=False)
    assert abs(loss.item() - ref_loss) <= 1e-2 * ref_loss
    got = _grad_groups(g.cpu().numpy())
    rnd = _grad_groups(U.flatten(ref))
    unr = _grad_groups(U.flatten(ref64))
    # bf16 storage of the gradients, amplified by the batch normalisation
    # backward (dy - mean(dy) - xhat mean(dy xhat) cancels), moves the rounded
    # oracle's gradients from the unrounded ones by 1e-3 (output layer) to
    # ~0.3 (first encoder block); the kernels round at the same points from
    # fp32 sums, so some values land on the neighbouring bf16 value, and the
    # GPU and the rounded oracle differ by 0.14 to 0.25 in the early groups
    # (two rounding sequences, each ~0.3 from the unrounded gradient; worst
    # 0.250, beta4 at 2x8x8x128, when the bound was set).  Two checks per
    # parameter group: against the rounded oracle, a fixed bound of 0.35 (a
    # wrong sign or a dropped term gives O(1)); against the unrounded oracle,
    # no farther than 1.5 times the rounded oracle is, plus 1e-3.
    worst, worst_rnd = 0.0, 0.0
    for k in got:
        budget = rel_l2(rnd[k], unr[k])
        err = rel_l2(got[k], unr[k])
        err_rnd = rel_l2(got[k], rnd[k])
        print("UNETGRAD %s %-8s vs unrounded %.3e budget %.3e vs rounded %.3e"
              % ("x".join(map(str, shape)), k, err, budget, err_rnd), flush=True)
        worst = max(worst, err / (1.5 * budget + 1e-3))
        worst_rnd = max(worst_rnd, err_rnd)
    assert report("unet training gradients vs rounded oracle (worst group)", worst_rnd, 0.35) <= 0.35
    assert report("unet training gradients (worst group / its bound)", worst, 1.0) <= 1.0
    # running statistics: momentum 0.1 from (0, 1) towards the batch statistics
    stats = U.init_stats()
    U.forward(x, p16, True, stats, act_round=True)
    _, got_s = C.clamp_unet_get_params(net)
    ref_s = _stats_vector(stats)
    err = rel_l2(got_s.astype(np.float64), ref_s.astype(np.float64))
    assert report("unet running statistics after one step", err, 1e-3) <= 1e-3


def test_adam_steps_reduce_loss(C):
    """Training-mode steps through clamp_unet_grad and clamp_unet_adam_step
    towards a target the output bias alone can reach (H(x) = x + 0.1)."""
    import torch
    p, _ = _params(11, last_scale=0.1)
    net = _make(C, p, {"mean": [np.zeros(32)] * U.CONVS, "var": [np.ones(32)] * U.CONVS})
    rng = np.random.default_rng(12)
    x = rng.uniform(0.05, 1.0, (4, 8, 16, 128)).astype(np.float32)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(x + 0.1).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(C.clamp_unet_workspace_size(*x.shape, True), dtype=torch.uint8, device="cuda")
    losses = []
    for _ in range(30):
        C.clamp_unet_grad(net, xt, tt, loss, ws)
        C.clamp_unet_adam_step(net, 1e-2)
        torch.cuda.synchronize()
        losses.append(loss.item())
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    # the running statistics moved away from (0, 1) and stay finite
    _, stats = C.clamp_unet_get_params(net)
    assert np.all(np.isfinite(stats)) and not np.allclose(stats[32:64], 1.0)
