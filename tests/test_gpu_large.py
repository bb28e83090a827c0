"""The large configuration (512x512x128, 32 looks, SNR 5 dB, four objects) in
the launch configuration of the large benchmark: one forward-agent
application against the oracle on the first and the last look, the Gaussian
prior and the Mann step on sampled range slices (both act voxel by voxel or
slice-locally in x, y, so a slab is exact), the CNN prior agent on sampled
voxels (oracle on each voxel's receptive field), and a short learned run
through the forward-only fallback driver."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle import cnn as ocnn
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu

TOL_OP = 1e-5


def f32(x):
    return float(np.float32(x))


@pytest.fixture(scope="module")
def large():
    import torch
    import paper_2406_13651_amd as G
    spec = synth.CONFIGS["large"]
    print("synthesising %dx%dx%d, %d looks" % (spec.nx, spec.ny, spec.nz, spec.looks), flush=True)
    r_true, y, s2w = synth.make_problem(spec, 0, workers=16)
    sigma2 = 1e-3
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, sigma2, with_prior=True)
    yt = torch.from_numpy(y).cuda()
    g.init(yt)
    torch.cuda.synchronize()
    return dict(torch=torch, G=G, spec=spec, r_true=r_true, y=y, yt=yt, s2w=s2w, sigma2=sigma2, g=g)


def test_large_agent_sampled_looks(large):
    torch, G, spec, g, y = large["torch"], large["G"], large["spec"], large["g"], large["y"]
    mu0 = [g.mu[l].cpu().numpy() for l in (0, spec.looks - 1)]
    r0 = [g.r[l].cpu().numpy() for l in (0, spec.looks - 1)]
    w0 = [g.w[l].cpu().numpy() for l in (0, spec.looks - 1)]
    beta = G.beta_schedule(1)
    g.fwd_agents(beta)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    alpha = oracle.aperture_fraction(mask)
    for i, l in enumerate((0, spec.looks - 1)):
        m1, r1, info = oracle.forward_agent(mu0[i].astype(np.complex128), y[l].astype(np.complex128),
                                            r0[i].astype(np.float64), w0[i].astype(np.float64), mask,
                                            f32(large["s2w"]), f32(large["sigma2"]), alpha, f32(beta))
        assert report("large agent mu look %d" % l, rel_l2(g.mu[l].cpu().numpy(), m1), TOL_OP) <= TOL_OP
        assert report("large agent r look %d" % l, rel_l2(g.r[l].cpu().numpy(), r1), TOL_OP) <= TOL_OP
        assert abs(g.diag[l, 0].item() - info["gamma"]) <= TOL_OP * info["gamma"]
    h0, h1 = g.h_values()
    assert bool(torch.all(h1 <= h0))


def test_large_prior_and_mann_step_on_slabs(large):
    torch, spec, g = large["torch"], large["spec"], large["g"]
    L = spec.looks
    slabs = (0, 77, spec.nz - 1)
    w_before = g.w[:, list(slabs)].cpu().numpy().astype(np.float64)
    w_prior = g.w[L].cpu().numpy().astype(np.float64)
    g.prior()
    g.mace()
    torch.cuda.synchronize()
    r_s = g.r[:, list(slabs)].cpu().numpy().astype(np.float64)
    ref_prior = oracle.gaussian_smooth(w_prior, 1.0)[list(slabs)]
    assert report("large prior slabs", rel_l2(r_s[L], ref_prior), 1e-6) <= 1e-6
    ups = oracle.agent_weights(L, True)
    wn = oracle.mann_step(w_before, r_s, ups, 0.5)
    got = g.w[:, list(slabs)].cpu().numpy()
    assert report("large mann w slabs", rel_l2(got, wn), 1e-6) <= 1e-6
    assert math.isfinite(g.conv_err())


def test_large_cnn_sampled_voxels(large):
    """Sampled outputs of the CNN at 128 x 512 x 512 against the oracle run on
    each sample's receptive field, with the same bf16-rounded weights and
    activations.  The fp32 sums of the kernels and the float64 sums of the
    oracle round a few activations to neighbouring bf16 values, which moves
    an output by ~1e-4..2e-3 whatever its size, so the error is measured
    against the RMS of the sampled residuals N(x), not per sample."""
    torch = large["torch"]
    from paper_2406_13651_amd import _clamp as C
    spec = large["spec"]
    shape = (1, spec.nz, spec.ny, spec.nx)
    rng = np.random.default_rng(11)
    params = ocnn.init_params(rng, last_scale=0.5)
    for w, b in params:
        b += 0.05 * rng.standard_normal(b.shape)
    params = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in params]
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)
    net = C.clamp_cnn_create()
    C.clamp_cnn_set_params(net, flat)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    x = torch.rand(shape, device="cuda", generator=gen) * 0.95 + 0.05
    out = torch.empty_like(x)
    ws = torch.empty(C.clamp_cnn_workspace_size(*shape, False), dtype=torch.uint8, device="cuda")
    C.clamp_cnn_apply(net, x, out, False, ws)
    torch.cuda.synchronize()
    p16 = [(ocnn.bf16_round(w), b) for w, b in params]
    # corners, edges and tile borders (16-row, 32-column tiles) and interior points
    samples = [(0, 0, 0), (127, 511, 511), (64, 200, 300), (5, 17, 255), (100, 480, 31), (64, 256, 256),
               (64, 255, 255), (1, 1, 1), (126, 510, 510), (64, 511, 0), (0, 511, 256), (64, 16, 32), (64, 15, 31),
               (64, 300, 480), (127, 0, 100)]
    diffs, resid = [], []
    for c in samples:
        lo = [max(0, c[d] - 8) for d in range(3)]
        hi = [min(shape[1 + d], c[d] + 9) for d in range(3)]
        crop = x[0, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy().astype(np.float64)
        ref, _ = ocnn.forward(crop, p16, act_round=True)
        xc = float(x[0][c].item())
        r = ref[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]] - xc
        diffs.append(float(out[0][c].item()) - xc - r)
        resid.append(r)
    err = float(np.max(np.abs(diffs)) / np.sqrt(np.mean(np.square(resid))))
    assert report("large cnn sampled voxels", err, 2e-2) <= 2e-2


def test_large_learned_run_through_fallback_driver(large):
    torch, G, spec = large["torch"], large["G"], large["spec"]
    from paper_2406_13651_amd import learned as Lm
    del large["g"]
    torch.cuda.empty_cache()
    prior = Lm.CnnPrior(Lm.init_params(0, last_scale=0.05))
    geo = (spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, large["s2w"], large["sigma2"])
    out, info = Lm.run_with_fallback(lambda: Lm.LearnedClamp(*geo, prior=prior),
                                     lambda: G.ClampGPU(*geo, with_prior=False), large["yt"], 5)
    print(info)
    assert not info["fallback"]
    assert bool(torch.isfinite(out).all())
