"""The full-size plain form (256x256x64, 16 looks, pupil radius 64, SNR 10 dB,
forward agents + Gaussian prior + Mann step) against the float64 oracle after
50 iterations of Alg. 2, in the launch configuration the benchmark times (the
Mann step fused into the forward agents' update pass); the
float32 drift of the residual recurrence over 100 iterations; and the
residual refresh (resid = D(a) y - D(a) F mu) against the oracle."""

import os

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu

TOL_OP = 1e-5
TOL_RUN = 1e-4


def f32(x):
    return float(np.float32(x))


def _say(capsys, msg):
    """Progress straight to the terminal (long oracle runs)."""
    with capsys.disabled():
        print("[fullsize] " + msg, flush=True)


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.mark.timeout(900)
def test_full_size_50_iterations_match_oracle(capsys):
    import torch
    import paper_2406_13651_amd as G
    spec = synth.CONFIGS["full"]
    r_true, y, s2w = synth.make_problem(spec, 0, workers=_workers())
    sigma2, iters = 1e-3, 50
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, sigma2, with_prior=True)
    g.init(torch.from_numpy(y).cuda())
    conv, mres = [], []
    for _ in range(iters):
        g.iterate()
        conv.append(g.conv_err())
        mres.append(g.mu_residual())
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    gpu = {"wbar": g.wbar.cpu().numpy(), "w": g.state_w().cpu().numpy(), "r": g.r.cpu().numpy(),
           "mu": g.mu.cpu().numpy()}
    del g
    torch.cuda.empty_cache()
    _say(capsys, "GPU run done; oracle: %d iterations on %d threads" % (iters, _workers()))
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    state = oracle.clamp_init(y, mask, True, 1.0)
    prior = lambda x: oracle.gaussian_smooth(x, 1.0)  # noqa: E731
    hist = []
    for it in range(iters):
        h = oracle.clamp_iteration(state, y, mask, f32(s2w), f32(sigma2), 0.5, prior, workers=_workers())
        hist.append({"conv_err": h["conv_err"], "mu_residual": h["mu_residual"],
                     "wbar": h["wbar"] if it == iters - 1 else None})
        if (it + 1) % 10 == 0:
            _say(capsys, "oracle iteration %d" % (it + 1))
    tag = "256x256x64 L=16 50 it"
    assert report(tag + " wbar", rel_l2(gpu["wbar"], hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report(tag + " w", rel_l2(gpu["w"], state.w), TOL_RUN) <= TOL_RUN
    assert report(tag + " r", rel_l2(gpu["r"], state.r), TOL_RUN) <= TOL_RUN
    assert report(tag + " mu", rel_l2(gpu["mu"], state.mu), TOL_RUN) <= TOL_RUN
    ref_conv = np.array([h["conv_err"] for h in hist])
    assert report(tag + " conv_err trajectory", rel_l2(np.array(conv), ref_conv), TOL_RUN) <= TOL_RUN
    ref_m2 = np.array([h["mu_residual"] for h in hist])
    assert report(tag + " mu-residual trajectory", rel_l2(np.array(mres), ref_m2), TOL_RUN) <= TOL_RUN


def _host_resid(mu, y, mask, idx):
    """D(a)(y - A mu) in the compact layout, float64."""
    a = oracle.apply_A(mu.astype(np.complex128), mask)
    d = (y.astype(np.complex128) - a).reshape(a.shape[:-2] + (-1,))
    return d[..., idx]


@pytest.mark.timeout(600)
def test_full_size_residual_drift_and_refresh(capsys):
    """100 iterations at full size without a refresh: the residual kept by
    the recurrence resid -= gamma D(a) F d drifts from D(a)(y - A mu) only by
    float32 rounding; clamp_fwd_refresh rebuilds it to float32 accuracy.
    Both figures are printed (first and last look, against float64 on the
    host)."""
    import torch
    import paper_2406_13651_amd as G
    spec = synth.CONFIGS["full"]
    r_true, y, s2w = synth.make_problem(spec, 0, workers=_workers())
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=True)
    g.init(torch.from_numpy(y).cuda())
    g.run(100)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    idx = G.clamp_plan_pupil_index(g.plan, 0)
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    looks = (0, spec.looks - 1)
    kept = g.resid[list(looks)].cpu().numpy()
    mu = g.mu[list(looks)].cpu().numpy()
    want = np.stack([_host_resid(mu[i], y[l], mask, idx) for i, l in enumerate(looks)])
    ynorm = np.linalg.norm(np.stack([y[l].reshape(spec.nz, -1)[:, idx] for l in looks]))
    drift = np.linalg.norm(kept - want) / ynorm
    report("resid drift after 100 it (rel. to ||D(a) y||)", drift, TOL_RUN)
    _say(capsys, "residual drift after 100 iterations: %.3e of ||D(a) y||; vs ||resid||: %.3e"
         % (drift, np.linalg.norm(kept - want) / np.linalg.norm(want)))
    g.refresh()
    torch.cuda.synchronize()
    fresh = g.resid[list(looks)].cpu().numpy()
    err = np.linalg.norm(fresh - want) / ynorm
    assert report("resid after refresh (rel. to ||D(a) y||)", err, TOL_OP) <= TOL_OP
    assert drift <= TOL_RUN


def test_refreshed_runs_match_oracle():
    """20 forward-only iterations at 32x32x16 with a refresh after every
    5th: the oracle forms the residual from y at every step, so refreshing
    keeps the GPU run on the oracle's trajectory."""
    import torch
    import paper_2406_13651_amd as G
    spec = synth.CONFIGS["tiny"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 2e-4, with_prior=False,
                   refresh_every=5)
    g.init(torch.from_numpy(y).cuda())
    g.run(20)
    torch.cuda.synchronize()
    st, hist = oracle.clamp_run(y, spec.radius, f32(s2w), f32(2e-4), 20, with_prior=False)
    assert report("tiny 20 it, refresh every 5: wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]),
                  TOL_RUN) <= TOL_RUN
    assert report("tiny 20 it, refresh every 5: mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN


def test_refresh_with_the_3d_operator():
    """The 3D operator's residual lives on the range box: the refresh gives
    box(D(a)(y - A mu)) for the 3D aperture."""
    import torch
    import paper_2406_13651_amd as G
    nx = ny = 32
    nz, K, L = 32, 16, 2
    spec = synth.SceneSpec("r3", nx, ny, nz, L, 8.0, 20.0, 6, 0.1, 1, 7)
    r_true, y, s2w = synth.make_problem(spec, 1, range_support=K)
    g = G.ClampGPU(nx, ny, nz, L, 8.0, s2w, 2e-4, with_prior=False, range_support=K)
    g.init(torch.from_numpy(y).cuda())
    g.run(3)
    rng = np.random.default_rng(1)
    mu = (rng.standard_normal(g.mu.shape) + 1j * rng.standard_normal(g.mu.shape)).astype(np.complex64)
    g.mu.copy_(torch.from_numpy(mu).cuda())
    g.refresh()
    torch.cuda.synchronize()
    mask = oracle.cylinder_mask(nz, ny, nx, 8.0, K)
    idx = G.clamp_plan_pupil_index(g.plan, 0)
    box = [k if k < (K + 1) // 2 else nz - K + k for k in range(K)]  # the library's box order
    d = y.astype(np.complex128) - oracle.apply_A(mu.astype(np.complex128), mask)
    want = d.reshape(L, nz, -1)[:, box][:, :, idx]
    assert report("3D refresh", rel_l2(g.resid.cpu().numpy(), want), TOL_OP) <= TOL_OP
