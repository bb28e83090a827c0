"""The forward agents with the Mann step of Alg. 1 fused into their update
pass (clamp_fwd_agent_mace) against the float64 oracle (forward agents,
prior, Mann step, consensus error of Sec. V-A) and against the separate
calls, including its representation of the Mann state (u_l = w_l - 2 rho
x_bar for the looks, the prior's w kept whole) and clamp_mace_state."""

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


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def compact(x, idx):
    flat = x.reshape(x.shape[:-2] + (-1,))
    return flat[..., idx]


@pytest.mark.parametrize("spec,with_prior,r_update", [
    (synth.SceneSpec("t", 32, 32, 16, 4, 8.0, 20.0, 6, 0.1), True, "quadratic"),
    (synth.SceneSpec("m", 128, 64, 6, 3, 20.0, 10.0, 8, 0.05), False, "quadratic"),
    (synth.SceneSpec("k", 192, 192, 3, 2, 48.0, 10.0, 8, 0.05), True, "quadratic"),
    (synth.SceneSpec("b", 512, 512, 2, 2, 128.0, 10.0, 8, 0.05), True, "quadratic"),
    (synth.SceneSpec("t", 32, 32, 16, 4, 8.0, 20.0, 6, 0.1), True, "exact"),
], ids=lambda v: "%dx%dx%d" % (v.nx, v.ny, v.nz) if hasattr(v, "nx") else str(v))
def test_fused_application_matches_oracle(spec, with_prior, r_update):
    """One fused call from a random state with a non-zero x_bar: mu, r, the
    Mann state, w_bar, x_bar, the consensus error and the mu-residual against
    the oracle's forward agents, prior and Mann step."""
    import torch
    import paper_2406_13651_amd as G
    r_true, y, s2w = synth.make_problem(spec, 0)
    L = spec.looks
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    alpha = oracle.aperture_fraction(mask)
    rng = np.random.default_rng(7)
    y64 = y.astype(np.complex128)
    b = np.stack([oracle.apply_AH(y64[l], mask) for l in range(L)])
    r0 = np.mean(np.abs(b) ** 2, axis=0)
    mu = (0.8 * b + 0.02 * np.sqrt(r0.mean()) * (rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)))
    mu = mu.astype(np.complex64)
    N = L + int(with_prior)
    shape = (N,) + r0.shape
    rp = (r0[None] * rng.uniform(0.5, 1.5, shape)).astype(np.float32) + np.float32(1e-6)
    w = (rp * rng.uniform(0.7, 1.3, shape)).astype(np.float32)
    xbar = (r0 * rng.uniform(0.5, 1.5, r0.shape)).astype(np.float32)
    ups = oracle.agent_weights(L, with_prior)
    sigma2, beta, rho = 0.0625, 2.0, 0.5
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, L, spec.radius, s2w, sigma2, with_prior=with_prior,
                   r_update=r_update)
    idx = G.clamp_plan_pupil_index(g.plan, 0)
    # the fused representation of w: u_l = w_l - 2 rho x_bar for the looks
    u = w.copy()
    u[:L] = (w[:L].astype(np.float64) - 2 * rho * xbar.astype(np.float64)).astype(np.float32)
    w_eff = u.astype(np.float64)
    w_eff[:L] += 2 * rho * xbar.astype(np.float64)
    wbar0 = oracle.weighted_average(w_eff, ups)
    ahy2 = np.array([np.sum(np.abs(mask * y64[l]) ** 2) for l in range(L)])
    g.mu.copy_(to_gpu(mu))
    g.resid.copy_(to_gpu(compact(y64 - oracle.apply_A(mu.astype(np.complex128), mask), idx).astype(np.complex64)))
    g.r.copy_(to_gpu(rp))
    g.w.copy_(to_gpu(u))
    g.xbar.copy_(to_gpu(xbar))
    g.wbar.copy_(to_gpu(wbar0.astype(np.float32)))
    g.ahy2.copy_(to_gpu(ahy2))
    if with_prior:
        g.prior()
    g.fwd_agents_mace(beta)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    # the oracle: forward agents at v = w_l, prior on w_{L+1}, Mann step
    r_new = np.empty(shape)
    dds = []
    for l in range(L):
        m1, r1, info = oracle.forward_agent(mu[l].astype(np.complex128), y64[l], rp[l].astype(np.float64),
                                            w_eff[l], mask, f32(s2w), sigma2, alpha, beta, r_update)
        tag = "fused %dx%dx%d %s look %d" % (spec.nx, spec.ny, spec.nz, r_update, l)
        assert report(tag + " mu", rel_l2(g.mu[l].cpu().numpy(), m1), TOL_OP) <= TOL_OP
        r_new[l] = r1
        dds.append(info["dd"])
    if with_prior:
        r_new[L] = oracle.gaussian_smooth(w_eff[L], 1.0)
    tag = "fused %dx%dx%d %s" % (spec.nx, spec.ny, spec.nz, r_update)
    assert report(tag + " r", rel_l2(g.r.cpu().numpy(), r_new), TOL_OP) <= TOL_OP
    w_new = oracle.mann_step(w_eff, r_new, ups, rho)
    assert report(tag + " w", rel_l2(g.state_w().cpu().numpy(), w_new), TOL_OP) <= TOL_OP
    assert report(tag + " wbar", rel_l2(g.wbar.cpu().numpy(), oracle.weighted_average(w_new, ups)), TOL_OP) <= TOL_OP
    xb = oracle.weighted_average(2 * r_new - w_eff, ups)
    assert report(tag + " xbar", rel_l2(g.xbar.cpu().numpy(), xb), TOL_OP) <= TOL_OP
    ce = oracle.convergence_error(r_new, w_eff, ups)
    assert abs(g.conv_err() - ce) <= TOL_OP * ce
    m2 = oracle.mu_residual(dds, ahy2, f32(s2w))
    assert abs(g.mu_residual() - m2) <= TOL_OP * m2


@pytest.mark.parametrize("with_prior", [True, False])
def test_fused_runs_match_separate_calls_and_oracle(with_prior):
    """20 iterations at 64x64x16 with 4 looks: the fused path against the
    separate calls (forward agents, prior, Mann step) and against the oracle."""
    import torch
    import paper_2406_13651_amd as G
    spec = synth.SceneSpec("r", 64, 64, 16, 4, 16.0, 10.0, 8, 0.05, 1, 1)
    r_true, y, s2w = synth.make_problem(spec, 0)
    runs = {}
    for fused in (True, False):
        g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=with_prior,
                       fused=fused)
        g.init(to_gpu(y))
        conv = []
        for _ in range(20):
            g.iterate()
            conv.append(g.conv_err())
        torch.cuda.synchronize()
        assert int(g.fault.item()) == 0
        runs[fused] = (g.wbar.cpu().numpy(), g.state_w().cpu().numpy(), g.mu.cpu().numpy(), np.array(conv))
    tag = "fused vs separate, 20 it, prior=%d" % with_prior
    for i, name in enumerate(("wbar", "w", "mu")):
        assert report(tag + " " + name, rel_l2(runs[True][i], runs[False][i]), 1e-5) <= 1e-5
    assert report(tag + " conv_err", rel_l2(runs[True][3], runs[False][3]), 1e-5) <= 1e-5
    st, hist = oracle.clamp_run(y, spec.radius, f32(s2w), f32(1e-3), 20, with_prior=with_prior)
    assert report("fused 20 it vs oracle wbar", rel_l2(runs[True][0], hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report("fused 20 it vs oracle w", rel_l2(runs[True][1], st.w), TOL_RUN) <= TOL_RUN
    ref = np.array([h["conv_err"] for h in hist])
    assert report("fused 20 it vs oracle conv_err", rel_l2(runs[True][3], ref), TOL_RUN) <= TOL_RUN


def test_mace_state_writes_out_the_representation():
    import torch
    from paper_2406_13651_amd import _clamp as C
    rng = np.random.default_rng(3)
    nx, ny, nz, L = 64, 32, 4, 3
    plan = C.clamp_plan_create([C.Scene(nx, ny, nz, L, 8.0)])
    ups = oracle.agent_weights(L, True)
    params = C.make_params(0.01, 1e-3, 0.3, 2.0, 1.0, ups)
    u = rng.standard_normal((L + 1, nz, ny, nx)).astype(np.float32)
    xb = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    out = torch.empty(L + 1, nz, ny, nx, device="cuda")
    C.clamp_mace_state(plan, 0, params, to_gpu(u), to_gpu(xb), out)
    torch.cuda.synchronize()
    want = u.astype(np.float64)
    want[:L] += 0.6 * xb.astype(np.float64)
    assert report("mace_state", rel_l2(out.cpu().numpy(), want), 1e-6) <= 1e-6
    np.testing.assert_array_equal(out[L].cpu().numpy(), u[L])
