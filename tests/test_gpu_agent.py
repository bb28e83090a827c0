"""GPU parity of the forward agent, initialisation, prior and Mann step
(Sec. III-A/B, Alg. 2, App. A) against the float64 oracle, through the C ABI."""

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu

TOL_OP = 1e-5     # one application of an operator or agent
TOL_RUN = 1e-4    # after a run of iterations


@pytest.fixture(scope="module")
def G():
    import torch  # noqa: F401
    import paper_2406_13651_amd as G
    return G


def f32(x):
    """The float32 value the GPU receives, as float64 for the oracle."""
    return float(np.float32(x))


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def compact(x, idx):
    """[..., ny, nx] -> [..., P] in the library's compact pupil order."""
    flat = x.reshape(x.shape[:-2] + (-1,))
    return flat[..., idx]


def _state(spec, seed=3):
    r_true, y, s2w = synth.make_problem(spec, 0)
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    rng = np.random.default_rng(seed)
    y64 = y.astype(np.complex128)
    b = np.stack([oracle.apply_AH(y64[l], mask) for l in range(spec.looks)])
    r0 = np.mean(np.abs(b) ** 2, axis=0)
    shape = b.shape
    mu = (0.8 * b + 0.02 * np.sqrt(r0.mean()) * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)))
    mu = mu.astype(np.complex64)
    rp = (r0[None] * rng.uniform(0.5, 1.5, shape)).astype(np.float32) + np.float32(1e-6)
    w = (rp * rng.uniform(0.7, 1.3, shape)).astype(np.float32)
    return r_true, y, s2w, mask, mu, rp, w


@pytest.mark.parametrize("spec", [
    synth.SceneSpec("t", 32, 32, 16, 4, 8.0, 20.0, 6, 0.1),
    synth.SceneSpec("m", 128, 64, 6, 3, 20.0, 10.0, 8, 0.05),
    synth.SceneSpec("k", 192, 192, 3, 2, 48.0, 10.0, 8, 0.05),
], ids=lambda s: "%dx%dx%d" % (s.nx, s.ny, s.nz))
@pytest.mark.parametrize("r_update", ["quadratic", "exact"])
def test_one_agent_application_matches_oracle(G, spec, r_update):
    import torch
    r_true, y, s2w, mask, mu, rp, w = _state(spec)
    sigma2, beta = 0.0625, 2.0
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, sigma2, with_prior=False,
                   r_update=r_update)
    idx = G.clamp_plan_pupil_index(g.plan, 0)
    y64 = y.astype(np.complex128)
    mu64 = mu.astype(np.complex128)
    resid = compact(y64 - oracle.apply_A(mu64, mask), idx).astype(np.complex64)
    ahy2 = np.array([np.sum(np.abs(mask * y64[l]) ** 2) for l in range(spec.looks)])
    g.mu.copy_(to_gpu(mu))
    g.resid.copy_(to_gpu(resid))
    g.r[: spec.looks].copy_(to_gpu(rp))
    g.w[: spec.looks].copy_(to_gpu(w))
    g.ahy2.copy_(to_gpu(ahy2))
    g.fwd_agents(beta)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    mu_g, r_g = g.mu.cpu().numpy(), g.r[: spec.looks].cpu().numpy()
    resid_g, diag = g.resid.cpu().numpy(), g.diag.cpu().numpy()
    alpha = oracle.aperture_fraction(mask)
    s2w32 = f32(s2w)
    dds = []
    for l in range(spec.looks):
        m1, r1, info = oracle.forward_agent(mu64[l], y64[l], rp[l].astype(np.float64), w[l].astype(np.float64),
                                            mask, s2w32, sigma2, alpha, beta, r_update)
        tag = "%dx%dx%d look %d %s" % (spec.nx, spec.ny, spec.nz, l, r_update)
        assert report("agent mu " + tag, rel_l2(mu_g[l], m1), TOL_OP) <= TOL_OP
        assert report("agent r " + tag, rel_l2(r_g[l], r1), TOL_OP) <= TOL_OP
        res1 = compact(y64[l] - oracle.apply_A(m1, mask), idx)
        assert report("agent resid " + tag, rel_l2(resid_g[l], res1), TOL_OP) <= TOL_OP
        for k, key in ((G.DG_GAMMA, "gamma"), (G.DG_DD, "dd"), (G.DG_AD, "ad"), (G.DG_WD, "wd")):
            assert abs(diag[l, k] - info[key]) <= TOL_OP * abs(info[key]), (key, diag[l, k], info[key])
        # the library's h leaves out the constant of the data off the pupil
        const = np.sum(np.abs((~mask) * y64[l]) ** 2) / (2 * s2w32)
        for k, key in ((G.DG_H0, "h0"), (G.DG_H1, "h1")):
            want = info[key] - const
            assert abs(diag[l, k] - want) <= TOL_OP * abs(want), (key, diag[l, k], want)
        want = oracle.mu_residual([info["dd"]], [ahy2[l]], s2w32)
        assert abs(diag[l, G.DG_MURES] - want) <= TOL_OP * want
        np.testing.assert_allclose(diag[l, G.DG_R2], np.sum(np.abs(res1) ** 2), rtol=TOL_OP)
        dds.append(info["dd"])
    want = oracle.mu_residual(dds, ahy2, s2w32)
    assert abs(g.mu_residual() - want) <= TOL_OP * want
    np.testing.assert_allclose(diag[spec.looks, 1:3], diag[: spec.looks, [G.DG_H0, G.DG_H1]].sum(axis=0),
                               rtol=1e-12)
    h0, h1 = g.h_values()
    h0, h1 = h0.numpy(), h1.numpy()
    assert np.all(h1 <= h0)
    assert np.allclose(h0 - h1, 0.5 * diag[: spec.looks, 0] * diag[: spec.looks, 1], rtol=0,
                       atol=1e-5 * np.max(h0))


def test_init_matches_oracle(G):
    import torch
    spec = synth.CONFIGS["tiny"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    for with_prior, s_mu in ((True, 1.0), (False, 1.0 / oracle.aperture_fraction(mask))):
        g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=with_prior,
                       mu_scale=s_mu)
        g.init(to_gpu(y))
        torch.cuda.synchronize()
        st = oracle.clamp_init(y, mask, with_prior, f32(s_mu))
        assert report("init mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_OP) <= TOL_OP
        assert report("init r", rel_l2(g.r.cpu().numpy(), st.r), TOL_OP) <= TOL_OP
        assert report("init w", rel_l2(g.w.cpu().numpy(), st.w), TOL_OP) <= TOL_OP
        assert rel_l2(g.ahy2.cpu().numpy(), st.ahy2) <= TOL_OP
        idx = G.clamp_plan_pupil_index(g.plan, 0)
        res = compact(y.astype(np.complex128) - oracle.apply_A(st.mu, mask), idx)
        got = g.resid.cpu().numpy()
        assert np.linalg.norm(got - res) <= TOL_OP * np.linalg.norm(compact(y.astype(np.complex128), idx))
        # D(a) y kept for the residual refresh
        assert np.array_equal(g.y_pupil.cpu().numpy(), compact(y, idx))


def test_prior_and_mann_step_match_oracle(G):
    import torch
    rng = np.random.default_rng(2)
    nx, ny, nz, L = 64, 32, 8, 3
    g = G.ClampGPU(nx, ny, nz, L, 8.0, 0.01, 1e-3, with_prior=True)
    x = rng.uniform(0.05, 1.0, (nz, ny, nx)).astype(np.float32)
    g.w[L].copy_(to_gpu(x))
    g.prior()
    torch.cuda.synchronize()
    ref = oracle.gaussian_smooth(x.astype(np.float64), 1.0)
    assert report("gaussian prior", rel_l2(g.r[L].cpu().numpy(), ref), 1e-6) <= 1e-6
    w = rng.uniform(0.05, 1.0, (L + 1, nz, ny, nx)).astype(np.float32)
    r = rng.uniform(0.05, 1.0, (L + 1, nz, ny, nx)).astype(np.float32)
    g.w.copy_(to_gpu(w))
    g.r.copy_(to_gpu(r))
    g.mace()
    torch.cuda.synchronize()
    ups = oracle.agent_weights(L, True)
    w64, r64 = w.astype(np.float64), r.astype(np.float64)
    wn = oracle.mann_step(w64, r64, ups, 0.5)
    assert report("mann w", rel_l2(g.w.cpu().numpy(), wn), 1e-6) <= 1e-6
    assert report("mann wbar", rel_l2(g.wbar.cpu().numpy(), oracle.weighted_average(wn, ups)), 1e-6) <= 1e-6
    ce = oracle.convergence_error(r64, w64, ups)
    assert abs(g.conv_err() - ce) <= 1e-5 * ce


@pytest.mark.parametrize("L,with_prior", [(3, False), (6, True), (16, True), (40, False)])
def test_mann_step_agent_counts(G, L, with_prior):
    """Agent counts that are and are not multiples of the kernel's register
    block (padding agents must neither contribute nor be written)."""
    import torch
    rng = np.random.default_rng(10 + L)
    nx, ny, nz = 64, 32, 4
    g = G.ClampGPU(nx, ny, nz, L, 8.0, 0.01, 1e-3, with_prior=with_prior)
    na = L + int(with_prior)
    w = rng.uniform(0.05, 1.0, (na, nz, ny, nx)).astype(np.float32)
    r = rng.uniform(0.05, 1.0, (na, nz, ny, nx)).astype(np.float32)
    g.w.copy_(to_gpu(w))
    g.r.copy_(to_gpu(r))
    g.mace()
    torch.cuda.synchronize()
    ups = oracle.agent_weights(L, with_prior)
    w64, r64 = w.astype(np.float64), r.astype(np.float64)
    wn = oracle.mann_step(w64, r64, ups, 0.5)
    assert report("mann w, %d agents" % na, rel_l2(g.w.cpu().numpy(), wn), 1e-6) <= 1e-6
    assert rel_l2(g.wbar.cpu().numpy(), oracle.weighted_average(wn, ups)) <= 1e-6
    np.testing.assert_array_equal(g.r.cpu().numpy(), r)
    ce = oracle.convergence_error(r64, w64, ups)
    assert abs(g.conv_err() - ce) <= 1e-5 * ce


def _run_pair(G, spec, sigma2, iters, with_prior, r_update="quadratic"):
    import torch
    r_true, y, s2w = synth.make_problem(spec, 0)
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, sigma2, with_prior=with_prior,
                   r_update=r_update)
    g.init(to_gpu(y))
    errs = []
    for _ in range(iters):
        g.iterate()
        errs.append(g.conv_err())
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    st, hist = oracle.clamp_run(y, spec.radius, f32(s2w), f32(sigma2), iters, with_prior=with_prior,
                                r_update=r_update)
    return g, st, hist, errs


def test_tiny_forward_only_20_iterations(G):
    spec = synth.CONFIGS["tiny"]
    g, st, hist, errs = _run_pair(G, spec, 2e-4, 20, False)
    assert report("tiny 20 it wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report("tiny 20 it r", rel_l2(g.r.cpu().numpy(), st.r), TOL_RUN) <= TOL_RUN
    assert report("tiny 20 it mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN
    ref = np.array([h["conv_err"] for h in hist])
    assert report("tiny 20 it conv_err", rel_l2(np.array(errs), ref), TOL_RUN) <= TOL_RUN


def test_tiny_forward_only_20_iterations_exact_prox(G):
    """The exact surrogate prox in place of the quadratic surrogate: 20
    forward-only iterations against the oracle run with the same r-update."""
    spec = synth.CONFIGS["tiny"]
    g, st, hist, errs = _run_pair(G, spec, 2e-4, 20, False, r_update="exact")
    assert report("tiny 20 it exact wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report("tiny 20 it exact r", rel_l2(g.r.cpu().numpy(), st.r), TOL_RUN) <= TOL_RUN
    assert report("tiny 20 it exact mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN


def test_exact_prox_run_with_prior(G):
    spec = synth.SceneSpec("r", 64, 64, 16, 4, 16.0, 10.0, 8, 0.05, 1, 1)
    g, st, hist, errs = _run_pair(G, spec, 1e-3, 20, True, r_update="exact")
    assert report("64x64x16 20 it exact w", rel_l2(g.state_w().cpu().numpy(), st.w), TOL_RUN) <= TOL_RUN
    assert report("64x64x16 20 it exact mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN


def test_reduced_full_recipe_50_iterations_with_prior(G):
    spec = synth.SceneSpec("r", 64, 64, 16, 4, 16.0, 10.0, 8, 0.05, 1, 1)
    g, st, hist, errs = _run_pair(G, spec, 1e-3, 50, True)
    assert report("64x64x16 50 it wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report("64x64x16 50 it w", rel_l2(g.state_w().cpu().numpy(), st.w), TOL_RUN) <= TOL_RUN
    assert report("64x64x16 50 it mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN
    mu_res = g.mu_residual()
    assert abs(mu_res - hist[-1]["mu_residual"]) <= 1e-3 * hist[-1]["mu_residual"]


def test_all_pass_pupil_one_step_closed_form(G):
    """a = 1 and a constant anchor: the mu-step lands on A^H y (r'+s)/(r'+2s)."""
    import torch
    nx = ny = 32
    nz, L = 4, 2
    rng = np.random.default_rng(4)
    y = (rng.standard_normal((L, nz, ny, nx)) + 1j * rng.standard_normal((L, nz, ny, nx))).astype(np.complex64)
    s2w = 0.25
    g = G.ClampGPU(nx, ny, nz, L, 0.0, s2w, 0.1, with_prior=False, mask=np.ones((ny, nx), np.uint8))
    g.init(to_gpu(y))
    g.r.fill_(0.75)
    g.w.fill_(0.75)
    g.fwd_agents(2.0)
    torch.cuda.synchronize()
    want = oracle.apply_AH(y.astype(np.complex128), np.ones((ny, nx), bool)) * (0.75 + s2w) / (0.75 + 2 * s2w)
    assert report("all-pass closed form", rel_l2(g.mu.cpu().numpy(), want), TOL_OP) <= TOL_OP


def test_runs_are_bitwise_deterministic(G):
    import torch
    spec = synth.SceneSpec("d", 64, 64, 8, 3, 16.0, 10.0, 6, 0.05)
    r_true, y, s2w = synth.make_problem(spec, 0)
    outs = []
    for _ in range(2):
        g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=True)
        g.init(to_gpu(y))
        g.run(5)
        torch.cuda.synchronize()
        outs.append((g.wbar.cpu().numpy().copy(), g.diag.cpu().numpy().copy(), g.conv_err()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_full_size_agent_sampled_looks(G):
    """256x256x64, 16 looks, in the launch configuration the benchmark uses:
    one forward-agent application from the initial state, checked against the
    oracle on the first and the last look (each look is independent), and the
    mu-step decrement identity on every look."""
    import torch
    spec = synth.CONFIGS["full"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    sigma2 = 1e-3
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, sigma2, with_prior=True)
    yt = to_gpu(y)
    g.init(yt)
    torch.cuda.synchronize()
    mu0 = g.mu.cpu().numpy()
    r0 = g.r.cpu().numpy()
    w0 = g.w.cpu().numpy()
    beta = G.beta_schedule(1)
    g.fwd_agents(beta)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    alpha = oracle.aperture_fraction(mask)
    for l in (0, spec.looks - 1):
        m1, r1, info = oracle.forward_agent(mu0[l].astype(np.complex128), y[l].astype(np.complex128),
                                            r0[l].astype(np.float64), w0[l].astype(np.float64), mask, f32(s2w),
                                            f32(sigma2), alpha, f32(beta))
        assert report("full agent mu look %d" % l, rel_l2(g.mu[l].cpu().numpy(), m1), TOL_OP) <= TOL_OP
        assert report("full agent r look %d" % l, rel_l2(g.r[l].cpu().numpy(), r1), TOL_OP) <= TOL_OP
        assert abs(g.diag[l, 0].item() - info["gamma"]) <= TOL_OP * info["gamma"]
    h0, h1 = g.h_values()
    assert bool(torch.all(h1 <= h0))
    # the rest of the iteration at full size: prior and Mann step on the GPU state
    w_before = g.w.cpu().numpy().astype(np.float64)
    g.prior()
    g.mace()
    torch.cuda.synchronize()
    r_all = g.r.cpu().numpy().astype(np.float64)
    ref_prior = oracle.gaussian_smooth(w_before[spec.looks], 1.0)
    assert report("full prior", rel_l2(r_all[spec.looks], ref_prior), 1e-6) <= 1e-6
    ups = oracle.agent_weights(spec.looks, True)
    wn = oracle.mann_step(w_before, r_all, ups, 0.5)
    assert report("full mann w", rel_l2(g.w.cpu().numpy(), wn), 1e-6) <= 1e-6


def test_full_size_run_properties(G):
    """50 iterations at 256x256x64, 16 looks: every mu-step decreases h, no
    fault is raised and the consensus error falls."""
    import torch
    spec = synth.CONFIGS["full"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=True)
    g.init(to_gpu(y))
    errs = []
    for _ in range(50):
        g.iterate()
        h0, h1 = g.h_values()
        assert bool(torch.all(h1 <= h0 * (1 + 1e-7)))
        errs.append(g.conv_err())
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    assert np.all(np.isfinite(errs)) and errs[-1] < errs[0]


def test_timing_of_selected_stages(G):
    """clamp_plan_set_timing_stages records events around the chosen stages
    only; clamp_plan_set_timing(1) around every stage of the call."""
    import torch
    from paper_2406_13651_amd import _clamp as C
    spec = synth.CONFIGS["tiny"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    for fused, update in ((False, "row_update"), (True, "row_update_mann")):
        g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=True, fused=fused)
        g.init(to_gpu(y))
        C.clamp_plan_set_timing_stages(g.plan, [update])
        g.iterate()
        torch.cuda.synchronize()
        C.clamp_plan_set_timing(g.plan, False)
        st = C.clamp_plan_get_timing(g.plan)
        assert set(st) == {update} and st[update][1] == 1 and st[update][0] > 0.0
        C.clamp_plan_set_timing(g.plan, True)
        g.iterate()
        C.clamp_plan_set_timing(g.plan, False)
        st = C.clamp_plan_get_timing(g.plan)
        assert {"col_inv", "row_grad", "col_fwd", update, "mace_step", "prior_gauss"} <= set(st)
    with pytest.raises(ValueError):
        C.clamp_plan_set_timing_stages(g.plan, ["no such stage"])
