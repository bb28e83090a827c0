"""GPU parity of the comparison set of Sec. V against the float64 oracle: the
l_{2,1} and TV prior agents (alone and as the prior of CLAMP runs), and the
speckle average."""

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu


def f32(x):
    return float(np.float32(x))


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan(C, nx, ny, nz):
    plan = C.clamp_plan_create([C.Scene(nx, ny, nz, 1, nx / 4.0)])
    return plan, plan.workspace()


@pytest.mark.parametrize("nx,ny,nz", [(64, 32, 8), (256, 256, 4), (32, 32, 1)])
def test_l21_prox_matches_oracle(nx, ny, nz):
    import torch
    from paper_2406_13651_amd import _clamp as C
    rng = np.random.default_rng(nx + nz)
    x = rng.uniform(0.0, 1.0, (nz, ny, nx)) * rng.uniform(0.05, 1.0, (nz, 1, 1))
    x = x.astype(np.float32)
    norms = np.sqrt(np.sum(x.astype(np.float64) ** 2, axis=(1, 2)))
    tau = float(np.median(norms))          # about half the slices are zeroed
    plan, ws = _plan(C, nx, ny, nz)
    out = torch.empty(nz, ny, nx, device="cuda")
    C.clamp_prior_l21(plan, 0, tau, to_gpu(x), out, ws)
    torch.cuda.synchronize()
    want = oracle.l21_prox(x.astype(np.float64), f32(tau))
    assert report("l21 prox %dx%dx%d" % (nx, ny, nz), rel_l2(out.cpu().numpy(), want), 1e-6) <= 1e-6
    zero = norms <= f32(tau)
    assert np.all(out.cpu().numpy()[zero] == 0)


@pytest.mark.parametrize("nx,ny,nz,iters", [(64, 32, 10, 30), (256, 256, 8, 20), (32, 32, 1, 40), (32, 64, 3, 0)])
def test_tv_prox_matches_oracle(nx, ny, nz, iters):
    import torch
    from paper_2406_13651_amd import _clamp as C
    rng = np.random.default_rng(nx + 7 * nz)
    x = (rng.uniform(0.0, 1.0, (nz, ny, nx)) + (rng.uniform(size=(nz, ny, nx)) > 0.9)).astype(np.float32)
    lam = 0.2
    plan, ws = _plan(C, nx, ny, nz)
    out = torch.empty(nz, ny, nx, device="cuda")
    C.clamp_prior_tv(plan, 0, lam, iters, to_gpu(x), out, ws)
    torch.cuda.synchronize()
    want, _ = oracle.tv_prox(x.astype(np.float64), f32(lam), iters)
    err = rel_l2(out.cpu().numpy(), want)
    assert report("tv prox %dx%dx%d, %d steps" % (nx, ny, nz, iters), err, 1e-5) <= 1e-5


@pytest.mark.parametrize("prior,weight", [("l21", 3.0), ("tv", 0.05)])
def test_clamp_runs_with_comparison_priors_match_oracle(prior, weight):
    """10 iterations at 64x64x16 with 4 looks, the forward agents and the
    Mann step fused, with the l_{2,1} or the TV agent as prior."""
    import torch
    import paper_2406_13651_amd as G
    spec = synth.SceneSpec("r", 64, 64, 16, 4, 16.0, 10.0, 8, 0.05, 1, 1)
    r_true, y, s2w = synth.make_problem(spec, 0)
    iters, tv_iters = 10, 15
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3, with_prior=True, prior=prior,
                   prior_weight=weight, tv_iters=tv_iters)
    g.init(to_gpu(y))
    for _ in range(iters):
        g.iterate()
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    mask = oracle.pupil_mask(spec.ny, spec.nx, spec.radius)
    if prior == "l21":
        H = lambda v: oracle.l21_prox(v, f32(weight))  # noqa: E731
    else:
        H = lambda v: oracle.tv_prox(v, f32(weight), tv_iters)[0]  # noqa: E731
    st = oracle.clamp_init(y, mask, True, 1.0)
    hist = [oracle.clamp_iteration(st, y, mask, f32(s2w), f32(1e-3), 0.5, H) for _ in range(iters)]
    tag = "%s prior, 10 it" % prior
    assert report(tag + " wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]), 1e-4) <= 1e-4
    assert report(tag + " w", rel_l2(g.state_w().cpu().numpy(), st.w), 1e-4) <= 1e-4
    assert report(tag + " r prior", rel_l2(g.r[spec.looks].cpu().numpy(), st.r[spec.looks]), 1e-4) <= 1e-4


def test_speckle_average_matches_oracle():
    import torch
    import paper_2406_13651_amd as G
    spec = synth.CONFIGS["tiny"]
    r_true, y, s2w = synth.make_problem(spec, 0)
    g = G.ClampGPU(spec.nx, spec.ny, spec.nz, spec.looks, spec.radius, s2w, 1e-3)
    g.init(to_gpu(y))
    torch.cuda.synchronize()
    want = oracle.speckle_average(y, oracle.pupil_mask(spec.ny, spec.nx, spec.radius))
    assert report("speckle average", rel_l2(g.speckle_average().cpu().numpy(), want), 1e-5) <= 1e-5


def test_regularizer_argument_errors():
    import torch
    from paper_2406_13651_amd import _clamp as C
    plan, ws = _plan(C, 32, 32, 4)
    x = torch.ones(4, 32, 32, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(C.ClampError):
        C.clamp_prior_l21(plan, 0, -1.0, x, out, ws)
    with pytest.raises(C.ClampError):
        C.clamp_prior_tv(plan, 0, 0.0, 10, x, out, ws)
    with pytest.raises(C.ClampError):
        C.clamp_prior_tv(plan, 0, 0.1, -1, x, out, ws)
    with pytest.raises(C.ClampError):
        C.clamp_prior_tv(plan, 0, 0.1, 5, x, x, ws)
