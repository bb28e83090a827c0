"""The learned form end to end on the GPU: a briefly trained CNN prior agent
against the plain form (Gaussian prior) on a held-out scene, and the
forward-only fallback when the learned prior produces non-finite values."""

import math
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GEO = dict(nx=64, ny=64, nz=32, looks=8, radius=16.0)


@pytest.fixture(scope="module")
def env():
    import torch
    import synth
    from paper_2406_13651_amd import learned as Lm
    spec = synth.SceneSpec("heldout", GEO["nx"], GEO["ny"], GEO["nz"], GEO["looks"], GEO["radius"], 10.0, 24,
                           0.05, 1, 6)
    r, y, s2 = synth.make_problem(spec, 0)
    return dict(torch=torch, Lm=Lm, rt=torch.from_numpy(r.astype(np.float32)).cuda(),
                yt=torch.from_numpy(y).cuda(), s2=s2)


@pytest.fixture(scope="module")
def trained(env):
    Lm = env["Lm"]
    X, T = Lm.make_pairs(480, seed=3)
    prior = Lm.CnnPrior(Lm.init_params(0))
    hist = Lm.train(prior, X, T, epochs=20, lr=5e-4)
    print("training: %d steps in %.2f s, val %.4f -> %.4f" % (hist["steps"], hist["seconds"], hist["val"][0],
                                                              hist["best_val"]))
    assert hist["best_val"] < hist["val"][0]
    return prior


def test_simulated_looks_have_the_forward_model_statistics(env):
    """Looks simulated on the GPU for the training pairs follow eqs.
    forward-model and g-given-r: with an orthonormal DFT, a pupil sample of
    slice z has E|y|^2 = mean_xy(r[z]) + sigma^2 and a sample outside the
    pupil E|y|^2 = sigma^2; the per-slice sample means agree within 5
    standard errors (|y|^2 is exponential, so its standard deviation equals
    its mean)."""
    import paper_2406_13651_amd as G
    import synth
    import oracle
    torch, Lm = env["torch"], env["Lm"]
    nx, ny, nz, L = 64, 64, 16, 12
    spec = synth.SceneSpec("sim", nx, ny, nz, L, 16.0, 10.0, 12, 0.05, 1, 6)
    r = synth.facet_scene(spec, np.random.Generator(np.random.PCG64(7)))
    s2 = synth.noise_variance(r, spec.snr_db)
    g = G.ClampGPU(nx, ny, nz, L, spec.radius, s2, 1e-3, with_prior=False)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    y = Lm.simulate_looks(g, torch.from_numpy(r.astype(np.float32)).cuda(), s2, gen)
    p2 = (y.abs() ** 2).double().cpu().numpy()          # [L, nz, ny, nx]
    mask = oracle.pupil_mask(ny, nx, spec.radius)
    n_in, n_out = int(mask.sum()) * L, int((~mask).sum()) * L
    for z in range(nz):
        want_in = float(r[z].mean()) + s2
        got_in = float(p2[:, z][:, mask].mean())
        assert abs(got_in - want_in) <= 5 * want_in / math.sqrt(n_in), (z, got_in, want_in)
        got_out = float(p2[:, z][:, ~mask].mean())
        assert abs(got_out - s2) <= 5 * s2 / math.sqrt(n_out), (z, got_out, s2)
    # the speckle average the pairs feed the network is A^H y's mean power
    g.init(y)
    sa = oracle.speckle_average(y.cpu().numpy(), mask)
    err = float(np.linalg.norm(g.r[0].cpu().numpy() - sa) / np.linalg.norm(sa))
    assert err < 1e-5, err


def _trace(g, env, iters):
    torch, Lm = env["torch"], env["Lm"]
    g.init(env["yt"])
    out = []
    for _ in range(iters):
        g.iterate()
        out.append(Lm.nrmse(g.wbar, env["rt"]))
    return out, int(g.fault.item())


def _ms_per_iter(g, env, iters=10):
    torch = env["torch"]
    g.init(env["yt"])
    g.iterate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        g.iterate()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters * 1e3


def test_learned_form_beats_plain_form(env, trained):
    """Over 20 iterations the learned form's reconstruction has a lower NRMSE
    than the plain form (Gaussian prior) and the forward agents alone, both at
    the last iteration and at each form's best iterate."""
    import paper_2406_13651_amd as G
    Lm = env["Lm"]
    geo = (GEO["nx"], GEO["ny"], GEO["nz"], GEO["looks"], GEO["radius"], env["s2"], 1e-3)
    forms = {"plain": G.ClampGPU(*geo, with_prior=True), "forward_only": G.ClampGPU(*geo, with_prior=False),
             "learned": Lm.LearnedClamp(*geo, prior=trained)}
    iters = 20
    tr = {}
    for name, g in forms.items():
        tr[name], fault = _trace(g, env, iters)
        assert fault == 0
        print("NRMSE %-12s %s  (%.3f ms per iteration)" % (name, np.round(tr[name], 4), _ms_per_iter(g, env)))
    for other in ("plain", "forward_only"):
        assert tr["learned"][-1] < tr[other][-1]
        assert min(tr["learned"]) < min(tr[other])


class NanPrior:
    """A prior agent whose output is not finite: writes NaN into r_{L+1}."""

    def __init__(self, prior):
        self.prior = prior

    def apply(self, x, out, normalize=True):
        self.prior.apply(x, out, normalize)
        out.view(-1)[::97] = float("nan")


def test_fallback_on_non_finite_prior(env, trained):
    """A prior whose output is not finite triggers the fallback, whose result
    is the forward-only reconstruction bit for bit."""
    import paper_2406_13651_amd as G
    torch, Lm = env["torch"], env["Lm"]
    geo = (GEO["nx"], GEO["ny"], GEO["nz"], GEO["looks"], GEO["radius"], env["s2"], 1e-3)
    out, info = Lm.run_with_fallback(lambda: Lm.LearnedClamp(*geo, prior=NanPrior(trained)),
                                     lambda: G.ClampGPU(*geo, with_prior=False), env["yt"], 10, env["rt"])
    assert info["fallback"] and info["reason"] == "fault"
    ref = G.ClampGPU(*geo, with_prior=False)
    ref.init(env["yt"])
    ref.run(10)
    torch.cuda.synchronize()
    assert torch.equal(out, ref.wbar)
    assert math.isfinite(info["nrmse"])


def test_nan_weights_are_rejected():
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd import learned as Lm
    p = Lm.init_params(0)
    p[5] = math.nan
    with pytest.raises(C.ClampError):
        Lm.CnnPrior(p)


def test_no_fallback_for_trained_prior(env, trained):
    import paper_2406_13651_amd as G
    Lm = env["Lm"]
    geo = (GEO["nx"], GEO["ny"], GEO["nz"], GEO["looks"], GEO["radius"], env["s2"], 1e-3)
    out, info = Lm.run_with_fallback(lambda: Lm.LearnedClamp(*geo, prior=trained),
                                     lambda: G.ClampGPU(*geo, with_prior=False), env["yt"], 20, env["rt"])
    print(info)
    assert not info["fallback"]
    assert bool(env["torch"].isfinite(out).all())
