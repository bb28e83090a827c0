"""GPU parity of the 3D operator with a zero-padded aperture (Sec. II-B eq. A
with the orthonormal 3D DFT; Sec. II-A zero-padding in range): the aperture
operator, one forward-agent application and CLAMP runs against the float64
oracle, the full range box against the per-slice operator, and the aperture
ablation a = 1."""

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


@pytest.fixture(scope="module")
def G():
    import torch  # noqa: F401
    import paper_2406_13651_amd as G
    return G


CASES = [
    # nx, ny, nz, K, radius, nbatch: zero-padding factor q = nz / K in range
    (32, 32, 16, 8, 8.0, 3),      # q = 2, batch larger than the looks
    (64, 32, 48, 32, 10.0, 2),    # q = 1.5: range length 48 (radix 3)
    (32, 64, 32, 32, 12.0, 1),    # full range box
    (32, 32, 64, 21, 9.0, 2),     # odd box
    (32, 32, 96, 64, 8.0, 2),     # q = 1.5 with the benchmark's 64-frequency box (range length 96)
    (32, 32, 128, 64, 8.0, 2),    # q = 2 with the benchmark's box (range length 128)
]


@pytest.mark.parametrize("nx,ny,nz,K,radius,nbatch", CASES)
def test_3d_operator_matches_oracle(G, nx, ny, nz, K, radius, nbatch):
    import torch
    from paper_2406_13651_amd import _clamp as C
    rng = np.random.default_rng(nx + 3 * nz + K)
    scene = C.Scene(nx, ny, nz, 2, radius, None, K)
    plan = C.clamp_plan_create([scene])
    ws = plan.workspace()
    shape = (nbatch, nz, ny, nx)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    mask = oracle.cylinder_mask(nz, ny, nx, radius, K)
    assert abs(plan.info[0]["alpha"] - oracle.aperture_fraction(mask)) <= 1e-15
    x64 = x.astype(np.complex128)
    xt = torch.from_numpy(x).cuda()
    for direction, ref in ((C.CLAMP_FWD, oracle.apply_A(x64, mask)),
                           (C.CLAMP_ADJ, oracle.apply_AH(x64, mask)),
                           (C.CLAMP_NORMAL, oracle.apply_AHA(x64, mask))):
        out = torch.empty_like(xt)
        C.clamp_aperture_op(plan, 0, direction, xt, out, nbatch, ws)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        err = report("3D aperture dir=%d %dx%dx%d K=%d" % (direction, nx, ny, nz, K), rel_l2(got, ref), TOL_OP)
        assert err <= TOL_OP
        if direction == C.CLAMP_FWD:
            assert np.all(got[:, ~mask] == 0)


def _compact_box(y, mask3, idx, K):
    """[L, nz, ny, nx] -> [L, K, P] in the library's box order (range
    frequency k for k < ceil(K/2), else nz - K + k) and pupil order idx."""
    nz = y.shape[1]
    w = [k if k < (K + 1) // 2 else nz - K + k for k in range(K)]
    flat = y[:, w].reshape(y.shape[0], K, -1)
    return flat[..., idx]


@pytest.mark.parametrize("nz,K,L", [(16, 8, 3), (96, 64, 2), (128, 64, 2)])
def test_3d_agent_application_matches_oracle(G, nz, K, L):
    import torch
    nx = ny = 32
    radius = 8.0
    spec = synth.SceneSpec("r3", nx, ny, nz, L, radius, 20.0, 6, 0.1, 1, 7)
    r_true, y, s2w = synth.make_problem(spec, 0, range_support=K)
    mask = oracle.cylinder_mask(nz, ny, nx, radius, K)
    rng = np.random.default_rng(5)
    y64 = y.astype(np.complex128)
    b = np.stack([oracle.apply_AH(y64[l], mask) for l in range(L)])
    r0 = np.mean(np.abs(b) ** 2, axis=0)
    mu = (0.8 * b + 0.02 * np.sqrt(r0.mean()) * (rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)))
    mu = mu.astype(np.complex64)
    rp = (r0[None] * rng.uniform(0.5, 1.5, b.shape)).astype(np.float32) + np.float32(1e-6)
    w = (rp * rng.uniform(0.7, 1.3, b.shape)).astype(np.float32)
    sigma2, beta = 0.0625, 2.0
    g = G.ClampGPU(nx, ny, nz, L, radius, s2w, sigma2, with_prior=False, range_support=K)
    idx = G.clamp_plan_pupil_index(g.plan, 0)
    resid = _compact_box(y64 - oracle.apply_A(mu.astype(np.complex128), mask), mask, idx, K).astype(np.complex64)
    g.mu.copy_(torch.from_numpy(mu).cuda())
    g.resid.copy_(torch.from_numpy(resid).cuda())
    g.r[:L].copy_(torch.from_numpy(rp).cuda())
    g.w[:L].copy_(torch.from_numpy(w).cuda())
    g.fwd_agents(beta)
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    alpha = oracle.aperture_fraction(mask)
    diag = g.diag.cpu().numpy()
    for l in range(L):
        m1, r1, info = oracle.forward_agent(mu[l].astype(np.complex128), y64[l], rp[l].astype(np.float64),
                                            w[l].astype(np.float64), mask, f32(s2w), sigma2, alpha, beta)
        assert report("3D agent mu nz=%d look %d" % (nz, l), rel_l2(g.mu[l].cpu().numpy(), m1), TOL_OP) <= TOL_OP
        assert report("3D agent r nz=%d look %d" % (nz, l), rel_l2(g.r[l].cpu().numpy(), r1), TOL_OP) <= TOL_OP
        res1 = _compact_box((y64[l] - oracle.apply_A(m1, mask))[None], mask, idx, K)[0]
        assert report("3D agent resid nz=%d look %d" % (nz, l), rel_l2(g.resid[l].cpu().numpy(), res1), TOL_OP) <= TOL_OP
        for k, key in ((G.DG_GAMMA, "gamma"), (G.DG_DD, "dd"), (G.DG_AD, "ad"), (G.DG_WD, "wd")):
            assert abs(diag[l, k] - info[key]) <= TOL_OP * abs(info[key]), (key, diag[l, k], info[key])
        const = np.sum(np.abs((~mask) * y64[l]) ** 2) / (2 * f32(s2w))
        for k, key in ((G.DG_H0, "h0"), (G.DG_H1, "h1")):
            want = info[key] - const
            assert abs(diag[l, k] - want) <= TOL_OP * abs(want), (key, diag[l, k], want)
    h0, h1 = g.h_values()
    assert bool(torch.all(h1 <= h0))


@pytest.mark.parametrize("nz,K,with_prior", [(16, 8, False), (48, 32, True), (96, 64, True), (128, 64, True)])
def test_3d_clamp_run_matches_oracle(G, nz, K, with_prior):
    import torch
    nx = ny = 32
    L, radius, sigma2 = 3, 8.0, 2e-4
    spec = synth.SceneSpec("r3", nx, ny, nz, L, radius, 20.0, 6, 0.1, 1, 7)
    r_true, y, s2w = synth.make_problem(spec, 1, range_support=K)
    g = G.ClampGPU(nx, ny, nz, L, radius, s2w, sigma2, with_prior=with_prior, range_support=K)
    g.init(torch.from_numpy(y).cuda())
    iters = 20
    for _ in range(iters):
        g.iterate()
    torch.cuda.synchronize()
    assert int(g.fault.item()) == 0
    mask = oracle.cylinder_mask(nz, ny, nx, radius, K)
    st, hist = oracle.clamp_run(y, radius, f32(s2w), f32(sigma2), iters, with_prior=with_prior, mask=mask)
    tag = "3D %dx%dx%d K=%d prior=%d 20 it" % (nx, ny, nz, K, with_prior)
    assert report(tag + " wbar", rel_l2(g.wbar.cpu().numpy(), hist[-1]["wbar"]), TOL_RUN) <= TOL_RUN
    assert report(tag + " mu", rel_l2(g.mu.cpu().numpy(), st.mu), TOL_RUN) <= TOL_RUN
    assert abs(g.conv_err() - hist[-1]["conv_err"]) <= TOL_RUN * hist[-1]["conv_err"] + 1e-12


def test_full_range_box_equals_per_slice_run(G):
    """3D looks that are the range DFT of per-slice looks, with a full range
    box, give the per-slice run's reconstruction."""
    import torch
    nx = ny = 32
    nz, L, radius = 16, 3, 8.0
    spec = synth.SceneSpec("t", nx, ny, nz, L, radius, 20.0, 6, 0.1, 1, 0)
    r_true, y2, s2w = synth.make_problem(spec, 0)
    y3 = np.fft.fft(y2.astype(np.complex128), axis=1, norm="ortho").astype(np.complex64)
    g2 = G.ClampGPU(nx, ny, nz, L, radius, s2w, 2e-4, with_prior=True)
    g3 = G.ClampGPU(nx, ny, nz, L, radius, s2w, 2e-4, with_prior=True, range_support=nz)
    g2.init(torch.from_numpy(y2).cuda())
    g3.init(torch.from_numpy(y3).cuda())
    for _ in range(10):
        g2.iterate()
        g3.iterate()
    torch.cuda.synchronize()
    assert report("full box vs per-slice wbar", rel_l2(g3.wbar.cpu().numpy(), g2.wbar.cpu().numpy()), TOL_RUN) <= TOL_RUN


def test_aperture_ablation_all_pass_3d(G):
    """a = 1 in 3D (all-pass pupil, full range box) and a constant anchor: the
    mu-step lands on the closed form A^H y (r' + s)/(r' + 2 s)."""
    import torch
    nx = ny = 32
    nz, L = 16, 2
    rng = np.random.default_rng(9)
    y = (rng.standard_normal((L, nz, ny, nx)) + 1j * rng.standard_normal((L, nz, ny, nx))).astype(np.complex64)
    s2w = 0.25
    g = G.ClampGPU(nx, ny, nz, L, 0.0, s2w, 0.1, with_prior=False, mask=np.ones((ny, nx), np.uint8),
                   range_support=nz)
    g.init(torch.from_numpy(y).cuda())
    g.r.fill_(0.75)
    g.w.fill_(0.75)
    g.fwd_agents(2.0)
    torch.cuda.synchronize()
    want = oracle.idft3(y.astype(np.complex128)) * (0.75 + s2w) / (0.75 + 2 * s2w)
    assert report("3D all-pass closed form", rel_l2(g.mu.cpu().numpy(), want), TOL_OP) <= TOL_OP


def test_3d_errors(G):
    from paper_2406_13651_amd import _clamp as C
    with pytest.raises(C.ClampError):
        C.clamp_plan_create([C.Scene(32, 32, 40, 1, 8.0, None, 20)])   # range length 40 unsupported
    with pytest.raises(C.ClampError):
        C.clamp_plan_create([C.Scene(32, 32, 16, 1, 8.0, None, 17)])   # box larger than nz
    with pytest.raises(C.ClampError):
        G.ClampBatchGPU([dict(nx=32, ny=32, nz=16, looks=2, radius=8.0, sigma_w2=0.01, sigma2=1e-3,
                              with_prior=True, range_support=8)])
