"""clamp_mace_step_noalloc (the Mann step of Alg. 1 with the library's own
scratch instead of a workspace) against clamp_mace_step with a workspace, and
both against the float64 oracle, on two calls in a row, the second on a
smaller volume; and its rejection of volumes beyond its scratch."""

import ctypes

import numpy as np
import pytest

import oracle
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu


def _case(C, torch, nx, ny, nz, L, seed):
    rng = np.random.default_rng(seed)
    plan = C.clamp_plan_create([C.Scene(nx, ny, nz, L, nx / 4.0)])
    na = L + 1
    ups = oracle.agent_weights(L, True)
    params = C.make_params(0.01, 1e-3, 0.5, 2.0, 1.0, ups)
    w = rng.uniform(0.05, 1.0, (na, nz, ny, nx)).astype(np.float32)
    r = rng.uniform(0.05, 1.0, (na, nz, ny, nx)).astype(np.float32)
    return plan, params, ups, w, r


def _run(C, torch, plan, params, w, r, noalloc):
    wt = torch.from_numpy(w).cuda()
    rt = torch.from_numpy(r).cuda()
    wbar = torch.empty(w.shape[1:], dtype=torch.float32, device="cuda")
    conv = torch.zeros(1, dtype=torch.float64, device="cuda")
    if noalloc:
        C.clamp_mace_step_noalloc(plan, 0, params, wt, rt, wbar, conv)
    else:
        C.clamp_mace_step(plan, 0, params, wt, rt, wbar, conv, plan.workspace())
    torch.cuda.synchronize()
    return wt.cpu().numpy(), wbar.cpu().numpy(), conv.item()


def test_noalloc_mann_step_matches_the_workspace_call_twice():
    import torch
    from paper_2406_13651_amd import _clamp as C
    for shape, seed in (((128, 128, 16, 6), 1), ((32, 32, 8, 3), 2)):
        plan, params, ups, w, r = _case(C, torch, *shape, seed)
        w_a, wbar_a, ce_a = _run(C, torch, plan, params, w, r, noalloc=False)
        w_b, wbar_b, ce_b = _run(C, torch, plan, params, w, r, noalloc=True)
        # the same kernels on the same grid: identical results
        assert np.array_equal(w_a, w_b) and np.array_equal(wbar_a, wbar_b) and ce_a == ce_b
        w64, r64 = w.astype(np.float64), r.astype(np.float64)
        wn = oracle.mann_step(w64, r64, ups, 0.5)
        tag = "noalloc mann %dx%dx%d L=%d" % shape
        assert report(tag + " w", rel_l2(w_b, wn), 1e-6) <= 1e-6
        assert report(tag + " wbar", rel_l2(wbar_b, oracle.weighted_average(wn, ups)), 1e-6) <= 1e-6
        ce = oracle.convergence_error(r64, w64, ups)
        assert abs(ce_b - ce) <= 1e-5 * ce


def test_noalloc_rejects_volumes_beyond_its_scratch():
    """512 x 512 x 256 voxels need 2 MiB of partial sums: CLAMP_ESHAPE,
    decided on the host before anything is enqueued (the pointers are never
    touched)."""
    import torch
    from paper_2406_13651_amd import _clamp as C
    plan = C.clamp_plan_create([C.Scene(512, 512, 256, 1, 128.0)])
    params = C.make_params(0.01, 1e-3, 0.5, 2.0, 1.0, [1.0])
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    st = C.lib.clamp_mace_step_noalloc(plan.handle, 0, ctypes.byref(params), p, p, p, p, None)
    assert st == C.CLAMP_ESHAPE
    assert b"scratch" in C.lib.clamp_last_error()
    # the largest volume it takes: 2^25 voxels
    plan = C.clamp_plan_create([C.Scene(512, 512, 128, 1, 128.0)])
    w = torch.rand(1, 128, 512, 512, device="cuda")
    r = torch.rand(1, 128, 512, 512, device="cuda")
    wbar = torch.empty(128, 512, 512, device="cuda")
    conv = torch.zeros(1, dtype=torch.float64, device="cuda")
    w0 = w.clone()
    C.clamp_mace_step_noalloc(plan, 0, params, w, r, wbar, conv)
    torch.cuda.synchronize()
    # one agent of weight 1: G is the identity, so x = 2 r - w and w moves to
    # w + 2 rho (x - r) = r at rho = 1/2; w_bar = w; M1 = ||r - w0|| / ||w0||
    assert torch.allclose(w, r, rtol=1e-5, atol=1e-6) and torch.equal(wbar, w[0])
    assert conv.item() == pytest.approx(float(torch.linalg.norm(r - w0) / torch.linalg.norm(w0)), rel=1e-5)
