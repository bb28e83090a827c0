"""Batched steps over uneven scenes (launches over work queues, graph replay,
autotuned grids), in both forms of the Mann step, against per-scene
single-scene steps of the same form and, scene by scene, against the float64
oracle."""

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l2, report

pytestmark = pytest.mark.gpu

SPECS = [
    # nx, ny, nz, looks, radius, with_prior
    (64, 64, 8, 3, 16.0, True),
    (192, 192, 4, 2, 48.0, False),
    (128, 128, 6, 5, 32.0, True),
    (32, 32, 16, 4, 8.0, True),
    (256, 256, 2, 2, 64.0, True),
    (384, 384, 2, 2, 96.0, True),    # 8-column tiles, radix 3
    (512, 512, 2, 2, 128.0, False),  # 8-column tiles, the longest rows
]


@pytest.fixture(scope="module")
def G():
    import torch  # noqa: F401
    import paper_2406_13651_amd as G
    return G


def _problems():
    out = []
    for i, (nx, ny, nz, L, R, wp) in enumerate(SPECS):
        spec = synth.SceneSpec("b%d" % i, nx, ny, nz, L, R, 10.0, 6, 0.05, 1, 7)
        r, y, s2 = synth.make_problem(spec, i)
        out.append((spec, y, s2, wp))
    return out


def _scene_dicts(probs, sigma2=1e-3):
    return [dict(nx=sp.nx, ny=sp.ny, nz=sp.nz, looks=sp.looks, radius=sp.radius, sigma_w2=s2, sigma2=sigma2,
                 with_prior=wp) for sp, y, s2, wp in probs]


def _batch(G, probs, fused=True):
    import torch
    b = G.ClampBatchGPU(_scene_dicts(probs), fused=fused)
    b.init([torch.from_numpy(y).cuda() for sp, y, s2, wp in probs])
    return b


@pytest.mark.parametrize("fused", [True, False])
def test_batch_steps_match_single_scene_runs(G, fused):
    """6 batched steps against the single-scene calls in the same form (the
    Mann step fused into the update pass, or a pass of its own): the same
    item code, so equal to float32 rounding."""
    import torch
    probs = _problems()
    b = _batch(G, probs, fused)
    iters = 6
    for _ in range(iters):
        b.step()
    torch.cuda.synchronize()
    assert int(b.fault.item()) == 0
    for i, (sp, y, s2, wp) in enumerate(probs):
        g = G.ClampGPU(sp.nx, sp.ny, sp.nz, sp.looks, sp.radius, s2, 1e-3, with_prior=wp, fused=fused)
        g.init(torch.from_numpy(y).cuda())
        g.run(iters)
        torch.cuda.synchronize()
        st = b.states[i]
        tag = "batch scene %d %dx%dx%d L=%d fused=%d" % (i, sp.nx, sp.ny, sp.nz, sp.looks, fused)
        assert report(tag + " w", rel_l2(b.state_w(i).cpu().numpy(), g.state_w().cpu().numpy()), 1e-6) <= 1e-6
        assert report(tag + " wbar", rel_l2(st["wbar"].cpu().numpy(), g.wbar.cpu().numpy()), 1e-6) <= 1e-6
        assert report(tag + " mu", rel_l2(st["mu"].cpu().numpy(), g.mu.cpu().numpy()), 1e-6) <= 1e-6
        assert report(tag + " r", rel_l2(st["r"].cpu().numpy(), g.r.cpu().numpy()), 1e-6) <= 1e-6
        assert abs(b.conv[i].item() - g.conv_err()) <= 1e-6 * g.conv_err()


def test_graph_replayed_batch_matches_oracle_on_every_scene(G):
    """Every scene of the batch (every supported size class from 32 to 512,
    with and without a prior) after 5 graph-replayed batched iterations,
    against the float64 oracle's run of the same scene."""
    import torch
    probs = _problems()
    b = _batch(G, probs)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    b.capture(stream)
    b.replay(5, stream)
    stream.synchronize()
    assert int(b.fault.item()) == 0
    for i, (sp, y, s2, wp) in enumerate(probs):
        st, hist = oracle.clamp_run(y, sp.radius, float(np.float32(s2)), float(np.float32(1e-3)), 5, with_prior=wp)
        tag = "batch scene %d %dx%dx%d L=%d prior=%d vs oracle, 5 graph replays" % (i, sp.nx, sp.ny, sp.nz,
                                                                                   sp.looks, wp)
        bs = b.states[i]
        assert report(tag + " wbar", rel_l2(bs["wbar"].cpu().numpy(), hist[-1]["wbar"]), 1e-4) <= 1e-4
        assert report(tag + " w", rel_l2(b.state_w(i).cpu().numpy(), st.w), 1e-4) <= 1e-4
        assert report(tag + " mu", rel_l2(bs["mu"].cpu().numpy(), st.mu), 1e-4) <= 1e-4
        ce = hist[-1]["conv_err"]
        assert abs(b.conv[i].item() - ce) <= 1e-4 * ce
        m2 = hist[-1]["mu_residual"]
        assert abs(bs["diag"][sp.looks, 0].item() - m2) <= 1e-4 * m2


def test_graph_replays_match_eager_steps(G):
    import torch
    probs = _problems()
    eager = _batch(G, probs)
    snaps = []
    for _ in range(4):
        eager.step()
        torch.cuda.synchronize()
        snaps.append([st["wbar"].cpu().numpy().copy() for st in eager.states])
    graph = _batch(G, probs)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph.capture(stream)
    filler = torch.randn(1 << 20, device="cuda")
    for k in range(4):
        graph.replay(1, stream)
        stream.synchronize()
        filler = filler * 1.0001 + 1.0  # eager work between replays
        torch.cuda.synchronize()
        for i, st in enumerate(graph.states):
            assert np.array_equal(st["wbar"].cpu().numpy(), snaps[k][i]), (k, i)
    assert int(graph.fault.item()) == 0


def test_autotuned_grids_give_identical_results(G):
    import torch
    probs = _problems()
    a = _batch(G, probs)
    b = _batch(G, probs)
    chosen = b.autotune()
    assert chosen["row_blocks_per_cu"] in (0, 2, 4, 8, 16) and chosen["col_blocks_per_cu"] in (0, 2, 4, 8, 16)
    for _ in range(3):
        a.step()
        b.step()
    torch.cuda.synchronize()
    for sa, sb in zip(a.states, b.states):
        assert np.array_equal(sa["w"].cpu().numpy(), sb["w"].cpu().numpy())
        assert np.array_equal(sa["mu"].cpu().numpy(), sb["mu"].cpu().numpy())


def test_batch_rejects_mixed_forms_of_the_mann_step(G):
    """xbar on some scenes only: CLAMP_EINVAL, nothing created."""
    import torch
    from paper_2406_13651_amd import _clamp as C
    probs = _problems()[:2]
    b = _batch(G, probs, fused=True)
    states = [dict(st) for st in b.states]
    del states[1]["xbar"]
    with pytest.raises(C.ClampError):
        C.clamp_batch_create(b.plan, states, b.fault, b.conv, torch.empty_like(b.ws))


def test_batch_rejects_the_exact_prox():
    import torch
    import paper_2406_13651_amd as G
    from paper_2406_13651_amd import _clamp as C
    sc = dict(nx=32, ny=32, nz=4, looks=2, radius=8.0, sigma_w2=0.01, sigma2=1e-3, with_prior=True,
              r_update="exact")
    with pytest.raises(C.ClampError):
        G.ClampBatchGPU([sc])
