"""The package's host metrics (k-d tree point clouds, PSNR, NRMSE) against the
oracle's brute-force definitions (Sec. V-A eqs. psnr, pc-distance, nrmse)."""

import numpy as np

import oracle
import synth


def _metrics():
    import importlib.util
    import os
    # the package imports the GPU library at import time; the metrics module
    # itself needs only numpy and scipy, so load it from its file
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2406_13651_amd",
                        "metrics.py")
    spec = importlib.util.spec_from_file_location("clamp_host_metrics", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_point_cloud_metrics_match_brute_force(rng):
    M = _metrics()
    spec = synth.SceneSpec("m", 32, 32, 16, 1, 8.0, 10.0, 6, 0.05)
    r = synth.facet_scene(spec, np.random.default_rng(3))
    # a reconstruction: the truth shifted by a voxel in range in places, blurred, with spurious points
    rec = 0.8 * np.roll(r, 1, axis=0) + 0.02 * rng.uniform(size=r.shape)
    rec[rng.uniform(size=r.shape) > 0.995] = 0.9
    for cut in (1.5, 3.0, 7.32):
        got = M.point_cloud_metrics(rec, r, 0.1, 0.05, cut)
        want = oracle.point_cloud_metrics(rec, r, 0.1, 0.05, cut)
        for k in ("points", "kept"):
            assert got[k] == want[k]
        for k in ("distance", "false_positive_rate", "nrmse", "beta"):
            assert abs(got[k] - want[k]) <= 1e-12 * max(1.0, abs(want[k])), (k, got[k], want[k])


def test_lattice_ties_take_the_first_point(rng):
    """Many equidistant lattice neighbours: the k-d tree search must pick the
    same (first) truth point as brute force."""
    M = _metrics()
    truth = np.zeros((9, 9, 9))
    truth[::2, ::2, ::2] = rng.uniform(0.5, 1.0, truth[::2, ::2, ::2].shape)
    rec = np.zeros_like(truth)
    rec[1::2, 1::2, 1::2] = 1.0          # every point has 8 nearest truth points at sqrt(3)
    got = M.point_cloud_metrics(rec, truth, 0.1, 0.1, 5.0)
    want = oracle.point_cloud_metrics(rec, truth, 0.1, 0.1, 5.0)
    assert got["nrmse"] == want["nrmse"] and got["beta"] == want["beta"]


def test_volumetric_measures_match_oracle(rng):
    M = _metrics()
    r = rng.uniform(0.05, 1.0, (4, 8, 8))
    rh = 2.3 * r + 0.05 * rng.standard_normal(r.shape)
    assert abs(M.psnr(rh, r) - oracle.psnr(rh, r)) < 1e-12
    assert abs(M.nrmse(rh, r) - oracle.nrmse(rh, r)) < 1e-14
    assert abs(M.rayleigh_cutoff(256, 64) - 3 * 1.22 * 2) < 1e-12
