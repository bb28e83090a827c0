"""The seeded input generator: determinism, recipe bounds and the uneven-batch
draw (no GPU)."""

import numpy as np
import pytest

import synth


def test_problem_is_seeded_and_shaped():
    spec = synth.CONFIGS["tiny"]
    r1, y1, s1 = synth.make_problem(spec, 0)
    r2, y2, s2 = synth.make_problem(spec, 0)
    assert np.array_equal(y1, y2) and np.array_equal(r1, r2) and s1 == s2
    assert y1.shape == (spec.looks, spec.nz, spec.ny, spec.nx) and y1.dtype == np.complex64
    assert r1.min() >= spec.r_min and np.isclose(r1.max(), 1.0)
    # one occupied range bin per pixel
    assert np.all(np.sum(r1 > spec.r_min, axis=0) <= 1)
    assert np.isclose(s1, r1.mean() * 10 ** (-spec.snr_db / 10))
    _, y3, _ = synth.make_problem(spec, 1)
    assert not np.array_equal(y1, y3)


def test_measurement_pupil_and_noise_level():
    spec = synth.SceneSpec("t", 32, 32, 8, 6, 8.0, 10.0, 4, 0.05)
    r, y, s2 = synth.make_problem(spec, 0)
    pupil = synth.synth_pupil(32, 32, 8.0)
    off = y[:, :, ~pupil]
    # outside the pupil only noise remains: per-sample power sigma_eta^2
    assert abs(np.mean(np.abs(off) ** 2) / s2 - 1) < 0.05


@pytest.mark.parametrize("workers", [1, 4])
def test_threaded_synthesis_is_deterministic(workers):
    spec = synth.SceneSpec("t", 32, 32, 4, 5, 8.0, 10.0, 4, 0.05)
    r1, y1, s1 = synth.make_problem(spec, 3)
    r2, y2, s2 = synth.make_problem(spec, 3, workers=workers)
    assert np.array_equal(y1, y2) and s1 == s2


def test_batch_spec_draw_respects_cap():
    specs = synth.batch_specs(32, seed=0, cap_voxel_looks=2.5e9)
    assert len(specs) == 32
    assert sum(s.n * s.looks for s in specs) <= 2.5e9
    assert {s.nx for s in specs} <= {128, 192, 256, 384, 512}
    assert all(s.radius == s.nx / 4 for s in specs)
