"""Pins of the CNN oracle: a library correlation, finite differences, the
identity at zero output weights, and bfloat16 rounding."""

import numpy as np
from scipy.ndimage import correlate

from oracle import cnn


def test_conv3d_matches_library_correlation(rng):
    x = rng.standard_normal((3, 5, 6, 7))
    w = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    y = cnn.conv3d(x, w, b)
    for co in range(2):
        want = np.full(x.shape[1:], b[co])
        for ci in range(3):
            k = np.zeros((3, 3, 3))
            for t, (dz, dy, dx) in enumerate(cnn.OFFSETS):
                k[dz + 1, dy + 1, dx + 1] = w[t, ci, co]
            want += correlate(x[ci], k, mode="constant", cval=0.0)
        np.testing.assert_allclose(y[co], want, atol=1e-12)


def _small_params(rng, width=3, layers=4):
    return cnn.init_params(rng, width, layers, last_scale=0.5)


def test_gradients_match_finite_differences(rng):
    params = _small_params(rng)
    for w, b in params:
        b += 0.05 * rng.standard_normal(b.shape)
    xs = rng.uniform(0.1, 1.0, (2, 3, 4, 5))
    ts = rng.uniform(0.1, 1.0, (2, 3, 4, 5))
    loss, grads = cnn.loss_and_grads(xs, ts, params)
    eps = 1e-6
    for i in range(len(params)):
        for j in range(2):
            p = params[i][j]
            flat = p.ravel()
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp, _ = cnn.loss_and_grads(xs, ts, params)
                flat[idx] = old - eps
                lm, _ = cnn.loss_and_grads(xs, ts, params)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = grads[i][j].ravel()[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, j, idx, fd, an)


def test_zero_last_layer_is_identity(rng):
    params = cnn.init_params(rng, 4, 8, last_scale=0.0)
    x = rng.uniform(0.1, 1.0, (4, 6, 8))
    out, _ = cnn.forward(x, params)
    np.testing.assert_array_equal(out, x)
    np.testing.assert_allclose(cnn.denoise(3.0 * x, params), 3.0 * x)


def test_denoise_is_scale_equivariant(rng):
    params = _small_params(rng, 3, 3)
    x = rng.uniform(0.1, 1.0, (3, 4, 5))
    np.testing.assert_allclose(cnn.denoise(7.0 * x, params), 7.0 * cnn.denoise(x, params), rtol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.1415926, 0.0])
    r = cnn.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie rounds to even (mantissa ...0)
    assert r[2] == 1.0 + 2 ** -7             # above the tie rounds up
    assert r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.1415926) <= 2 ** -8 * 4
    # idempotent
    np.testing.assert_array_equal(cnn.bf16_round(r), r)


def test_adam_first_step_moves_by_lr(rng):
    params = [(np.ones((2, 2)), np.zeros(2))]
    grads = [(np.array([[1.0, -2.0], [0.5, 0.0]]), np.array([3.0, -1.0]))]
    state = {}
    new = cnn.adam_step(params, grads, state, 0.1)
    # first bias-corrected step: p - lr * sign(g) (for g != 0)
    np.testing.assert_allclose(new[0][0], [[0.9, 1.1], [0.9, 1.0]], atol=1e-6)
    np.testing.assert_allclose(new[0][1], [-0.1, 0.1], atol=1e-6)
