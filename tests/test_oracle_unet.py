"""Pins of the U-Net oracle (oracle/unet.py) against definitions written as
brute-force loops, adjoint identities, closed forms of batch normalisation,
and central finite differences of the whole network's loss."""

import numpy as np
import pytest

from oracle import unet as U


def test_maxpool_brute_force_and_gradient():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 6, 8))
    y = U.maxpool2(x)
    for c in range(3):
        for z in range(2):
            for yy in range(3):
                for xx in range(4):
                    win = x[c, 2 * z:2 * z + 2, 2 * yy:2 * yy + 2, 2 * xx:2 * xx + 2]
                    assert y[c, z, yy, xx] == win.max()
    g = rng.standard_normal(y.shape)
    gx = U.maxpool2_grad(x, g)
    assert np.isclose(gx.sum(), g.sum()) and np.count_nonzero(gx) == g.size
    # the gradient sits where the maximum is: central differences (no ties in random data)
    i = (1, 2, 3, 5)
    h = 1e-6
    xp, xm = x.copy(), x.copy()
    xp[i] += h
    xm[i] -= h
    fd = (np.sum(g * U.maxpool2(xp)) - np.sum(g * U.maxpool2(xm))) / (2 * h)
    assert np.isclose(fd, gx[i], atol=1e-8)


def test_maxpool_ties_go_to_the_first_position():
    x = np.zeros((1, 2, 2, 2))
    g = np.ones((1, 1, 1, 1))
    gx = U.maxpool2_grad(x, g)
    assert gx[0, 0, 0, 0] == 1.0 and gx.sum() == 1.0


def test_upconv_brute_force_adjoint_and_weight_gradient():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 2, 3, 2))
    w = rng.standard_normal((8, 4, 5))
    b = rng.standard_normal(5)
    y = U.upconv(x, w, b)
    ref = np.zeros_like(y)
    for co in range(5):
        for z in range(2):
            for yy in range(3):
                for xx in range(2):
                    for a in range(2):
                        for bb in range(2):
                            for c in range(2):
                                ref[co, 2 * z + a, 2 * yy + bb, 2 * xx + c] = b[co] + sum(
                                    x[ci, z, yy, xx] * w[4 * a + 2 * bb + c, ci, co] for ci in range(4))
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)
    g = rng.standard_normal(y.shape)
    # adjoint: <upconv(x, w, 0), g> = <x, upconv_input_grad(g, w)>
    lhs = np.sum(U.upconv(x, w, np.zeros(5)) * g)
    assert np.isclose(lhs, np.sum(x * U.upconv_input_grad(g, w)), rtol=1e-12)
    # linear in w: <upconv(x, w, 0), g> = <w, dw>, and db = sum of g
    dw, db = U.upconv_weight_grad(x, g)
    assert np.isclose(lhs, np.sum(w * dw), rtol=1e-12)
    np.testing.assert_allclose(db, g.sum(axis=(1, 2, 3)))


def test_batchnorm_closed_form_and_gradient():
    rng = np.random.default_rng(2)
    z = rng.standard_normal((2, 3, 2, 3, 4)) * 2.0 + 1.0
    gamma, beta = rng.uniform(0.5, 2, 3), rng.standard_normal(3)
    y, xhat, rstd, mean, var = U.bn_train(z, gamma, beta)
    # per channel: mean beta, standard deviation gamma sqrt(var / (var + eps))
    np.testing.assert_allclose(y.mean(axis=(0, 2, 3, 4)), beta, atol=1e-12)
    np.testing.assert_allclose(y.std(axis=(0, 2, 3, 4)), gamma * np.sqrt(var / (var + U.BN_EPS)), rtol=1e-12)
    dy = rng.standard_normal(y.shape)
    dz, dg, db = U.bn_train_grad(dy, xhat, gamma, rstd)
    f = lambda zz, gg, bb: np.sum(dy * U.bn_train(zz, gg, bb)[0])
    h = 1e-6
    for i in [(0, 1, 1, 2, 3), (1, 0, 0, 0, 0), (1, 2, 1, 1, 1)]:
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        assert np.isclose((f(zp, gamma, beta) - f(zm, gamma, beta)) / (2 * h), dz[i], rtol=1e-6, atol=1e-8)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        assert np.isclose((f(z, gamma + e, beta) - f(z, gamma - e, beta)) / (2 * h), dg[c], rtol=1e-6)
        assert np.isclose((f(z, gamma, beta + e) - f(z, gamma, beta - e)) / (2 * h), db[c], rtol=1e-6)


def _tiny(seed=3):
    rng = np.random.default_rng(seed)
    p = U.init_params(rng, width=4, last_scale=1.0)
    for i in range(U.CONVS):
        p["gamma"][i] = rng.uniform(0.5, 1.5, 4)
        p["beta"][i] = 0.1 * rng.standard_normal(4)
    for j in range(U.LEVELS):
        p["up_b"][j] = 0.1 * rng.standard_normal(4)
    p["final_b"] = np.array([0.05])
    xs = rng.uniform(0.05, 1.0, (2, 8, 8, 8))
    ts = rng.uniform(0.05, 1.0, (2, 8, 8, 8))
    return p, xs, ts


def test_parameter_layout_round_trip():
    p, _, _ = _tiny()
    v = U.flatten(p)
    q = U.unflatten(v, width=4)
    np.testing.assert_array_equal(U.flatten(q), v)
    assert U.param_count() == U.flatten(U.init_params(np.random.default_rng(0))).size == 331297


def test_folded_evaluation_equals_batchnorm_evaluation():
    """Folding evaluation-mode BN into the convolutions changes nothing."""
    p, xs, _ = _tiny()
    rng = np.random.default_rng(4)
    stats = {"mean": [0.1 * rng.standard_normal(4) for _ in range(U.CONVS)],
             "var": [rng.uniform(0.5, 2.0, 4) for _ in range(U.CONVS)]}
    out, _ = U.forward(xs, p, False, stats)
    np.testing.assert_allclose(U.forward_folded(xs, U.fold_params(p, stats)), out, rtol=1e-12, atol=1e-12)


def test_running_statistics_update():
    p, xs, _ = _tiny()
    stats = U.init_stats(width=4)
    _, c = U.forward(xs, p, True, stats)
    z0 = c["layers"][0]
    # the first layer's batch mean, recomputed from its pre-activations
    zpre = np.stack([U.conv3d(x, p["conv"][0], np.zeros(4)) for x in xs[:, None]])
    m = zpre.mean(axis=(0, 2, 3, 4))
    n = zpre.shape[0] * np.prod(zpre.shape[2:])
    np.testing.assert_allclose(stats["mean"][0], 0.1 * m, rtol=1e-12)
    np.testing.assert_allclose(stats["var"][0], 0.9 + 0.1 * zpre.var(axis=(0, 2, 3, 4)) * n / (n - 1), rtol=1e-12)
    assert z0["out"].min() >= 0.0


@pytest.mark.parametrize("group,index", [("conv", (0, (4, 0, 1))), ("conv", (3, (13, 2, 3))), ("conv", (7, (0, 1, 2))),
                                         ("conv", (11, (26, 3, 0))), ("gamma", (2, 1)), ("beta", (9, 3)),
                                         ("up_w", (0, (5, 1, 2))), ("up_w", (2, (0, 3, 3))), ("up_b", (1, 2)),
                                         ("final_w", (None, (20, 1, 0))), ("final_b", (None, 0))])
def test_loss_gradient_against_finite_differences(group, index):
    p, xs, ts = _tiny()
    _, gr = U.loss_and_grads(xs, ts, p)
    i, j = index
    def get(q):
        return q[group] if i is None else q[group][i]
    h = 1e-5
    pp = {k: ([a.copy() for a in v] if isinstance(v, list) else v.copy()) for k, v in p.items()}
    pm = {k: ([a.copy() for a in v] if isinstance(v, list) else v.copy()) for k, v in p.items()}
    get(pp)[j] += h
    get(pm)[j] -= h
    loss = lambda q: float(np.mean((U.forward(xs, q, True)[0] - ts) ** 2))
    fd = (loss(pp) - loss(pm)) / (2 * h)
    an = get(gr)[j]
    assert np.isclose(fd, an, rtol=2e-4, atol=1e-9), (fd, an)
