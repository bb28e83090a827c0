"""Pins of the comparison regularizers (Sec. V: the l_{2,1} and isotropic TV
agents), the speckle average, and the point-cloud metrics (Sec. V-A eqs.
pc-distance and nrmse) against closed forms, exact solvers on tiny inputs
and hand-computed cases."""

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize

import oracle
import synth


def test_l21_prox_is_block_soft_thresholding_and_minimal(rng):
    v = rng.standard_normal((4, 3, 5))
    norms = np.sqrt(np.sum(v ** 2, axis=(1, 2)))
    tau = float(np.sort(norms)[1])          # one slice below, others above the threshold
    r = oracle.l21_prox(v, tau)
    for z in range(4):
        if norms[z] <= tau:
            assert np.all(r[z] == 0)
        else:
            np.testing.assert_allclose(r[z], v[z] * (1 - tau / norms[z]), rtol=1e-14)

    def obj(x):
        return tau * oracle.l21_norm(x) + 0.5 * np.sum((x - v) ** 2)
    best = obj(r)
    for _ in range(2000):
        assert obj(r + 1e-3 * rng.standard_normal(v.shape)) >= best - 1e-12
    np.testing.assert_array_equal(oracle.l21_prox(v, 0.0), v)
    assert np.all(oracle.l21_prox(v, norms.max() * 1.01) == 0)


def test_l21_prox_against_numerical_minimisation(rng):
    """Two slices of two voxels: the objective minimised numerically from
    several starts lands on the closed form."""
    v = np.array([[[0.3, -0.4]], [[1.0, 2.0]]])
    tau = 0.8                                  # slice 0 (norm 0.5) is zeroed
    r = oracle.l21_prox(v, tau)

    def obj(x):
        x = x.reshape(v.shape)
        return tau * oracle.l21_norm(x) + 0.5 * np.sum((x - v) ** 2)
    best = min((minimize(obj, rng.standard_normal(4), method="Powell", options={"xtol": 1e-12, "ftol": 1e-14})
                for _ in range(5)), key=lambda o: o.fun)
    np.testing.assert_allclose(best.x.reshape(v.shape), r, atol=1e-6)


def test_grad_div_adjoint_and_differences(rng):
    u = rng.standard_normal((3, 4, 5))
    p = rng.standard_normal((3, 3, 4, 5))
    g = oracle.grad3(u)
    assert abs(np.sum(g * p) + np.sum(u * oracle.div3(p))) < 1e-12
    # the differences by loops
    for z in range(3):
        for y in range(4):
            for x in range(5):
                assert g[0, z, y, x] == (u[z + 1, y, x] - u[z, y, x] if z < 2 else 0.0)
                assert g[1, z, y, x] == (u[z, y + 1, x] - u[z, y, x] if y < 3 else 0.0)
                assert g[2, z, y, x] == (u[z, y, x + 1] - u[z, y, x] if x < 4 else 0.0)
    # a single-voxel axis has no difference
    assert np.all(oracle.grad3(rng.standard_normal((1, 3, 3)))[0] == 0)


def test_tv_prox_of_a_constant_and_dual_feasibility(rng):
    v = np.full((3, 4, 5), 0.7)
    r, p = oracle.tv_prox(v, 0.5, 50)
    np.testing.assert_allclose(r, v, atol=1e-14)
    v = rng.standard_normal((4, 5, 6))
    r, p = oracle.tv_prox(v, 0.3, 200)
    assert np.max(np.sqrt(np.sum(p ** 2, axis=0))) <= 1 + 1e-12
    assert oracle.tv_dual_gap(v, 0.3, r, p) >= -1e-9


def test_tv_prox_1d_against_bounded_least_squares(rng):
    """A 1 x 1 x n volume: TV is the 1D total variation, whose prox has the
    dual min_p ||v - lam D^T p||^2 over |p_i| <= 1 (D the forward-difference
    matrix), solved exactly by bounded least squares."""
    n, lam = 12, 0.35
    v = rng.standard_normal(n)
    D = np.zeros((n - 1, n))
    for i in range(n - 1):
        D[i, i], D[i, i + 1] = -1.0, 1.0
    sol = lsq_linear(lam * D.T, v, bounds=(-1.0, 1.0), tol=1e-14, method="bvls")
    want = v - lam * D.T @ sol.x
    r, _ = oracle.tv_prox(v.reshape(1, 1, n), lam, 20000)
    np.testing.assert_allclose(r.ravel(), want, atol=1e-6)


def test_tv_prox_3d_isotropic_against_constrained_dual(rng):
    """A 2 x 2 x 2 volume: the isotropic dual min_p ||v - lam div p||^2 / 2
    with |p_voxel|_2 <= 1, solved by SLSQP; the oracle's iteration reaches
    the same primal image."""
    shape, lam = (2, 2, 2), 0.4
    v = rng.standard_normal(shape)

    def obj(x):
        return 0.5 * np.sum((v - lam * oracle.div3(x.reshape((3,) + shape))) ** 2)

    cons = [{"type": "ineq", "fun": (lambda x, i=i: 1.0 - np.sum(x.reshape(3, -1)[:, i] ** 2))} for i in range(8)]
    sol = minimize(obj, np.zeros(24), method="SLSQP", constraints=cons, options={"ftol": 1e-15, "maxiter": 500})
    want = v - lam * oracle.div3(sol.x.reshape((3,) + shape))
    r, p = oracle.tv_prox(v, lam, 20000)
    np.testing.assert_allclose(r, want, atol=1e-6)
    assert oracle.tv_dual_gap(v, lam, r, p) < 1e-9


def test_speckle_average_is_the_initial_image():
    spec = synth.SceneSpec("t", 16, 16, 4, 3, 4.0, 20.0, 4, 0.1)
    r, y, s2 = synth.make_problem(spec, 0)
    mask = oracle.pupil_mask(16, 16, spec.radius)
    sa = oracle.speckle_average(y, mask)
    st = oracle.clamp_init(y, mask, True, 1.0)
    np.testing.assert_allclose(st.r[0], np.maximum(sa, 1e-12 * sa.mean()), rtol=1e-15)


def test_point_cloud_metrics_hand_computed():
    """Truth: (0,0,0) r=1 and (0,0,4) r=0.5.  Reconstruction: (0,0,1) r=2 and
    (0,0,3) r=1 at distance 1, and (0,0,20) at distance 16 beyond the cutoff
    5 (a false positive).  Kept pairs (2, 1) and (1, 0.5): beta* = 1/2 and
    NRMSE 0; mean distance 1; false-positive rate 1/3."""
    truth = np.zeros((1, 1, 24))
    truth[0, 0, 0], truth[0, 0, 4] = 1.0, 0.5
    rec = np.zeros((1, 1, 24))
    rec[0, 0, 1], rec[0, 0, 3], rec[0, 0, 20] = 2.0, 1.0, 1.0
    m = oracle.point_cloud_metrics(rec, truth, 0.1, 0.1, 5.0)
    assert m["points"] == 3 and m["kept"] == 2
    assert m["distance"] == 1.0 and abs(m["false_positive_rate"] - 1 / 3) < 1e-15
    assert m["beta"] == 0.5 and m["nrmse"] == 0.0
    # a point equidistant from both takes the first in (z, y, x) order
    rec = np.zeros((1, 1, 24))
    rec[0, 0, 2] = 3.0
    m = oracle.point_cloud_metrics(rec, truth, 0.1, 0.1, 5.0)
    assert m["distance"] == 2.0 and m["beta"] == pytest.approx(1 / 3)
