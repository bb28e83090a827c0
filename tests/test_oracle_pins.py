"""Pins of the oracle's convergence measures, initialisation, quality metrics
and clipped optimiser against hand-computed values and dense brute force
(Sec. V-A eqs. mace-convergence-error, residual and psnr; Alg. 2
initialisation).  Each pin is chosen so that a plausible slip (a wrong
normalisation, a sum in place of a mean, a dropped scale fit) fails it."""

import numpy as np

import oracle
from oracle import cnn


def _dense_dft(n):
    return np.array([[np.exp(-2j * np.pi * k * j / n) for j in range(n)] for k in range(n)]) / np.sqrt(n)


def _dense_A(ny, nx, mask):
    """A = D(a) F as a dense matrix acting on one slice flattened x-fastest."""
    F = np.kron(_dense_dft(ny), _dense_dft(nx))
    return np.diag(mask.ravel().astype(float)) @ F


def test_convergence_error_hand_computed():
    """Three agents, one voxel: w = (1, 2, 3), weights (1/4, 1/4, 1/2) give
    w_bar = 9/4; with F(w) = (2, 2, 3) the stacked difference F(w) - G(w) is
    (-1/4, -1/4, 3/4), of squared norm 11/16, and G(w) stacks w_bar three
    times, of squared norm 243/16: M1 = sqrt(11/243).  Dividing by ||w_bar||
    alone would give sqrt(11/81)."""
    w = np.array([[1.0], [2.0], [3.0]])
    r = np.array([[2.0], [2.0], [3.0]])
    ups = np.array([0.25, 0.25, 0.5])
    assert abs(oracle.convergence_error(r, w, ups) - np.sqrt(11.0 / 243.0)) < 1e-15


def test_convergence_error_against_explicit_stack(rng):
    """G(w) written out as N copies of the weighted average, built by a loop
    over agents, and the norms taken over the flattened stacks."""
    N, shape = 3, (2, 3, 4)
    w = rng.standard_normal((N,) + shape)
    r = rng.standard_normal((N,) + shape)
    ups = np.array([0.2, 0.3, 0.5])
    wbar = np.zeros(shape)
    for j in range(N):
        wbar += ups[j] * w[j]
    G = np.stack([wbar] * N)
    want = np.linalg.norm((r - G).ravel()) / np.linalg.norm(G.ravel())
    assert abs(oracle.convergence_error(r, w, ups) - want) < 1e-14 * want


def test_mu_residual_against_dense_normal_equations(rng):
    """eq. residual with the noise-floored inverse covariance: per look
    ||((1/s) A^H A + D(omega)) mu - A^H y / s|| / ||A^H y / s||, averaged over
    looks, with A a dense matrix; the oracle gets ||d||^2 of the forward agent
    at the same mu (before its step) and ||A^H y||^2."""
    nz, ny, nx, L = 1, 6, 8, 3
    mask = oracle.pupil_mask(ny, nx, 2)
    alpha = oracle.aperture_fraction(mask)
    s2w = 0.37
    A = _dense_A(ny, nx, mask[0] if mask.ndim == 3 else mask)
    terms, dds, ahy2 = [], [], []
    for _ in range(L):
        y = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
        mu = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
        rp = rng.uniform(0.2, 2.0, (nz, ny, nx))
        w = rng.uniform(0.2, 2.0, (nz, ny, nx))
        omega = 1.0 / (rp.ravel() + s2w / alpha)
        M = A.conj().T @ A / s2w + np.diag(omega)
        b = A.conj().T @ y.ravel() / s2w
        terms.append(np.linalg.norm(M @ mu.ravel() - b) / np.linalg.norm(b))
        _, _, info = oracle.forward_agent(mu, y, rp, w, mask, s2w, 0.1, alpha, 2.0)
        dds.append(info["dd"])
        ahy2.append(float(np.sum(np.abs(A.conj().T @ y.ravel()) ** 2)))
    want = np.mean(terms)
    assert abs(oracle.mu_residual(dds, ahy2, s2w) - want) < 1e-12 * want


def test_initial_reflectance_is_the_look_average(rng):
    """r0 = (1/L) sum_l |A^H y_l|^2 voxel by voxel, with A^H as a dense
    matrix and the sum over looks written as a loop; every agent's anchor and
    state start there (a sum instead of the mean would be L times larger)."""
    nz, ny, nx, L = 2, 6, 8, 3
    mask = oracle.pupil_mask(ny, nx, 2.5)
    A = _dense_A(ny, nx, mask)
    y = rng.standard_normal((L, nz, ny, nx)) + 1j * rng.standard_normal((L, nz, ny, nx))
    want = np.zeros((nz, ny, nx))
    for l in range(L):
        for z in range(nz):
            b = A.conj().T @ y[l, z].ravel()
            want[z] += np.abs(b.reshape(ny, nx)) ** 2
    want /= L
    st = oracle.clamp_init(y, mask, looks_with_prior=True, mu_scale=1.0)
    assert st.r.shape[0] == L + 1
    for j in range(L + 1):
        np.testing.assert_allclose(st.r[j], want, rtol=1e-12)
        np.testing.assert_allclose(st.w[j], want, rtol=1e-12)
    for l in range(L):
        b = np.stack([(A.conj().T @ y[l, z].ravel()).reshape(ny, nx) for z in range(nz)])
        assert abs(st.ahy2[l] - np.sum(np.abs(b) ** 2)) < 1e-12 * st.ahy2[l]


def test_psnr_and_nrmse_hand_computed():
    """r = (1, 0), r_hat = (1, 1): beta* = 1/2, beta* r_hat - r = (-1/2, 1/2),
    squared error 1/2, so PSNR = 10 log10(2 / (1/2)) = 10 log10 4 and
    NRMSE = sqrt(1/2).  Without the scale fit PSNR would be 10 log10 2."""
    r = np.array([1.0, 0.0])
    rh = np.array([1.0, 1.0])
    assert oracle.scale_fit(rh, r) == 0.5
    assert abs(oracle.psnr(rh, r) - 10.0 * np.log10(4.0)) < 1e-12
    assert abs(oracle.nrmse(rh, r) - np.sqrt(0.5)) < 1e-15


def _params_like(rng):
    return [(rng.standard_normal((3, 2, 4)), rng.standard_normal(4)), (rng.standard_normal((3, 4, 1)),
                                                                       rng.standard_normal(1))]


def _grads_with_norm(rng, params, norm):
    g = [(rng.standard_normal(w.shape), rng.standard_normal(b.shape)) for w, b in params]
    cur = np.sqrt(sum(np.sum(a * a) + np.sum(b * b) for a, b in g))
    return [(a * norm / cur, b * norm / cur) for a, b in g]


def test_clipped_adam_equals_plain_adam_while_norms_stay_below_the_cap(rng):
    """Gradient norms within a factor 1.5 of each other never reach three
    times the running average, so the clipped rule is plain Adam (itself
    pinned by its first step, which moves every parameter by lr sign(g))."""
    params = _params_like(rng)
    pa, pb = params, params
    sa, sb = {}, {}
    for k in range(6):
        g = _grads_with_norm(rng, params, 1.0 + 0.5 * (k % 2))
        pa = cnn.adam_step(pa, g, sa, 0.01)
        pb = cnn.adam_step_clipped(pb, g, sb, 0.01)
    for (wa, ba), (wb, bb) in zip(pa, pb):
        np.testing.assert_array_equal(wa, wb)
        np.testing.assert_array_equal(ba, bb)


def test_clipped_adam_caps_the_gradient_at_three_running_norms(rng):
    """After steps of gradient norm 2 the running average is 2; a gradient of
    norm 600 enters the first moment as a vector of norm 3 * 2 = 6, so the
    moment moves by 0.1 * 6, and the average moves to 0.95 * 2 + 0.05 * 6."""
    params = _params_like(rng)
    st = {}
    for _ in range(4):
        params = cnn.adam_step_clipped(params, _grads_with_norm(rng, params, 2.0), st, 1e-3)
    assert abs(st["run_norm"] - 2.0) < 1e-12
    m_before = {k: v.copy() for k, v in st.items() if isinstance(k, tuple) and k[0] == "m"}
    params = cnn.adam_step_clipped(params, _grads_with_norm(rng, params, 600.0), st, 1e-3)
    moved = np.sqrt(sum(np.sum((st[k] - 0.9 * m_before[k]) ** 2) for k in m_before))
    assert abs(moved - 0.1 * 6.0) < 1e-12
    assert abs(st["run_norm"] - (0.95 * 2.0 + 0.05 * 6.0)) < 1e-12


def test_clipped_adam_skips_a_non_finite_gradient(rng):
    """A NaN gradient leaves parameters, moments and the average as they were;
    the bias correction's step count still advances, so the next finite step
    equals plain Adam run with a zero gradient in the skipped step's place
    only for the step count (its moments are those of the earlier steps)."""
    params = _params_like(rng)
    st = {}
    g1 = _grads_with_norm(rng, params, 1.0)
    p1 = cnn.adam_step_clipped(params, g1, st, 1e-2)
    snap = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    bad = [(a.copy(), b.copy()) for a, b in g1]
    bad[0][0].flat[0] = np.nan
    p2 = cnn.adam_step_clipped(p1, bad, st, 1e-2)
    for (wa, ba), (wb, bb) in zip(p1, p2):
        np.testing.assert_array_equal(wa, wb)
        np.testing.assert_array_equal(ba, bb)
    assert st["t"] == 2 and st["run_norm"] == snap["run_norm"]
    for k, v in snap.items():
        if isinstance(k, tuple):
            np.testing.assert_array_equal(st[k], v)
    # the third step is bias-corrected with t = 3
    g3 = _grads_with_norm(rng, params, 1.0)
    ref_state = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in snap.items()}
    ref_state["t"] = 2
    want = cnn.adam_step(p2, g3, ref_state, 1e-2)
    got = cnn.adam_step_clipped(p2, g3, st, 1e-2)
    for (wa, ba), (wb, bb) in zip(want, got):
        np.testing.assert_allclose(wa, wb, rtol=1e-15)
        np.testing.assert_allclose(ba, bb, rtol=1e-15)
