"""Pins of the oracle's forward agent (Sec. III-B, App. A) against finite
differences, a numerical line search, closed forms, a dense solve and the
roots of the exact-prox cubic."""

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle


def _problem(rng, shape=(2, 8, 8), radius=2.5, sigma_w2=0.3):
    mask = oracle.pupil_mask(shape[1], shape[2], radius)
    alpha = oracle.aperture_fraction(mask)
    y = mask * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    mu = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    r_anchor = rng.uniform(0.1, 2.0, shape)
    return mask, alpha, y, mu, r_anchor, sigma_w2


def test_gradient_matches_finite_differences(rng):
    mask, alpha, y, mu, rp, s2 = _problem(rng)
    d = oracle.neg_grad_h(mu, y, rp, mask, s2, alpha)
    for _ in range(5):
        delta = rng.standard_normal(mu.shape) + 1j * rng.standard_normal(mu.shape)
        eps = 1e-5
        hp = oracle.h_objective(mu + eps * delta, y, rp, mask, s2, alpha)
        hm = oracle.h_objective(mu - eps * delta, y, rp, mask, s2, alpha)
        fd = (hp - hm) / (2 * eps)
        # dh/dt along delta = Re <grad, delta> and grad = -d in (Re, Im) coordinates
        assert np.isclose(fd, -np.vdot(d, delta).real, rtol=1e-7)


def test_exact_step_is_line_minimum(rng):
    mask, alpha, y, mu, rp, s2 = _problem(rng)
    d = oracle.neg_grad_h(mu, y, rp, mask, s2, alpha)
    gamma, dd, ad, wd = oracle.exact_step(d, rp, mask, s2, alpha)
    res = minimize_scalar(lambda g: oracle.h_objective(mu + g * d, y, rp, mask, s2, alpha),
                          bracket=(0.0, 1.0), tol=1e-12)
    assert gamma > 0
    assert np.isclose(gamma, res.x, rtol=1e-6)


def test_mu_step_decrement_is_half_gamma_dd(rng):
    mask, alpha, y, mu, rp, s2 = _problem(rng)
    v = rng.uniform(0.1, 2.0, mu.shape)
    mu1, r1, info = oracle.forward_agent(mu, y, rp, v, mask, s2, 0.1, alpha, 2.0)
    assert info["h1"] <= info["h0"]
    assert np.isclose(info["h0"] - info["h1"], 0.5 * info["gamma"] * info["dd"], rtol=1e-9)


def test_zero_direction_gives_zero_step():
    mask = oracle.pupil_mask(8, 8, 2)
    d = np.zeros((1, 8, 8), dtype=np.complex128)
    gamma, dd, _, _ = oracle.exact_step(d, np.ones((1, 8, 8)), mask, 0.1, 0.2)
    assert gamma == 0.0 and dd == 0.0


def test_all_pass_constant_anchor_one_step_closed_form(rng):
    """a = 1, constant r': h is isotropic, so one exact steepest-descent step
    lands on mu* = A^H y (r' + s)/(r' + 2 s) (the closed-form mu-update of the
    aperture ablation, Sec. V)."""
    shape = (2, 8, 8)
    mask = np.ones(shape[1:], dtype=bool)
    s2 = 0.4
    y = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    rp = np.full(shape, 0.7)
    mu0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    mu1, _, _ = oracle.forward_agent(mu0, y, rp, rp, mask, s2, 0.1, 1.0, 2.0)
    want = oracle.apply_AH(y, mask) * (0.7 + s2) / (0.7 + 2 * s2)
    np.testing.assert_allclose(mu1, want, atol=1e-12)


def test_mu_steps_converge_to_dense_solve(rng):
    """Fixed anchor: repeated steps minimise h, whose normal equations are
    ((1/s) A^H A + D(omega)) mu = A^H y / s; solved densely with A built from
    brute-force DFT matrices."""
    nz, ny, nx = 1, 6, 8
    mask = oracle.pupil_mask(ny, nx, 2)
    alpha = oracle.aperture_fraction(mask)
    s2 = 1.0
    y = mask * (rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx)))
    rp = rng.uniform(0.5, 1.0, (nz, ny, nx))
    fy = np.array([[np.exp(-2j * np.pi * k * j / ny) for j in range(ny)] for k in range(ny)]) / np.sqrt(ny)
    fx = np.array([[np.exp(-2j * np.pi * k * j / nx) for j in range(nx)] for k in range(nx)]) / np.sqrt(nx)
    F = np.kron(fy, fx)
    A = np.diag(mask.ravel().astype(float)) @ F
    omega = 1.0 / (rp.ravel() + s2 / alpha)
    M = A.conj().T @ A / s2 + np.diag(omega)
    mu_star = np.linalg.solve(M, A.conj().T @ y.ravel() / s2).reshape(nz, ny, nx)
    mu = np.zeros_like(y)
    for _ in range(200):
        d = oracle.neg_grad_h(mu, y, rp, mask, s2, alpha)
        gamma, *_ = oracle.exact_step(d, rp, mask, s2, alpha)
        mu = mu + gamma * d
    np.testing.assert_allclose(mu, mu_star, atol=1e-10)


def test_cov_diag_limits():
    s2, alpha = 0.3, 0.2
    assert np.isclose(oracle.cov_diag(1e12, s2, alpha), s2 / alpha, rtol=1e-9)
    assert np.isclose(oracle.cov_diag(1e-9, s2, alpha), 1e-9, rtol=1e-6)
    # exact posterior variance when A^H A = alpha I: 1 / (alpha/s2 + 1/r')
    rp = 0.37
    assert np.isclose(oracle.cov_diag(rp, s2, alpha), 1.0 / (alpha / s2 + 1.0 / rp), rtol=1e-14)


def test_beta_schedule_values():
    assert np.isclose(oracle.beta_schedule(1), 1 + 2 / np.log(2))
    assert oracle.beta_schedule(1) > oracle.beta_schedule(50) > oracle.beta_schedule(250) > 1


def _phi(r, rp, s, v, sigma2):
    return r / rp + s / r + (r - v) ** 2 / (2 * sigma2)


def test_qs_prox_fixed_point_solves_exact_prox_cubic(rng):
    """Iterating the surrogate update with the anchor moved to its output
    converges to a stationary point of log r + s/r + (r - v)^2/(2 sigma^2),
    i.e. a positive root of r^3 - v r^2 + sigma^2 r - sigma^2 s = 0 (the
    per-voxel cubic of the exact surrogate prox, Sec. III-B)."""
    m = 400
    s = rng.uniform(0.05, 2.0, m)
    v = rng.uniform(0.05, 2.0, m)
    sigma2 = rng.uniform(0.01, 1.0, m)
    r = rng.uniform(0.05, 2.0, m)
    for _ in range(3000):
        r = oracle.qs_prox(r, s, v, sigma2, 1.3)
    for j in range(m):
        roots = np.roots([1.0, -v[j], sigma2[j], -sigma2[j] * s[j]])
        real = roots[np.abs(roots.imag) < 1e-9].real
        pos = real[real > 0]
        assert np.min(np.abs(pos - r[j])) < 1e-8 * max(1.0, r[j]), (j, r[j], pos)


def test_qs_prox_large_sigma_gives_em_update(rng):
    """sigma^2 -> inf removes the proximal term; the fixed point of the MM
    update of log r + s/r is r = s."""
    s = rng.uniform(0.05, 2.0, 100)
    r = rng.uniform(0.05, 2.0, 100)
    for _ in range(2000):
        r = oracle.qs_prox(r, s, np.zeros_like(s), 1e14, 1.5)
    np.testing.assert_allclose(r, s, rtol=1e-8)


def test_qs_prox_stays_in_interval_and_descends_downward(rng):
    m = 20000
    rp = rng.uniform(0.01, 3.0, m)
    s = rng.uniform(0.0, 3.0, m)
    v = rng.uniform(0.0, 3.0, m)
    sigma2 = 10 ** rng.uniform(-3, 0, m)
    beta = rng.uniform(1.05, 4.0, m)
    r = oracle.qs_prox(rp, s, v, sigma2, beta)
    lo = np.minimum(rp / beta, rp) * (1 - 1e-12)
    hi = np.maximum(beta * rp, rp) * (1 + 1e-12)
    assert np.all((r >= lo) & (r <= hi)) and np.all(r > 0)
    drho = 1 / rp - s / rp ** 2 + (rp - v) / sigma2
    # moves go towards the minimum of rho
    assert np.all(np.where(drho > 0, r <= rp * (1 + 1e-12), r >= rp * (1 - 1e-12)))
    # the chord of the concave q' lies below q' on the way down: the surrogate
    # majorises rho there and the update never increases it
    down = r < rp
    assert np.all(_phi(r[down], rp[down], s[down], v[down], sigma2[down])
                  <= _phi(rp[down], rp[down], s[down], v[down], sigma2[down]) * (1 + 1e-12))


def test_qs_prox_tie_returns_anchor():
    rp, sigma2 = 0.8, 0.5
    s = 0.3
    # choose v so that rho'(r') = 0 exactly
    v = rp + sigma2 * (1 / rp - s / rp ** 2)
    assert np.isclose(oracle.qs_prox(np.array([rp]), np.array([s]), np.array([v]), sigma2, 2.0)[0], rp)


# ---------------------------------------------------------------------------
# Exact proximal map of the EM surrogate (eq. surrogate-prox)

def _grid_minimum(s, v, sigma2):
    """Global minimum of phi over r > 0 by a dense log grid refined with a
    bounded scalar minimisation around the best grid point (brute force)."""
    from scipy.optimize import minimize_scalar
    grid = np.geomspace(1e-8, 1e3, 200001)
    phi = oracle.surrogate_prox_objective(grid, s, v, sigma2)
    k = int(np.argmin(phi))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)]
    res = minimize_scalar(lambda r: oracle.surrogate_prox_objective(r, s, v, sigma2), bounds=(lo, hi),
                          method="bounded", options={"xatol": 1e-14 * hi})
    return res.x


def test_exact_prox_is_the_global_minimum(rng):
    for _ in range(60):
        s = float(rng.uniform(0.01, 2.0))
        v = float(rng.uniform(0.01, 3.0))
        sigma2 = float(10 ** rng.uniform(-3, 0.5))
        r = float(oracle.exact_prox(s, v, sigma2))
        rb = _grid_minimum(s, v, sigma2)
        phi = oracle.surrogate_prox_objective
        assert phi(r, s, v, sigma2) <= phi(rb, s, v, sigma2) + 1e-12 * max(1.0, abs(phi(rb, s, v, sigma2)))
        assert abs(r - rb) <= 1e-6 * max(r, rb) + 1e-12


def test_exact_prox_is_stationary_and_vectorised(rng):
    s = rng.uniform(0.01, 2.0, (7, 9))
    v = rng.uniform(0.01, 3.0, (7, 9))
    sigma2 = 0.05
    r = oracle.exact_prox(s, v, sigma2)
    assert r.shape == s.shape and np.all(r > 0)
    dphi = 1.0 / r - s / r ** 2 + (r - v) / sigma2
    assert np.max(np.abs(dphi) * r ** 2 * sigma2) <= 1e-10
    for i in (0, 3, 6):
        assert r[i, 2] == oracle.exact_prox(s[i, 2], v[i, 2], sigma2)


def test_exact_prox_limits():
    s = np.array([0.3, 1.2, 0.05])
    v = np.array([0.7, 0.1, 2.0])
    # a vanishing proximal term leaves the EM M-step r = s
    np.testing.assert_allclose(oracle.exact_prox(s, v, 1e9), s, rtol=1e-6)
    # a dominant proximal term keeps r at v, to first order in sigma^2:
    # r = v - sigma^2 (1/v - s/v^2) + O(sigma^4)
    sig = 1e-9
    np.testing.assert_allclose(oracle.exact_prox(s, v, sig), v - sig * (1.0 / v - s / v ** 2), rtol=1e-10)


def test_exact_prox_picks_the_lower_of_two_minima():
    # phi is not convex for r > 2 s: a small s with v far above it gives two
    # local minima, one near s and one near v
    s, v, sigma2 = 0.01, 1.0, 0.1
    r = float(oracle.exact_prox(s, v, sigma2))
    roots = np.roots([1.0, -v, sigma2, -sigma2 * s])
    pos = np.sort(roots[np.abs(roots.imag) < 1e-12].real)
    pos = pos[pos > 0]
    assert pos.size == 3  # two minima and the maximum between them
    phi = oracle.surrogate_prox_objective
    best = min(pos[[0, 2]], key=lambda x: phi(x, s, v, sigma2))
    assert abs(r - best) <= 1e-9 * best


def test_forward_agent_exact_r_update_uses_the_same_mu_step(rng):
    mask = oracle.pupil_mask(8, 8, 2.5)
    alpha = oracle.aperture_fraction(mask)
    y = rng.standard_normal((2, 8, 8)) + 1j * rng.standard_normal((2, 8, 8))
    mu = oracle.apply_AH(y, mask)
    rp = rng.uniform(0.2, 1.0, (2, 8, 8))
    w = rng.uniform(0.2, 1.0, (2, 8, 8))
    m_q, r_q, _ = oracle.forward_agent(mu, y, rp, w, mask, 0.1, 0.05, alpha, 2.0)
    m_e, r_e, info = oracle.forward_agent(mu, y, rp, w, mask, 0.1, 0.05, alpha, 2.0, r_update="exact")
    np.testing.assert_array_equal(m_q, m_e)
    s = oracle.cov_diag(rp, 0.1, alpha) + np.abs(m_e) ** 2
    np.testing.assert_allclose(r_e, oracle.exact_prox(s, w, 0.05))
