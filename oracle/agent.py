"""EM-surrogate forward agent of one look (Sec. III-B, Alg. 2, App. A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (each listed with its reason in the design notes):
* sigma_w^2 is the data-noise variance sigma_eta^2 of eq. forward-model.
* The covariance diagonal uses the anchor r' in numerator and denominator:
  c = sigma_w^2 r' / (alpha r' + sigma_w^2).
* The step size is the exact minimiser of h along d (the objective that
  defines d), so its diagonal term uses omega = 1/(r' + sigma_w^2/alpha);
  mu moves to mu + gamma d with gamma >= 0, and gamma = 0 when d = 0.
* The quadratic surrogate direction point is xi = r'/beta when the
  derivative of rho at r' is positive and xi = beta r' otherwise (the tie
  gives r = r' either way); the update is clipped to the closed interval
  between r' and xi.
* beta_k = 1 + 2 / ln(k + 1) with k = 1, 2, ... the iteration number.
"""

import math

import numpy as np

from .operator import apply_A, apply_AH


def noise_floor_weight(r_anchor, sigma_w2, alpha):
    """omega = 1 / (r' + sigma_w^2 / alpha): the noise-floored prior weight of
    eq. mu-objective."""
    return 1.0 / (r_anchor + sigma_w2 / alpha)


def h_objective(mu, y, r_anchor, mask, sigma_w2, alpha):
    """h(g; y, r') = ||y - A g||^2 / (2 sigma_w^2) + g^H D(omega) g / 2 (eq. mu-objective)."""
    resid = y - apply_A(mu, mask)
    omega = noise_floor_weight(r_anchor, sigma_w2, alpha)
    return (0.5 / sigma_w2) * float(np.sum(np.abs(resid) ** 2)) + \
        0.5 * float(np.sum(omega * np.abs(mu) ** 2))


def neg_grad_h(mu, y, r_anchor, mask, sigma_w2, alpha):
    """d = -grad h(mu) (eq. h-gradient), the steepest-descent direction in the
    real coordinates (Re g, Im g):  d = A^H (y - A mu) / sigma_w^2 - omega * mu."""
    omega = noise_floor_weight(r_anchor, sigma_w2, alpha)
    return apply_AH(y - apply_A(mu, mask), mask) / sigma_w2 - omega * mu


def exact_step(d, r_anchor, mask, sigma_w2, alpha):
    """gamma* = argmin_gamma h(mu + gamma d) (the gamma* equation of Sec. III-B).

    With d = -grad h, the numerator of the paper's expression equals ||d||^2
    and the curvature along d is ||A d||^2 / sigma_w^2 + sum omega |d|^2.
    Returns (gamma, ||d||^2, ||A d||^2, sum omega |d|^2)."""
    omega = noise_floor_weight(r_anchor, sigma_w2, alpha)
    dd = float(np.sum(np.abs(d) ** 2))
    ad = float(np.sum(np.abs(apply_A(d, mask)) ** 2))
    wd = float(np.sum(omega * np.abs(d) ** 2))
    den = ad / sigma_w2 + wd
    gamma = dd / den if dd > 0.0 else 0.0
    return gamma, dd, ad, wd


def cov_diag(r_anchor, sigma_w2, alpha):
    """c_j = sigma_w^2 r'_j / (alpha r'_j + sigma_w^2): the diagonal of the
    posterior covariance when A^H A is replaced by alpha I (Sec. III-B)."""
    return sigma_w2 * r_anchor / (alpha * r_anchor + sigma_w2)


def beta_schedule(k):
    """Interval factor beta = 1 + 2 / log(k) of App. A, with natural log and
    the 1-based iteration number shifted by one so that beta_1 is finite."""
    return 1.0 + 2.0 / math.log(k + 1.0)


def qs_prox(r_anchor, s, v, sigma2, beta):
    """Quadratic-surrogate proximal update of App. A, voxel by voxel.

    rho_j(r) = r / r'_j + s_j / r + (r - v_j)^2 / (2 sigma^2)   (eq. g, with
    s = c + |mu|^2).  The linearised-log part q(r) = r/r' + s/r is replaced by a
    quadratic a r^2/2 + b r whose derivative interpolates q' at r' and at xi
    (eq. quadratic-surrogate); xi lies towards the minimum of rho.  The
    minimiser of that quadratic plus the proximal term is
    r = (v - sigma^2 b) / (1 + sigma^2 a) (eq. r-update2), clipped to the
    interval between r' and xi (eq. r-update)."""
    rp = r_anchor
    dq_rp = 1.0 / rp - s / rp ** 2                  # q'(r')
    drho_rp = dq_rp + (rp - v) / sigma2             # rho'(r')
    xi = np.where(drho_rp > 0.0, rp / beta, beta * rp)
    dq_xi = 1.0 / rp - s / xi ** 2                  # q'(xi)
    a = (dq_xi - dq_rp) / (xi - rp)                 # slope of the interpolated q'
    b = dq_rp - a * rp
    r_new = (v - sigma2 * b) / (1.0 + sigma2 * a)
    lo = np.minimum(rp, xi)
    hi = np.maximum(rp, xi)
    return np.clip(r_new, lo, hi)


def surrogate_prox_objective(r, s, v, sigma2):
    """phi_j(r) = log r + s_j / r + (r - v_j)^2 / (2 sigma^2): the voxel term of
    the EM surrogate plus the proximal term (eq. surrogate-prox)."""
    return np.log(r) + s / r + (r - v) ** 2 / (2.0 * sigma2)


def exact_prox(s, v, sigma2):
    """Exact proximal map of the EM surrogate (eq. surrogate-prox), voxel by
    voxel: argmin over r > 0 of phi(r) = log r + s/r + (r - v)^2/(2 sigma^2).

    phi'(r) = 1/r - s/r^2 + (r - v)/sigma^2; multiplied by sigma^2 r^2 it is
    the cubic r^3 - v r^2 + sigma^2 r - sigma^2 s, whose value at 0 is
    -sigma^2 s < 0, so it has a positive root.  The roots are the eigenvalues
    of the cubic's companion matrix; phi is not convex for r > 2 s, so when
    there are several positive roots the one with the smallest phi is kept."""
    s, v = np.broadcast_arrays(np.asarray(s, dtype=np.float64), np.asarray(v, dtype=np.float64))
    shape = s.shape
    s = s.ravel()
    v = v.ravel()
    comp = np.zeros((s.size, 3, 3))
    comp[:, 0, 0] = v                  # companion matrix of r^3 + c2 r^2 + c1 r + c0
    comp[:, 0, 1] = -sigma2            # with c2 = -v, c1 = sigma^2, c0 = -sigma^2 s
    comp[:, 0, 2] = sigma2 * s
    comp[:, 1, 0] = 1.0
    comp[:, 2, 1] = 1.0
    roots = np.linalg.eigvals(comp)
    scale = np.maximum(np.abs(roots), 1e-300)
    real = (np.abs(roots.imag) <= 1e-7 * scale) & (roots.real > 0.0)
    cand = np.where(real, roots.real, np.nan)
    with np.errstate(invalid="ignore", divide="ignore"):
        phi = surrogate_prox_objective(cand, s[:, None], v[:, None], sigma2)
    phi = np.where(real, phi, np.inf)
    best = np.argmin(phi, axis=1)
    out = cand[np.arange(s.size), best]
    return out.reshape(shape)


def forward_agent(mu, y, r_anchor, v, mask, sigma_w2, sigma2, alpha, beta, r_update="quadratic"):
    """One application of the CLAMP forward agent for one look (Alg. 2, the
    body of the per-look loop): covariance diagonal, one exact steepest-descent
    step on mu, and the surrogate proximal update of r at v.

    r_update selects the r-update: "quadratic" is the quadratic surrogate of
    App. A (the paper's choice), "exact" the exact proximal map of the EM
    surrogate (eq. surrogate-prox, a cubic per voxel).

    Returns (mu_new, r_new, info) with info holding gamma, ||d||^2, ||A d||^2,
    sum omega |d|^2 and h before and after the mu step."""
    c = cov_diag(r_anchor, sigma_w2, alpha)
    d = neg_grad_h(mu, y, r_anchor, mask, sigma_w2, alpha)
    gamma, dd, ad, wd = exact_step(d, r_anchor, mask, sigma_w2, alpha)
    h0 = h_objective(mu, y, r_anchor, mask, sigma_w2, alpha)
    mu_new = mu + gamma * d
    h1 = h_objective(mu_new, y, r_anchor, mask, sigma_w2, alpha)
    s = c + np.abs(mu_new) ** 2
    if r_update == "exact":
        r_new = exact_prox(s, v, sigma2)
    else:
        r_new = qs_prox(r_anchor, s, v, sigma2, beta)
    info = {"gamma": gamma, "dd": dd, "ad": ad, "wd": wd, "h0": h0, "h1": h1,
            "d": d}
    return mu_new, r_new, info
