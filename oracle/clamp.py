"""CLAMP (Alg. 2) with the forward agents, an optional prior agent and the
Mann consensus step, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Initialisation (Alg. 2 and Sec. V-A): b_l = A^H y_l; r0 = (1/L) sum_l |b_l|^2
(floored at 1e-12 mean(r0) so every anchor is positive); mu_l = s_mu b_l with
s_mu = 1 as in Alg. 2 (Sec. V-A uses 1/alpha, available through mu_scale);
every forward agent's anchor r_l and every agent's state w_j start at r0.
Forward-only runs (no prior) use L agents with weights 1/L.

Parity unpinned as a whole trajectory (the paper prints no worked example);
its parts are pinned individually and the run is checked for a vanishing
consensus error and a monotone per-step decrease of h.
"""

import dataclasses

import numpy as np

from .agent import beta_schedule, forward_agent
from .mace import agent_weights, convergence_error, mann_step, mu_residual, weighted_average
from .operator import aperture_fraction, apply_AH, pupil_mask
from .prior import gaussian_smooth


@dataclasses.dataclass
class ClampState:
    mu: np.ndarray          # complex128 [L, nz, ny, nx]
    r: np.ndarray           # float64 [N, nz, ny, nx] agents' outputs (anchors for l < L)
    w: np.ndarray           # float64 [N, nz, ny, nx] Mann state
    k: int                  # iterations done
    ahy2: np.ndarray        # float64 [L] ||A^H y_l||^2


def clamp_init(y, mask, looks_with_prior=True, mu_scale=1.0):
    """Alg. 2 initialisation from looks y[L, nz, ny, nx]."""
    y = np.asarray(y, dtype=np.complex128)
    L = y.shape[0]
    b = np.stack([apply_AH(y[l], mask) for l in range(L)])
    r0 = np.mean(np.abs(b) ** 2, axis=0)
    r0 = np.maximum(r0, 1e-12 * float(np.mean(r0)))
    n_agents = L + 1 if looks_with_prior else L
    r = np.repeat(r0[None], n_agents, axis=0)
    w = r.copy()
    ahy2 = np.array([float(np.sum(np.abs(b[l]) ** 2)) for l in range(L)])
    return ClampState(mu=mu_scale * b, r=r, w=w, k=0, ahy2=ahy2)


def clamp_iteration(state, y, mask, sigma_w2, sigma2, rho=0.5, prior=None,
                    beta=None, r_update="quadratic", workers=1):
    """One pass of the Alg. 2 loop body.  `prior` is a callable H(w_{L+1}) or
    None for forward-only runs; `r_update` is "quadratic" (App. A) or "exact"
    (eq. surrogate-prox).  The looks' agents depend only on their own look's
    state, so `workers` > 1 applies them from a thread pool; each look's
    arithmetic is the same either way.  Returns a dict of diagnostics."""
    y = np.asarray(y, dtype=np.complex128)
    L = y.shape[0]
    alpha = aperture_fraction(mask)
    k = state.k + 1
    if beta is None:
        beta = beta_schedule(k)
    r_new = state.r.copy()
    mu_new = state.mu.copy()

    def agent(l):
        return forward_agent(state.mu[l], y[l], state.r[l], state.w[l], mask, sigma_w2, sigma2, alpha, beta,
                             r_update)

    if workers > 1 and L > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(workers, L)) as ex:
            results = list(ex.map(agent, range(L)))
    else:
        results = [agent(l) for l in range(L)]
    infos = []
    for l, (mu_l, r_l, info) in enumerate(results):
        mu_new[l] = mu_l
        r_new[l] = r_l
        infos.append(info)
    with_prior = state.w.shape[0] == L + 1
    if with_prior:
        r_new[L] = prior(state.w[L])
    ups = agent_weights(L, with_prior)
    m1 = convergence_error(r_new, state.w, ups)
    w_new = mann_step(state.w, r_new, ups, rho)
    state.mu, state.r, state.w, state.k = mu_new, r_new, w_new, k
    m2 = mu_residual([i["dd"] for i in infos], state.ahy2, sigma_w2)
    return {"k": k, "beta": beta, "conv_err": m1, "mu_residual": m2,
            "gamma": np.array([i["gamma"] for i in infos]),
            "dd": np.array([i["dd"] for i in infos]),
            "ad": np.array([i["ad"] for i in infos]),
            "h0": np.array([i["h0"] for i in infos]),
            "h1": np.array([i["h1"] for i in infos]),
            "wbar": weighted_average(w_new, ups)}


def clamp_run(y, radius, sigma_w2, sigma2, iters, rho=0.5, with_prior=True,
              mu_scale=1.0, prior_sigma=1.0, mask=None, r_update="quadratic", workers=1, keep_hist=True):
    """Alg. 2 for `iters` iterations; returns (state, list of diagnostics).
    keep_hist=False keeps only scalars and the last iteration's w_bar in the
    diagnostics (large volumes)."""
    y = np.asarray(y)
    if mask is None:
        mask = pupil_mask(y.shape[-2], y.shape[-1], radius)
    state = clamp_init(y, mask, with_prior, mu_scale)
    prior = (lambda x: gaussian_smooth(x, prior_sigma)) if with_prior else None
    hist = []
    for it in range(iters):
        h = clamp_iteration(state, y, mask, sigma_w2, sigma2, rho, prior, r_update=r_update, workers=workers)
        if not keep_hist and it < iters - 1:
            h.pop("wbar")
        hist.append(h)
    return state, hist
