"""MACE consensus: weighted average G, Mann iteration and convergence measures
(Sec. III-A, eqs. mace and mann, Alg. 1; Sec. V-A eqs. mace-convergence-error
and residual).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings: the weighted average is w_bar = sum_j upsilon_j w_j with
sum upsilon = 1 (the extra 1/(L+1) factor in the text would normalise twice);
the convergence error compares the agents' outputs F(w) on the current state
with G(w) before the Mann update, in the unweighted 2-norm over the stack.
"""

import numpy as np


def agent_weights(looks, with_prior=True):
    """upsilon_l = 1/(2L) for the L forward agents and 1/2 for the prior
    (Sec. III-A); 1/L each when the run has forward agents only."""
    if with_prior:
        return np.array([0.5 / looks] * looks + [0.5], dtype=np.float64)
    return np.full(looks, 1.0 / looks, dtype=np.float64)


def weighted_average(stack, upsilon):
    """w_bar = sum_j upsilon_j w_j over the leading (agent) axis."""
    return np.tensordot(upsilon, stack, axes=(0, 0))


def mann_step(w, r, upsilon, rho):
    """Alg. 1: x = 2 r - w;  w <- w + 2 rho (G(x) - r), with r = F(w) given.
    Equivalent to w <- (1 - rho) w + rho T w with T = (2G - I)(2F - I)."""
    x = 2.0 * r - w
    xbar = weighted_average(x, upsilon)
    return w + 2.0 * rho * (xbar[None] - r)


def convergence_error(r, w, upsilon):
    """||F(w) - G(w)|| / ||G(w)|| with G(w) = [w_bar, ..., w_bar]
    (eq. mace-convergence-error)."""
    wbar = weighted_average(w, upsilon)
    num = float(np.sum((r - wbar[None]) ** 2))
    den = float(r.shape[0] * np.sum(wbar ** 2))
    return float(np.sqrt(num / den))


def mu_residual(dd_per_look, ahy2_per_look, sigma_w2):
    """mu-residual of eq. residual, in its noise-floored form: with h the
    objective that the mu-step minimises, C^-1 mu - A^H y / sigma_w^2 is -d, so
    each look contributes ||d|| / ||A^H y / sigma_w^2||, averaged over looks."""
    dd = np.asarray(dd_per_look, dtype=np.float64)
    ahy = np.sqrt(np.asarray(ahy2_per_look, dtype=np.float64)) / sigma_w2
    return float(np.mean(np.sqrt(dd) / ahy))
