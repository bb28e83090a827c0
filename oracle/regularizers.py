"""Comparison regularizers of Sec. V, used as the prior agent of Alg. 2 in
place of the deep prior: the l_{2,1} agent (l2 in cross-range, l1 in range)
and the isotropic total-variation agent, each the proximal map of its
regularizer; and the speckle average, the comparison reconstruction.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper names the regularizers and gives no formula or
parameter):
* l_{2,1}: the groups are the range slices; within a slice (the cross-range
  plane) the l2 norm, across slices (range) the l1 sum:
  R(r) = sum_z ||r[z, :, :]||_2.  Its proximal map with threshold tau
  (the regularization weight times the proximal parameter) scales each
  slice by max(0, 1 - tau / ||v_z||_2).
* TV: the isotropic 3D total variation with forward differences and
  Neumann boundaries (the difference leaving the volume is zero),
  TV(r) = sum_voxels sqrt((D_x r)^2 + (D_y r)^2 + (D_z r)^2).  Its proximal
  map argmin_r lam TV(r) + ||r - v||^2 / 2 has no closed form; it is taken
  as a fixed number of steps of Chambolle's dual projection iteration
  (J. Math. Imaging Vis. 20, 2004): with div the negative adjoint of the
  forward-difference gradient, p <- (p + tau grad(div p - v / lam)) /
  (1 + tau |grad(div p - v / lam)|) from p = 0, and r = v - lam div p.
  Its steps converge for tau <= 1/12 in three dimensions.
"""

import numpy as np

from .operator import apply_AH


def l21_prox(v, tau):
    """argmin_r sum_z ||r_z||_2 tau + ||r - v||^2 / 2 for v[nz, ny, nx]:
    block soft thresholding of each range slice."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    for z in range(v.shape[0]):
        nrm = float(np.sqrt(np.sum(v[z] ** 2)))
        scale = max(0.0, 1.0 - tau / nrm) if nrm > 0.0 else 0.0
        out[z] = scale * v[z]
    return out


def l21_norm(r):
    r = np.asarray(r, dtype=np.float64)
    return float(sum(np.sqrt(np.sum(r[z] ** 2)) for z in range(r.shape[0])))


def grad3(u):
    """Forward differences along z, y, x with the last difference of each
    axis set to zero (Neumann boundary); returns g[3, nz, ny, nx]."""
    u = np.asarray(u, dtype=np.float64)
    g = np.zeros((3,) + u.shape)
    g[0, :-1] = u[1:] - u[:-1]
    g[1, :, :-1] = u[:, 1:] - u[:, :-1]
    g[2, :, :, :-1] = u[:, :, 1:] - u[:, :, :-1]
    return g


def div3(p):
    """Divergence, the negative adjoint of grad3: <grad3 u, p> = -<u, div3 p>."""
    p = np.asarray(p, dtype=np.float64)
    d = np.zeros(p.shape[1:])
    for a in range(3):
        q = np.moveaxis(p[a], a, 0)
        dq = np.zeros_like(q)
        n = q.shape[0]
        if n > 1:
            dq[0] = q[0]
            dq[1:n - 1] = q[1:n - 1] - q[:n - 2]
            dq[n - 1] = -q[n - 2]
        d += np.moveaxis(dq, 0, a)
    return d


def tv_norm(r):
    g = grad3(r)
    return float(np.sum(np.sqrt(np.sum(g ** 2, axis=0))))


def tv_prox(v, lam, iters, tau=1.0 / 12.0):
    """Chambolle's dual projection iteration for argmin_r lam TV(r) +
    ||r - v||^2 / 2, `iters` steps from p = 0.  Returns (r, p)."""
    v = np.asarray(v, dtype=np.float64)
    p = np.zeros((3,) + v.shape)
    for _ in range(iters):
        g = grad3(div3(p) - v / lam)
        mag = np.sqrt(np.sum(g ** 2, axis=0))
        p = (p + tau * g) / (1.0 + tau * mag)
    return v - lam * div3(p), p


def tv_dual_gap(v, lam, r, p):
    """Gap between the primal objective lam TV(r) + ||r - v||^2 / 2 and the
    dual objective of a feasible p (|p| <= 1 at every voxel):
    ||v||^2 / 2 - ||v - lam div p||^2 / 2.  Non-negative; zero at the
    solution."""
    primal = lam * tv_norm(r) + 0.5 * float(np.sum((r - v) ** 2))
    dual = 0.5 * float(np.sum(v ** 2)) - 0.5 * float(np.sum((v - lam * div3(p)) ** 2))
    return primal - dual


def speckle_average(y, mask):
    """r_SA = (1/L) sum_l |A^H y_l|^2 (the comparison reconstruction of Sec. V,
    and the initial image of Alg. 2)."""
    y = np.asarray(y, dtype=np.complex128)
    acc = np.zeros(y.shape[1:])
    for l in range(y.shape[0]):
        acc += np.abs(apply_AH(y[l], mask)) ** 2
    return acc / y.shape[0]
