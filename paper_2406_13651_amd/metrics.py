"""Reconstruction quality on the host (Sec. V-A): PSNR and volumetric NRMSE
with the least-squares scale beta* (eq. psnr), and the point-cloud metrics
(eqs. pc-distance and nrmse) with a k-d tree nearest-neighbour search.

The point cloud of an image is every voxel above a threshold, at its (z, y,
x) index in voxel units.  Each reconstructed point takes its nearest
ground-truth point (among equidistant ones, the first in (z, y, x) order);
points farther than `cutoff` are removed and counted as false positives; the
mean distance and the surface NRMSE (with its minimising scale) are taken
over the kept points.  The paper's cutoff is three times the Rayleigh
resolution; rayleigh_cutoff gives that in voxels for a circular pupil.
"""

from __future__ import annotations

import numpy as np


def scale_fit(r_hat, r_true):
    a = np.asarray(r_hat, dtype=np.float64).ravel()
    b = np.asarray(r_true, dtype=np.float64).ravel()
    return float(a @ b / (a @ a))


def nrmse(r_hat, r_true):
    """||beta* r_hat - r|| / ||r|| with beta* = r_hat^T r / ||r_hat||^2."""
    a = np.asarray(r_hat, dtype=np.float64)
    b = np.asarray(r_true, dtype=np.float64)
    return float(np.linalg.norm(scale_fit(a, b) * a - b) / np.linalg.norm(b))


def psnr(r_hat, r_true):
    """10 log10(n / ||beta* r_hat - r||^2) (eq. psnr)."""
    a = np.asarray(r_hat, dtype=np.float64)
    b = np.asarray(r_true, dtype=np.float64)
    return float(10.0 * np.log10(b.size / np.sum((scale_fit(a, b) * a - b) ** 2)))


def rayleigh_cutoff(n, radius, factor=3.0):
    """`factor` times the Rayleigh resolution 1.22 n / (2 R) voxels of a
    circular pupil of radius R samples in an n-point grid."""
    return factor * 1.22 * n / (2.0 * radius)


def _nearest(tree, P, count):
    """Index of each point's nearest tree point, ties to the lowest index."""
    k = min(16, count)
    while True:
        d, j = tree.query(P, k=k)
        if k == 1:
            return d, j
        dmin = d[:, :1]
        tied = d == dmin
        if k == count or not np.any(tied[:, -1]):
            big = np.iinfo(np.int64).max
            jj = np.where(tied, j, big)
            return d[:, 0], jj.min(axis=1)
        k = min(count, 2 * k)


def point_cloud_metrics(r_hat, r_true, threshold_hat, threshold_true, cutoff):
    """Mean distance, false-positive rate and surface NRMSE of r_hat's point
    cloud against r_true's (eqs. pc-distance and nrmse)."""
    from scipy.spatial import cKDTree
    r_hat = np.asarray(r_hat, dtype=np.float64)
    r_true = np.asarray(r_true, dtype=np.float64)
    P = np.argwhere(r_hat > threshold_hat).astype(np.float64)
    Q = np.argwhere(r_true > threshold_true).astype(np.float64)
    if len(P) == 0 or len(Q) == 0:
        return {"points": int(len(P)), "kept": 0, "distance": float("nan"), "false_positive_rate": float("nan"),
                "nrmse": float("nan"), "beta": float("nan")}
    rp = r_hat[tuple(P.astype(np.int64).T)]
    rq = r_true[tuple(Q.astype(np.int64).T)]
    dist, near = _nearest(cKDTree(Q), P, len(Q))
    keep = dist <= cutoff
    a, b = rp[keep], rq[near[keep]]
    if a.size == 0:
        return {"points": int(len(P)), "kept": 0, "distance": float("nan"), "false_positive_rate": 1.0,
                "nrmse": float("nan"), "beta": float("nan")}
    beta = float(a @ b / (a @ a))
    return {"points": int(len(P)), "kept": int(keep.sum()), "distance": float(dist[keep].mean()),
            "false_positive_rate": float(1.0 - keep.mean()),
            "nrmse": float(np.sqrt(np.sum((beta * a - b) ** 2) / np.sum(b ** 2))), "beta": beta}
