"""Reconstruction quality with a least-squares scale fit (Sec. V-A, eq. psnr).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

import numpy as np


def scale_fit(r_hat, r_true):
    """beta* = r_hat^T r / ||r_hat||^2, the scale that best matches r_hat to r."""
    a = np.asarray(r_hat, dtype=np.float64).ravel()
    b = np.asarray(r_true, dtype=np.float64).ravel()
    return float(a @ b / (a @ a))


def nrmse(r_hat, r_true):
    """Volumetric ||beta* r_hat - r|| / ||r||."""
    a = np.asarray(r_hat, dtype=np.float64)
    b = np.asarray(r_true, dtype=np.float64)
    bs = scale_fit(a, b)
    return float(np.linalg.norm(bs * a - b) / np.linalg.norm(b))


def psnr(r_hat, r_true):
    """10 log10(n / ||beta* r_hat - r||^2) (eq. psnr)."""
    a = np.asarray(r_hat, dtype=np.float64)
    b = np.asarray(r_true, dtype=np.float64)
    bs = scale_fit(a, b)
    return float(10.0 * np.log10(b.size / np.sum((bs * a - b) ** 2)))


def point_cloud(r, threshold):
    """The image as a point cloud (Sec. V-A): every voxel whose value exceeds
    `threshold`, as its (z, y, x) index (voxel units) and its value."""
    r = np.asarray(r, dtype=np.float64)
    idx = np.argwhere(r > threshold)
    return idx.astype(np.float64), r[tuple(idx.T)]


def point_cloud_metrics(r_hat, r_true, threshold_hat, threshold_true, cutoff):
    """eqs. pc-distance and nrmse by brute force.  Every reconstructed point
    p gets its nearest ground-truth point n(p) in space (ties: the first in
    (z, y, x) order); points farther than `cutoff` are removed and counted as
    false positives.  Over the kept points: the mean distance, and the NRMSE
    sqrt(sum (b r_hat_p - r_n(p))^2 / sum r_n(p)^2) with the minimising scale
    b = sum r_hat_p r_n(p) / sum r_hat_p^2.  Returns a dict."""
    P, rp = point_cloud(r_hat, threshold_hat)
    Q, rq = point_cloud(r_true, threshold_true)
    if len(P) == 0 or len(Q) == 0:
        return {"points": len(P), "kept": 0, "distance": float("nan"), "false_positive_rate": float("nan"),
                "nrmse": float("nan")}
    dist = np.empty(len(P))
    near = np.empty(len(P), dtype=np.int64)
    for i in range(len(P)):
        d2 = np.sum((Q - P[i]) ** 2, axis=1)
        j = int(np.argmin(d2))          # argmin returns the first of equal minima
        near[i] = j
        dist[i] = float(np.sqrt(d2[j]))
    keep = dist <= cutoff
    a = rp[keep]
    b = rq[near[keep]]
    beta = float(a @ b / (a @ a)) if a.size else float("nan")
    nr = float(np.sqrt(np.sum((beta * a - b) ** 2) / np.sum(b ** 2))) if a.size else float("nan")
    return {"points": int(len(P)), "kept": int(keep.sum()), "distance": float(dist[keep].mean()) if a.size else
            float("nan"), "false_positive_rate": float(1.0 - keep.mean()), "nrmse": nr, "beta": beta}
