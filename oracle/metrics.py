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
