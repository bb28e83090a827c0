"""Fixed Gaussian smoothing prior agent H (the prior slot of Alg. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's prior is a trained 3D U-Net (Sec. III-C).  The plain method here
uses a fixed smoother instead: a separable 3D Gaussian with standard deviation
1 voxel, 7 taps per axis, normalised to unit sum, with periodic boundaries.
Its DFT is strictly positive, so it is the proximal map of a convex quadratic
and the consensus theory of Sec. IV covers it.
"""

import numpy as np


def gaussian_taps(sigma=1.0, taps=7):
    """Normalised 1D Gaussian kernel on offsets -(taps//2) .. taps//2."""
    half = taps // 2
    k = np.arange(-half, half + 1, dtype=np.float64)
    g = np.exp(-0.5 * (k / sigma) ** 2)
    return g / g.sum()


def gaussian_smooth(x, sigma=1.0, taps=7):
    """Separable periodic smoothing of x[nz, ny, nx] along x, then y, then z."""
    g = gaussian_taps(sigma, taps)
    half = taps // 2
    out = np.asarray(x, dtype=np.float64)
    for axis in (2, 1, 0):
        acc = np.zeros_like(out)
        for i, off in enumerate(range(-half, half + 1)):
            acc += g[i] * np.roll(out, -off, axis=axis)
        out = acc
    return out
