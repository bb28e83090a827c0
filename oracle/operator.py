"""Aperture operator A = D(a) F and its adjoint (Sec. II-B, eq. A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading used throughout: F is the orthonormal 2D DFT of each range slice
(forward kernel exp(-2 pi i (u y / ny + v x / nx)) scaled by (nx ny)^-1/2),
and a is the same binary pupil on every slice.  This equals the paper's 3D
operator whenever the range-frequency part of the aperture passes every
sample (zero-padding factor 1 in range): the range DFT is then a unitary
change of data coordinates that leaves every quantity of the algorithm
unchanged.
"""

import numpy as np


def pupil_mask(ny, nx, radius):
    """Binary aperture a (eq. A): a circular pupil centred at DC, in signed DFT
    indices, including the boundary (ku^2 + kv^2 <= R^2)."""
    ku = np.fft.fftfreq(ny) * ny
    kv = np.fft.fftfreq(nx) * nx
    return (ku[:, None] ** 2 + kv[None, :] ** 2) <= float(radius) ** 2


def aperture_fraction(mask):
    """alpha = ||a||_1 / n (Sec. III-B): the fraction of samples the pupil passes."""
    return float(np.count_nonzero(mask)) / mask.size


def dft2(x):
    """Orthonormal DFT of each range slice of x[..., ny, nx]."""
    return np.fft.fft2(x, axes=(-2, -1), norm="ortho")


def idft2(x):
    """Inverse orthonormal DFT of each range slice (F^H = F^-1)."""
    return np.fft.ifft2(x, axes=(-2, -1), norm="ortho")


def apply_A(x, mask):
    """A x = D(a) F x (eq. A)."""
    return mask * dft2(x)


def apply_AH(y, mask):
    """A^H y = F^H D(a) y."""
    return idft2(mask * y)


def apply_AHA(x, mask):
    """A^H A x = F^H D(a) F x (D(a) is idempotent for a binary a)."""
    return apply_AH(apply_A(x, mask), mask)
