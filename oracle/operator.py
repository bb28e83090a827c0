"""Aperture operator A = D(a) F and its adjoint (Sec. II-B, eq. A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two forms, chosen by the rank of the aperture mask:
- a 2D mask [ny, nx]: F is the orthonormal 2D DFT of each range slice
  (forward kernel exp(-2 pi i (u y / ny + v x / nx)) scaled by (nx ny)^-1/2)
  and a is the same pupil on every slice;
- a 3D mask [nz, ny, nx]: F is the orthonormal 3D DFT of eq. A and a the
  zero-padded aperture, a cylinder: the pupil disk times the range-frequency
  samples that hold data (Nt of the q Nt samples after zero-padding by q in
  range, Sec. II-A).
The 2D form equals the 3D one with a range box that passes every sample: the
range DFT is then a unitary change of data coordinates that leaves every
quantity of the algorithm unchanged.
"""

import numpy as np


def pupil_mask(ny, nx, radius):
    """Binary aperture a (eq. A): a circular pupil centred at DC, in signed DFT
    indices, including the boundary (ku^2 + kv^2 <= R^2)."""
    ku = np.fft.fftfreq(ny) * ny
    kv = np.fft.fftfreq(nx) * nx
    return (ku[:, None] ** 2 + kv[None, :] ** 2) <= float(radius) ** 2


def range_box(nz, k):
    """Range part of the zero-padded aperture: the k range-frequency samples
    nearest DC (signed indices -floor(k/2) .. ceil(k/2) - 1)."""
    kw = np.fft.fftfreq(nz) * nz
    return (kw >= -(k // 2)) & (kw <= (k + 1) // 2 - 1)


def cylinder_mask(nz, ny, nx, radius, k):
    """3D aperture: the pupil disk on the k range frequencies of range_box."""
    return range_box(nz, k)[:, None, None] & pupil_mask(ny, nx, radius)[None]


def aperture_fraction(mask):
    """alpha = ||a||_1 / n (Sec. III-B): the fraction of samples the pupil passes."""
    return float(np.count_nonzero(mask)) / mask.size


def dft2(x):
    """Orthonormal DFT of each range slice of x[..., ny, nx]."""
    return np.fft.fft2(x, axes=(-2, -1), norm="ortho")


def idft2(x):
    """Inverse orthonormal DFT of each range slice (F^H = F^-1)."""
    return np.fft.ifft2(x, axes=(-2, -1), norm="ortho")


def dft3(x):
    """Orthonormal 3D DFT of x[..., nz, ny, nx]."""
    return np.fft.fftn(x, axes=(-3, -2, -1), norm="ortho")


def idft3(x):
    """Inverse orthonormal 3D DFT."""
    return np.fft.ifftn(x, axes=(-3, -2, -1), norm="ortho")


def apply_A(x, mask):
    """A x = D(a) F x (eq. A); F per range slice for a 2D mask, 3D for a 3D mask."""
    return mask * (dft3(x) if mask.ndim == 3 else dft2(x))


def apply_AH(y, mask):
    """A^H y = F^H D(a) y."""
    return idft3(mask * y) if mask.ndim == 3 else idft2(mask * y)


def apply_AHA(x, mask):
    """A^H A x = F^H D(a) F x (D(a) is idempotent for a binary a)."""
    return apply_AH(apply_A(x, mask), mask)
