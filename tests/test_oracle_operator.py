"""Pins of the oracle's aperture operator (Sec. II-B, eq. A) against brute-force
DFT matrices, Parseval, adjointness and the projector structure of A^H A."""

import numpy as np
import pytest

import oracle


def dft_matrix(n):
    """Orthonormal DFT matrix written out element by element."""
    m = np.empty((n, n), dtype=np.complex128)
    for k in range(n):
        for j in range(n):
            m[k, j] = np.exp(-2j * np.pi * k * j / n) / np.sqrt(n)
    return m


def brute_dft2(x):
    ny, nx = x.shape[-2:]
    fy, fx = dft_matrix(ny), dft_matrix(nx)
    return np.einsum("uy,zyx,vx->zuv", fy, x, fx)


def brute_pupil(ny, nx, radius):
    out = np.zeros((ny, nx), dtype=bool)
    for u in range(ny):
        for v in range(nx):
            su = u if u < ny - u else u - ny
            sv = v if v < nx - v else v - nx
            out[u, v] = su * su + sv * sv <= radius * radius
    return out


@pytest.mark.parametrize("shape", [(4, 8, 8), (3, 4, 8), (2, 6, 12)])
def test_dft_matches_brute_force(rng, shape):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np.testing.assert_allclose(oracle.dft2(x), brute_dft2(x), atol=1e-12)
    xh = np.conj(brute_dft2(np.conj(x)))  # F^H x = conj(F conj(x)) for symmetric F
    np.testing.assert_allclose(oracle.idft2(x), xh, atol=1e-12)


def test_parseval_and_inverse(rng):
    x = rng.standard_normal((5, 16, 16)) + 1j * rng.standard_normal((5, 16, 16))
    assert np.isclose(np.linalg.norm(oracle.dft2(x)), np.linalg.norm(x), rtol=1e-13)
    np.testing.assert_allclose(oracle.idft2(oracle.dft2(x)), x, atol=1e-12)


# Gauss circle numbers N(R) = #{(i, j) in Z^2 : i^2 + j^2 <= R^2}
# (OEIS A000328: N(2)=13, N(3)=29, N(8)=197).
@pytest.mark.parametrize("n,radius,count", [(16, 2, 13), (16, 3, 29), (32, 8, 197)])
def test_pupil_counts_gauss_circle(n, radius, count):
    m = oracle.pupil_mask(n, n, radius)
    assert int(m.sum()) == count
    np.testing.assert_array_equal(m, brute_pupil(n, n, radius))
    assert oracle.aperture_fraction(m) == count / (n * n)


def test_pupil_large_grids_match_brute_force():
    for n, radius in [(256, 64), (128, 32), (192, 48)]:
        np.testing.assert_array_equal(oracle.pupil_mask(n, n, radius),
                                      brute_pupil(n, n, radius))


def test_A_matches_dense_construction(rng):
    nz, ny, nx = 2, 4, 8
    mask = brute_pupil(ny, nx, 2)
    x = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    want = mask[None] * brute_dft2(x)
    np.testing.assert_allclose(oracle.apply_A(x, mask), want, atol=1e-12)


def test_adjoint_identity(rng):
    mask = oracle.pupil_mask(16, 16, 4)
    x = rng.standard_normal((3, 16, 16)) + 1j * rng.standard_normal((3, 16, 16))
    y = rng.standard_normal((3, 16, 16)) + 1j * rng.standard_normal((3, 16, 16))
    lhs = np.vdot(oracle.apply_A(x, mask), y)
    rhs = np.vdot(x, oracle.apply_AH(y, mask))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_normal_operator_is_projector_with_pupil_trace():
    nz, ny, nx = 2, 8, 8
    mask = oracle.pupil_mask(ny, nx, 2)
    n = nz * ny * nx
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        cols.append(oracle.apply_AHA(e.reshape(nz, ny, nx), mask).ravel())
    P = np.stack(cols, axis=1)
    np.testing.assert_allclose(P, P.conj().T, atol=1e-13)
    np.testing.assert_allclose(P @ P, P, atol=1e-13)
    assert np.isclose(np.trace(P).real, mask.sum() * nz, atol=1e-10)
    ev = np.linalg.eigvalsh(P)
    assert np.all((np.abs(ev) < 1e-10) | (np.abs(ev - 1) < 1e-10))


def test_all_pass_pupil_is_identity(rng):
    mask = np.ones((8, 8), dtype=bool)
    x = rng.standard_normal((3, 8, 8)) + 1j * rng.standard_normal((3, 8, 8))
    np.testing.assert_allclose(oracle.apply_AHA(x, mask), x, atol=1e-13)
    assert oracle.aperture_fraction(mask) == 1.0


def test_contraction(rng):
    mask = oracle.pupil_mask(16, 16, 5)
    x = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    assert np.linalg.norm(oracle.apply_A(x, mask)) <= np.linalg.norm(x)


def test_A_AH_is_pupil_restriction(rng):
    """A A^H = D(a): the initial residual y - A (s A^H y) is (1 - s) D(a) y."""
    mask = oracle.pupil_mask(16, 16, 4)
    y = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    for s in (1.0, 0.5, 1.0 / oracle.aperture_fraction(mask)):
        res = mask * (y - oracle.apply_A(s * oracle.apply_AH(y, mask), mask))
        np.testing.assert_allclose(res, (1 - s) * mask * y, atol=1e-12)


# ---------------------------------------------------------------------------
# The 3D operator with a zero-padded (cylinder) aperture

def test_dft3_matches_brute_force(rng):
    nz, ny, nx = 4, 3, 5
    x = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    want = np.zeros_like(x)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for w in range(nz):
        for u in range(ny):
            for v in range(nx):
                ph = np.exp(-2j * np.pi * (w * zz / nz + u * yy / ny + v * xx / nx))
                want[w, u, v] = np.sum(x * ph) / np.sqrt(nz * ny * nx)
    np.testing.assert_allclose(oracle.dft3(x), want, atol=1e-12)
    np.testing.assert_allclose(oracle.idft3(oracle.dft3(x)), x, atol=1e-12)


def test_range_box_counts_and_centre():
    for nz, k in ((8, 8), (8, 5), (12, 8), (9, 4), (16, 1)):
        box = oracle.range_box(nz, k)
        assert box.sum() == k and box[0]
        sw = np.fft.fftfreq(nz) * nz
        assert sw[box].min() == -(k // 2) and sw[box].max() == (k + 1) // 2 - 1


def test_cylinder_operator_adjoint_projector_and_alpha(rng):
    nz, ny, nx = 12, 16, 16
    m = oracle.cylinder_mask(nz, ny, nx, 5.0, 8)
    x = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    y = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    lhs = np.vdot(oracle.apply_A(x, m), y)
    rhs = np.vdot(x, oracle.apply_AH(y, m))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    p1 = oracle.apply_AHA(x, m)
    np.testing.assert_allclose(oracle.apply_AHA(p1, m), p1, atol=1e-12)
    disk = oracle.pupil_mask(ny, nx, 5.0).sum()
    assert oracle.aperture_fraction(m) == disk * 8 / (nz * ny * nx)
    # trace of the projector
    assert abs(np.count_nonzero(m) - disk * 8) == 0


def test_full_range_box_equals_per_slice_operator(rng):
    """With every range frequency passed, the 3D operator is the per-slice
    operator followed by a unitary range DFT: same A^H A, same norms."""
    nz, ny, nx = 6, 16, 8
    m2 = oracle.pupil_mask(ny, nx, 4.0)
    m3 = oracle.cylinder_mask(nz, ny, nx, 4.0, nz)
    x = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    np.testing.assert_allclose(oracle.apply_AHA(x, m3), oracle.apply_AHA(x, m2), atol=1e-12)
    np.testing.assert_allclose(oracle.apply_A(x, m3), np.fft.fft(oracle.apply_A(x, m2), axis=0, norm="ortho"),
                               atol=1e-12)


def test_full_range_box_clamp_run_equals_per_slice_run(rng):
    """A CLAMP run on 3D data with a full range box reproduces the per-slice
    run on the same looks (the 3D data are the range DFT of the 2D data)."""
    nz, ny, nx, L = 4, 16, 16, 2
    m2 = oracle.pupil_mask(ny, nx, 4.0)
    m3 = oracle.cylinder_mask(nz, ny, nx, 4.0, nz)
    r = rng.uniform(0.1, 1.0, (nz, ny, nx))
    g = np.sqrt(r) * (rng.standard_normal((L, nz, ny, nx)) + 1j * rng.standard_normal((L, nz, ny, nx))) / np.sqrt(2)
    y2 = oracle.apply_A(g, m2) + 0.01 * m2 * (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape))
    y3 = np.fft.fft(y2, axis=1, norm="ortho")
    s2, _ = oracle.clamp_run(y2, 4.0, 0.01, 1e-3, 5, with_prior=False, mask=m2)
    s3, _ = oracle.clamp_run(y3, 4.0, 0.01, 1e-3, 5, with_prior=False, mask=m3)
    np.testing.assert_allclose(s3.r, s2.r, rtol=1e-9)
    np.testing.assert_allclose(s3.mu, s2.mu, atol=1e-9 * np.abs(s2.mu).max())
