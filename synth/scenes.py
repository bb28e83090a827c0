"""Faceted scenes, speckle and noisy pupil-plane looks (paper Sec. II-B, Sec. V-B).

Recipe (the paper's synthetic train model is not available, so seeded facet
scenes stand in for it, with the paper's structure):

* Scene.  The (x, y) plane is split into Voronoi facets around seeded sites.
  Each facet is a tilted plane: depth z = z0 + gx (x - xf) + gy (y - yf) with
  z0 ~ U[0.2, 0.8] nz.  Its tilt angle theta ~ U[0, 60 deg] and azimuth
  phi ~ U[0, 2 pi) give a Lambertian reflectivity cos(theta) (Sec. V-B: the
  reflectivity is proportional to the cosine between the normal and the
  viewing direction, normalised so the brightest point is 1), and a depth
  slope of 0.3 (nz/nx) tan(theta)/tan(60 deg) bins per pixel along phi.  Every
  pixel occupies one range bin, round(z) clamped to [0, nz-1]; all other
  voxels hold the background r_min.  Several objects (multi-object scenes)
  overlap with the nearest depth winning.
* Speckle.  g_l = sqrt(r) * z_l with z_l ~ CN(0, 1) per voxel and look
  (eq. g-given-r: g | r ~ CN(0, D(r))).
* Measurement.  y_l = D(a) F g_l + eta_l, with F the orthonormal 2D DFT of each
  range slice (forward sign e^{-2 pi i ...}), a a centred circular pupil of
  radius R in signed DFT indices (kx^2 + ky^2 <= R^2), and eta_l ~ CN(0,
  sigma_eta^2 I) on every sample (eq. forward-model).  The noise variance
  follows from the SNR as sigma_eta^2 = mean(r) 10^(-SNR/10).
* Seeds.  numpy SeedSequence([2406, 13651, config_id, scene_id]) spawns
  independent PCG64 streams for the scene, and per look for speckle and noise.

Everything is drawn and transformed in float64 and rounded once to complex64;
both sides of a comparison consume the same complex64 looks.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """One synthetic workload: grid, looks, pupil, SNR and scene recipe."""

    name: str
    nx: int
    ny: int
    nz: int
    looks: int
    radius: float
    snr_db: float
    n_facets: int
    r_min: float
    n_objects: int = 1
    config_id: int = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


# The five workloads: a tiny forward-only scene, the full-size plain method,
# a representative uneven-batch member, the learned-denoiser evaluation
# scene, and the large multi-object reconstruction.
CONFIGS = {
    "tiny": SceneSpec("tiny", 32, 32, 16, 4, 8.0, 20.0, 6, 0.1, 1, 0),
    "full": SceneSpec("full", 256, 256, 64, 16, 64.0, 10.0, 24, 0.05, 1, 1),
    "batch": SceneSpec("batch", 256, 256, 64, 16, 64.0, 10.0, 24, 0.05, 1, 2),
    "learned": SceneSpec("learned", 256, 256, 64, 16, 64.0, 10.0, 24, 0.05, 1, 3),
    "large": SceneSpec("large", 512, 512, 128, 32, 128.0, 5.0, 12, 0.05, 4, 4),
}


def seed_sequence(config_id: int, scene_id: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([2406, 13651, int(config_id), int(scene_id)])


def synth_pupil(ny: int, nx: int, radius: float) -> np.ndarray:
    """Circular pupil in signed DFT indices, built pixel by pixel."""
    out = np.zeros((ny, nx), dtype=bool)
    r2 = float(radius) * float(radius)
    for u in range(ny):
        su = u - ny if 2 * u >= ny else u
        for v in range(nx):
            sv = v - nx if 2 * v >= nx else v
            out[u, v] = su * su + sv * sv <= r2
    return out


def facet_scene(spec: SceneSpec, rng: np.random.Generator) -> np.ndarray:
    """Reflectivity r[nz, ny, nx] (float64) of a seeded faceted scene."""
    nx, ny, nz = spec.nx, spec.ny, spec.nz
    xs, ys = np.meshgrid(np.arange(nx, dtype=np.float64),
                         np.arange(ny, dtype=np.float64), indexing="xy")
    depth = np.full((ny, nx), np.inf)
    refl = np.zeros((ny, nx))
    tan_max = math.tan(math.radians(60.0))
    for _obj in range(spec.n_objects):
        m = spec.n_facets
        sx = rng.uniform(0, nx, m)
        sy = rng.uniform(0, ny, m)
        z0 = rng.uniform(0.2, 0.8, m) * nz
        tilt = rng.uniform(0.0, math.radians(60.0), m)
        azim = rng.uniform(0.0, 2 * math.pi, m)
        slope = 0.3 * (nz / nx) * np.tan(tilt) / tan_max
        gx = slope * np.cos(azim)
        gy = slope * np.sin(azim)
        cos_t = np.cos(tilt)
        d2 = (xs[None] - sx[:, None, None]) ** 2 + (ys[None] - sy[:, None, None]) ** 2
        f = np.argmin(d2, axis=0)
        z = z0[f] + gx[f] * (xs - sx[f]) + gy[f] * (ys - sy[f])
        if spec.n_objects > 1:
            # each object covers a seeded disk of the field of view
            cx, cy = rng.uniform(0.2, 0.8, 2) * (nx, ny)
            rad = rng.uniform(0.25, 0.45) * min(nx, ny)
            inside = (xs - cx) ** 2 + (ys - cy) ** 2 <= rad * rad
        else:
            inside = np.ones((ny, nx), dtype=bool)
        closer = inside & (z < depth)
        depth = np.where(closer, z, depth)
        refl = np.where(closer, cos_t[f], refl)
    r = np.full((nz, ny, nx), float(spec.r_min))
    hit = np.isfinite(depth)
    if refl[hit].size:
        refl = refl / refl[hit].max()
    zb = np.clip(np.rint(np.where(hit, depth, 0.0)), 0, nz - 1).astype(np.int64)
    yy, xx = np.nonzero(hit)
    r[zb[yy, xx], yy, xx] = np.maximum(refl[yy, xx], spec.r_min)
    return r


def noise_variance(r: np.ndarray, snr_db: float) -> float:
    """sigma_eta^2 = mean(r) 10^(-SNR/10): mean(r) is the expected per-sample
    power of F g under an orthonormal F (speckle variance r)."""
    return float(np.mean(r)) * 10.0 ** (-float(snr_db) / 10.0)


def synth_range_support(nz: int, k: int) -> np.ndarray:
    """Range frequencies that hold data after zero-padding in range: the k
    samples nearest DC (signed index -floor(k/2) .. ceil(k/2) - 1)."""
    w = np.arange(nz)
    sw = np.where(2 * w >= nz, w - nz, w)
    return (sw >= -(k // 2)) & (sw <= (k + 1) // 2 - 1)


def measure_looks(r: np.ndarray, looks: int, radius: float, sigma_eta2: float,
                  rngs, out: np.ndarray | None = None, workers: int = 1, range_support: int = 0) -> np.ndarray:
    """y[l] = D(a) F (sqrt(r) z_l) + eta_l as complex64 [looks, nz, ny, nx].

    range_support = 0: F is the orthonormal 2D DFT of each range slice and a
    the pupil.  range_support = k > 0: F is the orthonormal 3D DFT and a the
    pupil on the k range frequencies nearest DC (zero-padding in range, Sec.
    II-A).  Each look draws from its own stream, so `workers` threads give the
    same looks as one."""
    nz, ny, nx = r.shape
    pupil = synth_pupil(ny, nx, radius)
    if range_support > 0:
        pupil = synth_range_support(nz, range_support)[:, None, None] & pupil[None]
    if out is None:
        out = np.empty((looks, nz, ny, nx), dtype=np.complex64)
    amp = np.sqrt(r)
    s_noise = math.sqrt(sigma_eta2 / 2.0)

    def one(ell):
        rng = rngs[ell]
        z = (rng.standard_normal(r.shape) + 1j * rng.standard_normal(r.shape)) / math.sqrt(2.0)
        if range_support > 0:
            field = np.fft.fftn(amp * z, axes=(-3, -2, -1), norm="ortho")
        else:
            field = np.fft.fft2(amp * z, axes=(-2, -1), norm="ortho")
        field *= pupil
        field += s_noise * (rng.standard_normal(r.shape) + 1j * rng.standard_normal(r.shape))
        out[ell] = field.astype(np.complex64)

    if workers > 1 and looks > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(workers, looks)) as ex:
            list(ex.map(one, range(looks)))
    else:
        for ell in range(looks):
            one(ell)
    return out


def make_problem(spec: SceneSpec, scene_id: int = 0, workers: int = 1, range_support: int = 0):
    """Scene, looks and noise variance for one seeded workload (range_support:
    see measure_looks).

    Returns (r_true float64 [nz,ny,nx], y complex64 [L,nz,ny,nx], sigma_eta2).
    """
    ss = seed_sequence(spec.config_id, scene_id)
    children = ss.spawn(1 + spec.looks)
    r = facet_scene(spec, np.random.Generator(np.random.PCG64(children[0])))
    s2 = noise_variance(r, spec.snr_db)
    rngs = [np.random.Generator(np.random.PCG64(c)) for c in children[1:]]
    y = measure_looks(r, spec.looks, spec.radius, s2, rngs, workers=workers, range_support=range_support)
    return r, y, s2


def batch_specs(n_scenes=32, seed=0, cap_voxel_looks=2.5e9, sizes=(128, 192, 256, 384, 512),
                depths=(32, 64, 128), looks=(4, 32), snr_db=10.0):
    """Uneven scenes for batched runs: N ~ U(sizes), nz ~ U(depths),
    L ~ U{looks[0] .. looks[1]}, pupil radius N/4, 24 facets, background
    0.05.  Draws whose total exceeds `cap_voxel_looks` are redrawn (the
    uncapped recipe averages about 4.5e9 voxel-looks for 32 scenes)."""
    rng = np.random.Generator(np.random.PCG64(seed_sequence(2, 10_000 + seed)))
    for _attempt in range(100_000):
        specs = []
        total = 0
        for i in range(n_scenes):
            n = int(rng.choice(sizes))
            nz = int(rng.choice(depths))
            L = int(rng.integers(looks[0], looks[1] + 1))
            specs.append(SceneSpec("batch%d" % i, n, n, nz, L, n / 4.0, snr_db, 24, 0.05, 1, 2))
            total += n * n * nz * L
        if total <= cap_voxel_looks:
            return specs
    raise RuntimeError("no draw under the cap")
