"""Seeded synthetic inputs for the tile solver: scenes, PSF grids and noise.

This module holds none of the deblurring method's arithmetic.  It only draws
the data the method is given: a ground-truth scene on the extended domain, a
grid of point-spread functions and the noise that turns a blurred image into
an observation.  The blur itself (the image-formation model, Eq. (2) of the
paper) is applied by whoever calls :func:`observe`: the CPU oracle in tests,
the HIP library in the benchmark.

The scenes stand in for the paper's natural test images (Section IV), which
are not used: point sources with heavy-tailed fluxes plus a few Gaussian
blobs on a constant background, the structure of a wide-field astronomical
frame.  PSFs follow Section IV's construction (a regular grid of normalised
PSFs whose width grows radially across the field): Gaussian for the small
case, elliptical Moffat profiles for the larger ones.

Every generator takes an explicit seed and uses ``numpy.random.Generator``
with ``PCG64``, so values are identical on every machine.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "star_field",
    "dead_leaves",
    "gaussian_psf_grid",
    "gaussian_psf_grid_radial",
    "moffat_psf_grid",
    "observe",
    "make_workload",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and solver settings of one synthetic deblurring workload.

    Attributes follow the paper's notation where it has one: ``lam`` is the
    regularisation weight lambda of Eq. (3), ``gamma`` scales the metric
    alpha_i = gamma * omega_i (Section III-B), ``rho`` is the D-R relaxation.
    """

    name: str
    M: int                # observed image is M x M
    tiles: int            # tiles per axis
    pitch: int            # tile pitch p
    overlap: int          # block overlap o
    grid: int             # PSF nodes per axis
    psf_size: int         # P = 2r+1
    psf_kind: str         # "gaussian" | "moffat"
    noise: str            # "gaussian" | "poisson"
    n_iter: int           # inner iterations (one iteration = one Local-Solver step on all tiles)
    n_inner: int = 10     # Local-Solver steps between consensus steps
    lam: float = 1e-3
    eps: float = 1e-3
    gamma: float = 0.4
    rho: float = 1.0
    seed: int = 1

    @property
    def r(self) -> int:
        return self.psf_size // 2

    @property
    def n_outer(self) -> int:
        return self.n_iter // self.n_inner


WORKLOADS = {
    # 256 x 256, 2 x 2 tiles, 16-px overlap, 2 x 2 Gaussian PSFs of 15 x 15.
    "small": Workload("small", M=256, tiles=2, pitch=128, overlap=16, grid=2,
                      psf_size=15, psf_kind="gaussian", noise="gaussian",
                      n_iter=50, seed=1),
    # 2048 x 2048, 8 x 8 tiles, 32-px overlap, 8 x 8 Moffat PSFs of 31 x 31.
    "batched": Workload("batched", M=2048, tiles=8, pitch=256, overlap=32, grid=8,
                        psf_size=31, psf_kind="moffat", noise="poisson",
                        n_iter=200, gamma=4.0, seed=2),
    # 8192 x 8192, 16 x 16 tiles (512-576 px), 64-px overlap, 63 x 63 Moffat PSFs.
    "large": Workload("large", M=8192, tiles=16, pitch=512, overlap=64, grid=16,
                      psf_size=63, psf_kind="moffat", noise="poisson",
                      n_iter=300, gamma=4.0, seed=3),
    # 16384 x 16384, 32 x 32 tiles, 64-px overlap, 63 x 63 Moffat PSFs.
    "combined": Workload("combined", M=16384, tiles=32, pitch=512, overlap=64, grid=32,
                         psf_size=63, psf_kind="moffat", noise="poisson",
                         n_iter=200, gamma=4.0, seed=5),
}


def star_field(shape, seed, *, stars_per_256sq=50.0, blobs_per_256sq=3.0,
               background=0.05, pareto_alpha=1.5, flux_min=1.0):
    """Ground-truth scene: background + point sources + Gaussian blobs.

    Star count ~ Poisson(stars_per_256sq * area/256^2) at uniform integer
    pixels with Pareto(alpha) fluxes (minimum ``flux_min``); blob count
    round(blobs_per_256sq * area/256^2) with amplitude U(0.1, 0.5) and width
    U(4, 16) px.  Returns a float64 array of ``shape``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = shape
    area = ny * nx / 65536.0
    img = np.full((ny, nx), background, dtype=np.float64)
    n_stars = rng.poisson(stars_per_256sq * area)
    ys = rng.integers(0, ny, size=n_stars)
    xs = rng.integers(0, nx, size=n_stars)
    flux = flux_min * (1.0 + rng.pareto(pareto_alpha, size=n_stars))
    np.add.at(img, (ys, xs), flux)
    n_blobs = max(1, int(round(blobs_per_256sq * area)))
    amp = rng.uniform(0.1, 0.5, size=n_blobs)
    sig = rng.uniform(4.0, 16.0, size=n_blobs)
    cy = rng.uniform(0, ny, size=n_blobs)
    cx = rng.uniform(0, nx, size=n_blobs)
    for a, s, y0, x0 in zip(amp, sig, cy, cx):
        # Evaluate each blob on a window of +-5 sigma only.
        h = int(math.ceil(5 * s))
        y_lo, y_hi = max(0, int(y0) - h), min(ny, int(y0) + h + 1)
        x_lo, x_hi = max(0, int(x0) - h), min(nx, int(x0) + h + 1)
        yy = np.arange(y_lo, y_hi)[:, None] - y0
        xx = np.arange(x_lo, x_hi)[None, :] - x0
        img[y_lo:y_hi, x_lo:x_hi] += a * np.exp(-(yy * yy + xx * xx) / (2 * s * s))
    return img


def dead_leaves(shape, seed, *, r_min=2.0, r_max=160.0, coverage=6.0, level_lo=0.05, level_hi=1.0):
    """Natural-image stand-in: the dead-leaves model (occluding opaque disks).

    Disk radii follow the scale-invariant density p(r) ~ r^-3 on
    [r_min, r_max] (inverse-CDF sampling), centres are uniform, grey levels
    uniform on [level_lo, level_hi]; disks are painted in draw order, later
    ones on top; their summed area is ``coverage`` times the area their
    centres are drawn from (the image grown by r_max on every side), and
    uncovered pixels keep level_lo.  Such images have the
    edge-and-flat-region structure and the power-law spectrum of natural
    photographs.  Returns a float64 array of ``shape``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = shape
    img = np.full((ny, nx), level_lo, dtype=np.float64)
    # mean disk area under p(r) ~ r^-3: pi r_min^2 r_max^2 ln(r_max/r_min) * 2 / (r_max^2 - r_min^2)
    a2, b2 = r_min * r_min, r_max * r_max
    mean_area = 2.0 * math.pi * a2 * b2 * math.log(r_max / r_min) / (b2 - a2)
    # centres fall on the image grown by r_max on every side
    n = int(math.ceil(coverage * (ny + 2 * r_max) * (nx + 2 * r_max) / mean_area))
    u = rng.random(n)
    # inverse CDF of p(r) ~ r^-3 on [a, b]: r = (1/a^2 - u (1/a^2 - 1/b^2))^(-1/2)
    rad = (1.0 / a2 - u * (1.0 / a2 - 1.0 / b2)) ** -0.5
    cy = rng.uniform(-r_max, ny + r_max, size=n)
    cx = rng.uniform(-r_max, nx + r_max, size=n)
    lev = rng.uniform(level_lo, level_hi, size=n)
    for r0, y0, x0, v in zip(rad, cy, cx, lev):
        y_lo, y_hi = max(0, int(math.floor(y0 - r0))), min(ny, int(math.ceil(y0 + r0)) + 1)
        x_lo, x_hi = max(0, int(math.floor(x0 - r0))), min(nx, int(math.ceil(x0 + r0)) + 1)
        if y_lo >= y_hi or x_lo >= x_hi:
            continue
        yy = np.arange(y_lo, y_hi)[:, None] - y0
        xx = np.arange(x_lo, x_hi)[None, :] - x0
        m = yy * yy + xx * xx <= r0 * r0
        img[y_lo:y_hi, x_lo:x_hi][m] = v
    return img


def _normalise(h):
    h = np.maximum(h, 0.0)
    return h / h.sum()


def gaussian_psf_grid(grid, size, sigma_lo=1.5, sigma_hi=3.0):
    """grid x grid isotropic Gaussian PSFs, size x size, unit sum.

    Node (a, b) has sigma = lo + (hi - lo) * (a + b) / (2 (grid - 1)), so the
    width runs from ``sigma_lo`` in one corner to ``sigma_hi`` in the other.
    Returns float64 [grid, grid, size, size].
    """
    r = size // 2
    q = np.arange(-r, r + 1, dtype=np.float64)
    yy, xx = np.meshgrid(q, q, indexing="ij")
    out = np.empty((grid, grid, size, size))
    for a in range(grid):
        for b in range(grid):
            t = 0.0 if grid == 1 else (a + b) / (2.0 * (grid - 1))
            s = sigma_lo + (sigma_hi - sigma_lo) * t
            out[a, b] = _normalise(np.exp(-(yy * yy + xx * xx) / (2 * s * s)))
    return out


def gaussian_psf_grid_radial(grid, size, fwhm_centre=3.5, fwhm_corner=(8.5, 6.5)):
    """grid x grid elliptical Gaussian PSFs, size x size, unit sum, in the
    manner of the smooth shift-variant experiments of Section IV: FWHM
    ``fwhm_centre`` at the field centre growing linearly with the node's
    normalised radius rho_n to ``fwhm_corner`` (major, minor) at the
    corners, major axis radial.  Returns float64 [grid, grid, size, size].
    """
    r = size // 2
    q = np.arange(-r, r + 1, dtype=np.float64)
    yy, xx = np.meshgrid(q, q, indexing="ij")
    c = (grid - 1) / 2.0
    rmax = max(math.hypot(c, c), 1e-12)
    f2s = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))   # FWHM -> sigma
    out = np.empty((grid, grid, size, size))
    for a in range(grid):
        for b in range(grid):
            dy, dx = a - c, b - c
            rho = math.hypot(dy, dx) / rmax if grid > 1 else 0.0
            s_major = (fwhm_centre + (fwhm_corner[0] - fwhm_centre) * rho) * f2s
            s_minor = (fwhm_centre + (fwhm_corner[1] - fwhm_centre) * rho) * f2s
            theta = math.atan2(dy, dx) if rho > 0 else 0.0
            ct, st = math.cos(theta), math.sin(theta)
            u = xx * ct + yy * st
            v = -xx * st + yy * ct
            out[a, b] = _normalise(np.exp(-0.5 * ((u / s_major) ** 2 + (v / s_minor) ** 2)))
    return out


def moffat_psf_grid(grid, size, beta=3.0, fwhm_lo=None, fwhm_hi=None, e_max=0.3,
                    rotate=False):
    """grid x grid elliptical Moffat PSFs, size x size, unit sum.

    With rho_n the node's distance from the field centre divided by the
    largest such distance: FWHM = lo + (hi - lo) rho_n (geometric mean of the
    two axes), ellipticity e = e_max rho_n with the major axis radial.  With
    ``rotate`` the major axis is the radial direction rotated by the node's
    polar angle again (a field-dependent rotation).  Defaults: FWHM 2 -> 6 px
    for size <= 31, 4 -> 12 px above.  Returns float64 [grid, grid, size, size].
    """
    if fwhm_lo is None:
        fwhm_lo, fwhm_hi = (2.0, 6.0) if size <= 31 else (4.0, 12.0)
    r = size // 2
    q = np.arange(-r, r + 1, dtype=np.float64)
    yy, xx = np.meshgrid(q, q, indexing="ij")
    c = (grid - 1) / 2.0
    rmax = max(math.hypot(c, c), 1e-12)
    out = np.empty((grid, grid, size, size))
    for a in range(grid):
        for b in range(grid):
            dy, dx = a - c, b - c
            rho = math.hypot(dy, dx) / rmax if grid > 1 else 0.0
            fwhm = fwhm_lo + (fwhm_hi - fwhm_lo) * rho
            e = e_max * rho
            theta = math.atan2(dy, dx) if rho > 0 else 0.0
            if rotate:
                theta = 2.0 * theta
            # Axis ratio from ellipticity e = 1 - b/a, geometric mean fixed.
            ratio = 1.0 - e
            fw_major = fwhm / math.sqrt(ratio)
            fw_minor = fwhm * math.sqrt(ratio)
            k = 1.0 / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
            al_major, al_minor = fw_major * k, fw_minor * k
            ct, st = math.cos(theta), math.sin(theta)
            u = xx * ct + yy * st
            v = -xx * st + yy * ct
            rr = (u / al_major) ** 2 + (v / al_minor) ** 2
            out[a, b] = _normalise((1.0 + rr) ** (-beta))
    return out


def observe(blurred, kind, seed, *, sigma=0.01, peak=1000.0, read_noise=5.0):
    """Add noise to a noiseless blurred image and give the weight map W.

    ``kind == "gaussian"``: y = blurred + N(0, sigma^2), W = 1 everywhere
    (uniform variance, so the unit-mean inverse variance is exactly one).

    ``kind == "poisson"``: the image is scaled so its maximum is ``peak``
    counts, Poisson-sampled, read noise N(0, read_noise^2) added, and the
    result divided by the same scale.  The variance model of Eq. (2) is
    sigma^2(l) = max(y_counts, 0) + read_noise^2; W = mean(sigma^2)/sigma^2,
    the inverse variance normalised to unit mean.

    Returns (y, W) as float64 arrays shaped like ``blurred``.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    if kind == "gaussian":
        y = blurred + sigma * rng.standard_normal(blurred.shape)
        return y, np.ones_like(blurred)
    if kind == "poisson":
        scale = peak / max(float(blurred.max()), 1e-30)
        counts = rng.poisson(np.maximum(blurred * scale, 0.0)).astype(np.float64)
        counts += read_noise * rng.standard_normal(blurred.shape)
        var = np.maximum(counts, 0.0) + read_noise * read_noise
        W = var.mean() / var
        return counts / scale, W
    raise ValueError(f"unknown noise kind {kind!r}")


def make_workload(w: Workload):
    """Scene on the extended domain (M + 2r)^2 and the PSF grid of ``w``."""
    n = w.M + 2 * w.r
    scene = star_field((n, n), w.seed)
    if w.psf_kind == "gaussian":
        psfs = gaussian_psf_grid(w.grid, w.psf_size)
    else:
        psfs = moffat_psf_grid(w.grid, w.psf_size, rotate=(w.psf_size > 31))
    return scene, psfs
