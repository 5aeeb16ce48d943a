"""The seeded input generators: reproducibility and the properties their
docstrings state (these hold none of the method's arithmetic)."""
import math

import numpy as np

from paper_1705_06603_amd import workloads


def test_dead_leaves_is_seeded_and_in_range():
    a = workloads.dead_leaves((96, 80), 3, r_max=30.0)
    b = workloads.dead_leaves((96, 80), 3, r_max=30.0)
    c = workloads.dead_leaves((96, 80), 4, r_max=30.0)
    assert a.shape == (96, 80) and np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.05 and a.max() <= 1.0
    # opaque disks: the image is piecewise constant with many distinct levels
    assert len(np.unique(a)) > 20
    # six-fold area coverage leaves few background pixels
    assert np.mean(a == 0.05) < 0.05


def test_dead_leaves_spectrum_falls_like_a_power_law():
    """Occluding disks with p(r) ~ r^-3 give a radially averaged power
    spectrum ~ f^-s with s near 2 (natural images: 1.6 .. 2.4)."""
    img = workloads.dead_leaves((512, 512), 11)
    F = np.abs(np.fft.fft2(img - img.mean())) ** 2
    fy = np.fft.fftfreq(512)[:, None]
    fx = np.fft.fftfreq(512)[None, :]
    f = np.hypot(fy, fx)
    bands = np.geomspace(0.01, 0.2, 9)
    p = [F[(f >= lo) & (f < hi)].mean() for lo, hi in zip(bands[:-1], bands[1:])]
    mid = np.sqrt(bands[:-1] * bands[1:])
    slope = np.polyfit(np.log(mid), np.log(p), 1)[0]
    assert -2.8 < slope < -1.4, slope


def _fwhm_along(h, direction):
    """Full width at half maximum of a centred PSF along a unit direction,
    by linear interpolation of the profile sampled at 0.01 px."""
    r = h.shape[0] // 2
    t = np.arange(-r, r + 1e-9, 0.01)
    ys, xs = r + t * direction[0], r + t * direction[1]
    y0, x0 = np.floor(ys).astype(int), np.floor(xs).astype(int)
    y0, x0 = np.clip(y0, 0, 2 * r - 1), np.clip(x0, 0, 2 * r - 1)
    wy, wx = ys - y0, xs - x0
    v = ((1 - wy) * (1 - wx) * h[y0, x0] + wy * (1 - wx) * h[y0 + 1, x0] + (1 - wy) * wx * h[y0, x0 + 1]
         + wy * wx * h[y0 + 1, x0 + 1])
    above = t[v >= 0.5 * h[r, r]]
    return above.max() - above.min()


def test_radial_gaussian_grid_widths():
    """Unit sums; the FWHM runs from 3.5 px at the centre to 8.5 (radial) x
    6.5 (tangential) px at the corners.  An odd grid has a node at the
    field centre."""
    g = workloads.gaussian_psf_grid_radial(5, 41)
    assert np.allclose(g.sum(axis=(2, 3)), 1.0)
    assert (g >= 0).all()
    c = g[2, 2]
    for d in ((0.0, 1.0), (1.0, 0.0)):
        assert abs(_fwhm_along(c, d) - 3.5) < 0.1
    k = g[4, 4]   # corner: radial direction is the diagonal
    rad = (1 / math.sqrt(2), 1 / math.sqrt(2))
    tan = (1 / math.sqrt(2), -1 / math.sqrt(2))
    # sampling a continuous Gaussian at pixel centres then interpolating
    # bilinearly widens the measured profile slightly
    assert abs(_fwhm_along(k, rad) - 8.5) < 0.2
    assert abs(_fwhm_along(k, tan) - 6.5) < 0.2
