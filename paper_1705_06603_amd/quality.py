"""Image-quality measures of Section IV-C, used to compare deblurred images
with the ground truth: the signal-to-noise ratio and the structural
similarity index (SSIM, Wang, Bovik, Sheikh and Simoncelli, 2004).

These are host-side evaluation helpers for reports; they are not part of the
solver.  SSIM follows the published definition with its standard constants:
an 11 x 11 circular-symmetric Gaussian window of standard deviation 1.5,
K1 = 0.01, K2 = 0.03 and L the dynamic range of the reference, evaluated
where the whole window lies inside the image and averaged (mean SSIM).
"""
from __future__ import annotations

import numpy as np


def snr_db(x, ref):
    """20 log10(||ref|| / ||x - ref||)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(20.0 * np.log10(np.linalg.norm(ref) / np.linalg.norm(x - ref)))


def gaussian_window(size=11, sigma=1.5):
    q = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-(q * q) / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def _local_mean(a, w):
    """Window-weighted local means where the window lies inside the image."""
    from scipy.signal import correlate2d
    return correlate2d(a, w, mode="valid")


def ssim(x, ref, data_range=None, size=11, sigma=1.5, k1=0.01, k2=0.03):
    """Mean structural similarity of x against ref."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    L = float(ref.max() - ref.min()) if data_range is None else float(data_range)
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    w = gaussian_window(size, sigma)
    mx, my = _local_mean(x, w), _local_mean(ref, w)
    sxx = _local_mean(x * x, w) - mx * mx
    syy = _local_mean(ref * ref, w) - my * my
    sxy = _local_mean(x * ref, w) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(np.mean(s))
