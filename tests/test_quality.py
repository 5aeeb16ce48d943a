"""Pins of the image-quality measures (SNR, SSIM) used by the lambda sweep."""
import numpy as np

from paper_1705_06603_amd import quality


def _ssim_brute(x, ref, L, size=11, sigma=1.5):
    """SSIM from its definition, one window position at a time."""
    w = quality.gaussian_window(size, sigma)
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    vals = []
    for i in range(x.shape[0] - size + 1):
        for j in range(x.shape[1] - size + 1):
            a, b = x[i:i + size, j:j + size], ref[i:i + size, j:j + size]
            ma, mb = np.sum(w * a), np.sum(w * b)
            va, vb = np.sum(w * (a - ma) ** 2), np.sum(w * (b - mb) ** 2)
            cab = np.sum(w * (a - ma) * (b - mb))
            vals.append((2 * ma * mb + c1) * (2 * cab + c2) / ((ma ** 2 + mb ** 2 + c1) * (va + vb + c2)))
    return float(np.mean(vals))


def test_ssim_matches_its_definition():
    rng = np.random.default_rng(0)
    ref = rng.random((24, 20))
    x = ref + 0.1 * rng.standard_normal(ref.shape)
    L = ref.max() - ref.min()
    assert abs(quality.ssim(x, ref) - _ssim_brute(x, ref, L)) <= 1e-12


def test_ssim_of_identical_images_is_one_and_drops_with_noise():
    rng = np.random.default_rng(1)
    ref = rng.random((40, 40))
    assert abs(quality.ssim(ref, ref) - 1.0) <= 1e-12
    a = quality.ssim(ref + 0.05 * rng.standard_normal(ref.shape), ref)
    b = quality.ssim(ref + 0.2 * rng.standard_normal(ref.shape), ref)
    assert 1.0 > a > b


def test_snr_closed_form():
    ref = np.ones((10, 10))
    x = ref + 0.1                     # ||x - ref|| / ||ref|| = 0.1
    assert abs(quality.snr_db(x, ref) - 20.0) <= 1e-12
