"""The oracle's FP64 FFT backend equals its direct-convolution operator on
the tile shapes of the batched workload (2048 x 2048, 8 x 8 tiles, 31 x 31
PSFs, 320 x 320 frames): corner, edge, interior and far-edge tiles, with 4,
6 and 9 PSF terms.  This licenses the FFT backend for the full-size
final-image parity runs."""
import numpy as np
import pytest

from oracle import operator as op
from oracle.layout import make_layout
from paper_1705_06603_amd import workloads


@pytest.mark.parametrize("t", [0, 1, 9, 7, 63])
def test_fft_backend_matches_direct_on_batched_tiles(t):
    w = workloads.WORKLOADS["batched"]
    psfs = workloads.moffat_psf_grid(w.grid, w.psf_size)
    L = make_layout(w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    F = op.FFTOperator(L, psfs, 320)
    rng = np.random.default_rng(40 + t)
    x = rng.random(L.support_shape(t))
    s = rng.standard_normal(L.block_shape(t))
    a, b = F.apply_H(t, x), op.apply_H(L, psfs, t, x)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    a, b = F.apply_Ht(t, s), op.apply_Ht(L, psfs, t, s)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
