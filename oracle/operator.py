"""Shift-variant blur operator by direct spatial convolution (FP64).

Section II-B writes the shift-variant blur as a sum of local shift-invariant
blurs of weighted copies of the image, sum_k Z_k H_k W_k C_k x, with W_k the
first-order interpolation weights and H_k the convolution by PSF h_k; the
per-node operator is a circular convolution followed by a chop to the valid
region, H_i = C_i calH_i.  Restricted to tile t this is, for an observed
pixel j of the block B_t,

    (H_t x)(j) = sum_k sum_{q in [-r, r]^2} h_k(q) w_k(j - q) x(j - q),

a true (flipped) convolution evaluated only where the whole PSF footprint
lies inside the support.  The adjoint is its exact transpose,

    (H_t^T s)(i) = sum_k w_k(i) sum_q h_k(q) s(i + q),   i + q in B_t.

PSF arrays are indexed h[q + r] for q in [-r, r]^2.
"""
from __future__ import annotations

import numpy as np


def valid_conv(z, h):
    """Valid part of the convolution h * z by explicit shifted sums."""
    P = h.shape[0]
    r = P // 2
    ny, nx = z.shape[0] - 2 * r, z.shape[1] - 2 * r
    out = np.zeros((ny, nx))
    for qy in range(-r, r + 1):
        for qx in range(-r, r + 1):
            c = h[qy + r, qx + r]
            if c != 0.0:
                out += c * z[r - qy:r - qy + ny, r - qx:r - qx + nx]
    return out


def valid_conv_adjoint(s, h):
    """Transpose of :func:`valid_conv`: spreads the block s over the support."""
    P = h.shape[0]
    r = P // 2
    ny, nx = s.shape
    out = np.zeros((ny + 2 * r, nx + 2 * r))
    for qy in range(-r, r + 1):
        for qx in range(-r, r + 1):
            c = h[qy + r, qx + r]
            if c != 0.0:
                out[r - qy:r - qy + ny, r - qx:r - qx + nx] += c * s
    return out


def _psf(psfs, node):
    G_x = psfs.shape[1]
    return psfs[node // G_x, node % G_x]


def apply_H(layout, psfs, t, x):
    """H_t x: support of tile t -> its observed block."""
    out = None
    for node, w in layout.terms(t):
        term = valid_conv(w * x, _psf(psfs, node))
        out = term if out is None else out + term
    return out


def apply_Ht(layout, psfs, t, s):
    """H_t^T s: observed block of tile t -> its support."""
    out = None
    for node, w in layout.terms(t):
        term = w * valid_conv_adjoint(s, _psf(psfs, node))
        out = term if out is None else out + term
    return out


def apply_H_global(layout, psfs, x_global):
    """The global interpolated operator y = R sum_k Z_k H_k W_k C_k x (Eq. (2)).

    x_global is on X = [-r, M+r)^2; the result is on the observed [0, M)^2.
    Each node only contributes where its tent is non-zero, so its weighted
    image is convolved over that window only (zeros elsewhere add nothing).
    """
    ay, ax = layout.ay, layout.ax
    r = ay.r
    Xy, Xx = layout.X_shape
    cy = np.arange(Xy) - r          # observed coordinate of each X row
    cx = np.arange(Xx) - r
    y = np.zeros((ay.M, ax.M))
    for ky in range(ay.G):
        wy = ay.tent(ky, cy)
        iy = np.nonzero(wy > 0)[0]
        for kx in range(ax.G):
            wx = ax.tent(kx, cx)
            ix = np.nonzero(wx > 0)[0]
            y0, y1 = iy[0], iy[-1] + 1
            x0, x1 = ix[0], ix[-1] + 1
            ny, nx = y1 - y0, x1 - x0
            # Pad the weighted window by 2r so every output it reaches is valid.
            z = np.zeros((ny + 4 * r, nx + 4 * r))
            z[2 * r:2 * r + ny, 2 * r:2 * r + nx] = np.outer(wy[y0:y1], wx[x0:x1]) * x_global[y0:y1, x0:x1]
            contrib = valid_conv(z, psfs[ky, kx])
            # contrib[m] sits at observed coordinate (X index y0) - 2r + m.
            oy0, ox0 = y0 - 2 * r, x0 - 2 * r
            sy0, sx0 = max(oy0, 0), max(ox0, 0)
            sy1 = min(oy0 + contrib.shape[0], ay.M)
            sx1 = min(ox0 + contrib.shape[1], ax.M)
            if sy1 > sy0 and sx1 > sx0:
                y[sy0:sy1, sx0:sx1] += contrib[sy0 - oy0:sy1 - oy0, sx0 - ox0:sx1 - ox0]
    return y


# ---------------------------------------------------------------------------
# FP64 FFT backend: same operator through circular convolution on a frame of
# size >= the support (Section II-B, H_i = C_i calH_i).  Used only for full
# solves of the larger workloads, after matching the direct form.
# ---------------------------------------------------------------------------

def _frame_spectrum(h, N):
    P = h.shape[0]
    r = P // 2
    f = np.zeros((N, N))
    for qy in range(-r, r + 1):
        for qx in range(-r, r + 1):
            f[qy % N, qx % N] += h[qy + r, qx + r]
    return np.fft.rfft2(f)


class FFTOperator:
    """H_t and H_t^T of one layout through FP64 FFTs on N x N frames."""

    def __init__(self, layout, psfs, N=None):
        self.layout = layout
        self.psfs = psfs
        shapes = [layout.support_shape(t) for t in range(layout.n_tiles)]
        self.N = N or max(max(s) for s in shapes)
        if any(max(s) > self.N for s in shapes):
            raise ValueError("frame smaller than a support")
        self._spec = {}

    def _spectrum(self, node):
        if node not in self._spec:
            self._spec[node] = _frame_spectrum(_psf(self.psfs, node), self.N)
        return self._spec[node]

    def apply_H(self, t, x):
        N, r = self.N, self.layout.r
        sy, sx = x.shape
        acc = None
        for node, w in self.layout.terms(t):
            f = np.zeros((N, N))
            f[:sy, :sx] = w * x
            term = np.fft.rfft2(f) * self._spectrum(node)
            acc = term if acc is None else acc + term
        full = np.fft.irfft2(acc, s=(N, N))
        return full[r:sy - r, r:sx - r]

    def apply_Ht(self, t, s):
        N, r = self.N, self.layout.r
        by, bx = s.shape
        f = np.zeros((N, N))
        f[r:r + by, r:r + bx] = s
        S = np.fft.rfft2(f)
        out = None
        for node, w in self.layout.terms(t):
            full = np.fft.irfft2(S * np.conj(self._spectrum(node)), s=(N, N))
            term = w * full[:by + 2 * r, :bx + 2 * r]
            out = term if out is None else out + term
        return out


class DirectOperator:
    """Same interface as :class:`FFTOperator`, by direct convolution."""

    def __init__(self, layout, psfs):
        self.layout = layout
        self.psfs = psfs

    def apply_H(self, t, x):
        return apply_H(self.layout, self.psfs, t, x)

    def apply_Ht(self, t, s):
        return apply_Ht(self.layout, self.psfs, t, s)
