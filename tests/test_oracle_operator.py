"""Pins of the oracle's blur operator H_t / H_t^T (direct convolution)."""
import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import operator as op
from oracle.layout import make_layout
from oracle.minimiser import dense_matrix
from tests._problems import random_psfs

LAYOUTS = [
    dict(M=40, T=2, p=20, o=4, P=5, G=2),
    dict(M=40, T=2, p=20, o=4, P=5, G=3),
    dict(M=45, T=3, p=14, o=3, P=5, G=3, M_x=38, T_x=2, G_x=2),   # ragged, non-square
]


@pytest.mark.parametrize("kw", LAYOUTS)
@pytest.mark.parametrize("model", ["interp", "local"])
def test_adjoint_identity(kw, model):
    if model == "local" and kw.get("G") != kw.get("T"):
        kw = dict(kw, G=kw["T"], G_x=kw.get("T_x"))
    L = make_layout(**kw, model=model)
    psfs = random_psfs(L.ay.G, L.ax.G, kw["P"], 3, positive=False)
    rng = np.random.default_rng(1)
    for t in range(L.n_tiles):
        x = rng.standard_normal(L.support_shape(t))
        s = rng.standard_normal(L.block_shape(t))
        lhs = np.vdot(op.apply_H(L, psfs, t, x), s)
        rhs = np.vdot(x, op.apply_Ht(L, psfs, t, s))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("model", ["interp", "local"])
def test_identical_psfs_is_plain_convolution(model):
    # With one PSF everywhere the tents sum to one, so both models reduce to
    # the 'valid' convolution of the support with h.
    L = make_layout(40, 2, 20, 4, 5, 2, model=model)
    h = random_psfs(1, 1, 5, 7)[0, 0]
    psfs = np.broadcast_to(h, (2, 2, 5, 5)).copy()
    rng = np.random.default_rng(2)
    for t in range(L.n_tiles):
        x = rng.standard_normal(L.support_shape(t))
        ref = convolve2d(x, h, mode="valid")
        got = op.apply_H(L, psfs, t, x)
        assert np.max(np.abs(got - ref)) <= 1e-13


def test_delta_psf_crops_and_pads():
    L = make_layout(40, 2, 20, 4, 5, 3)
    psfs = np.zeros((3, 3, 5, 5))
    psfs[:, :, 2, 2] = 1.0
    rng = np.random.default_rng(3)
    for t in range(L.n_tiles):
        x = rng.standard_normal(L.support_shape(t))
        assert np.allclose(op.apply_H(L, psfs, t, x), x[2:-2, 2:-2], atol=1e-14, rtol=0)
        s = rng.standard_normal(L.block_shape(t))
        pad = np.zeros(L.support_shape(t))
        pad[2:-2, 2:-2] = s
        assert np.allclose(op.apply_Ht(L, psfs, t, s), pad, atol=1e-14, rtol=0)


def test_shifted_delta_moves_image():
    # h(q) = delta at q = (1, -2): (H x)(j) = x(j - q)  (true convolution, not correlation)
    L = make_layout(40, 2, 20, 4, 5, 2)
    psfs = np.zeros((2, 2, 5, 5))
    psfs[:, :, 2 + 1, 2 - 2] = 1.0
    x = np.random.default_rng(4).standard_normal(L.support_shape(0))
    got = op.apply_H(L, psfs, 0, x)
    by, bx = L.block_shape(0)
    jy, jx = np.arange(by)[:, None] + 2, np.arange(bx)[None, :] + 2
    assert np.allclose(got, x[jy - 1, jx + 2], atol=1e-15, rtol=0)


def test_dense_matrix_properties():
    L = make_layout(12, 2, 6, 2, 3, 2)
    psfs = random_psfs(2, 2, 3, 5)
    for t in range(L.n_tiles):
        H = dense_matrix(lambda z: op.apply_H(L, psfs, t, z), L.support_shape(t))
        Ht = dense_matrix(lambda z: op.apply_Ht(L, psfs, t, z), L.block_shape(t))
        assert np.max(np.abs(Ht - H.T)) <= 1e-14
        assert H.sum(0).max() <= 1 + 1e-14          # column sums <= 1
        ones = np.ones(L.support_shape(t))
        assert np.allclose(H.sum(1), op.apply_H(L, psfs, t, ones).ravel(), atol=1e-14)
        assert np.all(H >= 0)


def _global_by_definition(L, psfs, xg):
    """sum over all nodes of convolve2d(w_k * x, h_k, 'valid') on the whole of X."""
    r = L.r
    cy = np.arange(L.X_shape[0]) - r
    cx = np.arange(L.X_shape[1]) - r
    out = np.zeros((L.ay.M, L.ax.M))
    for ky in range(L.ay.G):
        for kx in range(L.ax.G):
            w = np.outer(L.ay.tent(ky, cy), L.ax.tent(kx, cx))
            out += convolve2d(w * xg, psfs[ky, kx], mode="valid")
    return out


@pytest.mark.parametrize("kw", LAYOUTS)
def test_tile_operator_is_restriction_of_global(kw):
    L = make_layout(**kw)
    psfs = random_psfs(L.ay.G, L.ax.G, kw["P"], 11)
    xg = np.random.default_rng(5).standard_normal(L.X_shape)
    yg = _global_by_definition(L, psfs, xg)
    assert np.max(np.abs(op.apply_H_global(L, psfs, xg) - yg)) <= 1e-13
    for t in range(L.n_tiles):
        got = op.apply_H(L, psfs, t, L.restrict(xg, t))
        assert np.max(np.abs(got - L.block_of(yg, t))) <= 1e-13


@pytest.mark.parametrize("model", ["interp", "local"])
@pytest.mark.parametrize("extra", [0, 3, 9])
def test_fft_backend_matches_direct(model, extra):
    L = make_layout(40, 2, 20, 4, 5, 2, model=model)
    psfs = random_psfs(2, 2, 5, 13)
    N = max(max(L.support_shape(t)) for t in range(L.n_tiles)) + extra
    F = op.FFTOperator(L, psfs, N=N)
    rng = np.random.default_rng(6)
    for t in range(L.n_tiles):
        x = rng.standard_normal(L.support_shape(t))
        s = rng.standard_normal(L.block_shape(t))
        a, b = F.apply_H(t, x), op.apply_H(L, psfs, t, x)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
        a, b = F.apply_Ht(t, s), op.apply_Ht(L, psfs, t, s)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
