"""Pins of the oracle's layout: partitions of unity, interpolation, sizes."""
import numpy as np
import pytest

from oracle.layout import AxisLayout, make_layout


@pytest.mark.parametrize("M,T,p,o,r,G", [(256, 2, 128, 16, 7, 2), (2048, 8, 256, 32, 15, 8),
                                          (8192, 16, 512, 64, 31, 16), (300, 3, 128, 10, 4, 5),
                                          (40, 2, 20, 4, 2, 3)])
def test_omega_partition_of_unity(M, T, p, o, r, G):
    ax = AxisLayout(M, T, p, o, r, G)
    tot = np.zeros(M + 2 * r)
    cnt = np.zeros(M + 2 * r, dtype=int)
    for a in range(T):
        s0, s1 = ax.support(a)
        w = ax.omega(a)
        assert w.shape == (s1 - s0,)
        assert np.all(w > 0) and np.all(w <= 1)
        tot[s0 + r:s1 + r] += w
        cnt[s0 + r:s1 + r] += 1
    assert np.allclose(tot, 1.0, atol=1e-15, rtol=0)
    assert cnt.min() >= 1 and cnt.max() <= 2


def test_omega_ramp_values():
    # Fig. 1: ramps between adjacent tiles over the overlap of the supports.
    ax = AxisLayout(40, 2, 20, 4, 2, 2)
    L = 4 + 2 * 2
    w0, w1 = ax.omega(0), ax.omega(1)
    assert np.allclose(w0[-L:], (L - np.arange(L) - 0.5) / L)
    assert np.allclose(w1[:L], (np.arange(L) + 0.5) / L)
    assert np.all(w0[:-L] == 1) and np.all(w1[L:] == 1)


@pytest.mark.parametrize("M,G", [(256, 2), (2048, 8), (300, 5), (64, 1)])
def test_tents_interpolate_linearly(M, G):
    ax = AxisLayout(M, 1, M, 0, 3, G)
    c = np.arange(-3, M + 3, dtype=float)
    W = np.stack([ax.tent(k, c) for k in range(G)])
    assert np.allclose(W.sum(0), 1.0, atol=1e-15)
    assert np.all(W >= 0)
    for k in range(G):
        assert ax.tent(k, [ax.node_centre(k)])[0] == 1.0
    # first-order interpolation reproduces linear functions between outer nodes
    inside = (c >= ax.node_centre(0)) & (c <= ax.node_centre(G - 1))
    centres = np.array([ax.node_centre(k) for k in range(G)])
    assert np.allclose((centres[:, None] * W).sum(0)[inside], c[inside], atol=1e-12)
    # at most two nodes overlap anywhere
    assert (W > 0).sum(0).max() <= 2


def test_workload_geometry():
    # 2048 px in 8 tiles of pitch 256, overlap 32, 31 x 31 PSFs
    ax = AxisLayout(2048, 8, 256, 32, 15, 8)
    assert [ax.block(a)[1] - ax.block(a)[0] for a in range(8)] == [288] * 7 + [256]
    assert [ax.support_len(a) for a in range(8)] == [318] * 7 + [286]
    assert [len(ax.tile_nodes(a)) for a in range(8)] == [2, 3, 3, 3, 3, 3, 3, 2]
    # 8192 px in 16 tiles: blocks of 512-576 px
    ax = AxisLayout(8192, 16, 512, 64, 31, 16)
    sizes = {ax.block(a)[1] - ax.block(a)[0] for a in range(16)}
    assert sizes == {512, 576}
    L = make_layout(2048, 8, 256, 32, 31, 8)
    counts = sorted({len(L.terms(t)) for t in range(L.n_tiles)})
    assert counts == [4, 6, 9]


def test_local_model_single_term():
    L = make_layout(40, 2, 20, 4, 5, 2, model="local")
    for t in range(L.n_tiles):
        terms = L.terms(t)
        assert len(terms) == 1 and terms[0][0] == t and np.all(terms[0][1] == 1)


def test_layout_rejects_bad_geometry():
    with pytest.raises(ValueError):
        AxisLayout(40, 2, 20, 20, 2, 2)     # overlap + 2r > pitch
    with pytest.raises(ValueError):
        AxisLayout(24, 2, 20, 4, 2, 2)      # last block inside the overlap
    with pytest.raises(ValueError):
        AxisLayout(10, 1, 10, 0, 5, 1)      # block smaller than the PSF
