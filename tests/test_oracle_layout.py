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


def test_grid_layout_blocks_and_weights():
    """Section III-C: blocks spanning three grid points, half-block overlaps
    (every observed pixel in two blocks per axis, one before the first and
    after the last node); consensus weights positive, a partition of unity
    over the covering supports, linear where exactly two supports cover."""
    from oracle.layout import AxisLayout
    for M, G, r in ((256, 4, 7), (300, 5, 15), (97, 3, 2)):
        A = AxisLayout(M, G, 0, 0, r, G, "grid")
        q = M / G
        count = np.zeros(M, dtype=int)
        for a in range(G):
            s, e = A.block(a)
            count[s:e] += 1
            lo = A.node_centre(a - 1) if a > 0 else -1.0
            hi = A.node_centre(a + 1) if a < G - 1 else M
            assert s == int(np.floor(lo)) + 1 and e == int(np.ceil(hi)) or (a == 0 and s == 0) or a == G - 1
        c0, cl = A.node_centre(0), A.node_centre(G - 1)
        i = np.arange(M)
        at_node = np.isin(i, [A.node_centre(k) for k in range(G)])   # a pixel on a node: its block only
        assert np.all(count[(i > c0) & (i < cl) & ~at_node] == 2)
        assert np.all(count[at_node] == 1)
        assert np.all(count[(i < c0) | (i > cl)] == 1)
        tot = np.zeros(M + 2 * r)
        cov = np.zeros(M + 2 * r, dtype=int)
        for a in range(G):
            s0, s1 = A.support(a)
            w = A.omega(a)
            assert np.all(w > 0)
            tot[s0 + r:s1 + r] += w
            cov[s0 + r:s1 + r] += 1
        assert np.allclose(tot, 1.0, rtol=0, atol=1e-14)
        assert cov.max() <= 3
        for a in range(G - 1):   # between nodes a and a+1, away from the triple zones: linear
            s0, _ = A.support(a)
            w = A.omega(a)
            lo = int(np.ceil(A.node_centre(a) + r)) + 1
            hi = int(np.floor(A.node_centre(a + 1) - r)) - 1
            seg = w[lo - s0:hi - s0]
            if len(seg) > 3:
                assert np.allclose(np.diff(seg, 2), 0.0, atol=1e-13)
    with pytest.raises(ValueError):
        AxisLayout(100, 4, 0, 0, 20, 4, "grid")          # 2r > q
    with pytest.raises(ValueError):
        AxisLayout(100, 3, 0, 0, 2, 4, "grid")           # T != G


def test_grid_layout_dr_limit_is_the_consensus_minimiser():
    """Algorithm 1 on the grid layout (one PSF per block, LOCAL operator)
    converges to the minimiser of its consensus problem, Eq. (4)."""
    from oracle import minimiser, solver
    from tests._problems import tiny_problem
    P = tiny_problem(M=18, T=3, p=0, o=0, P=3, G=3, seed=13, model="local", kind="grid", lam=0.05,
                     reg_param=0.5, gamma=1.0)
    P.y = P.y - 0.4
    res = solver.solve(P, n_outer=400, n_inner=10)
    xstar, kkt = minimiser.minimise(P, tol=1e-14)
    assert kkt < 1e-11 and (xstar == 0).any()
    assert np.max(np.abs(res.x_hat - xstar)) <= 1e-7 * np.max(np.abs(xstar))

