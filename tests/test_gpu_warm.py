"""Warm start on the GPU (network input transform, network start, per-tile
fallback judge) against the warm-start oracle, and a warm-started solve
against the oracle run from the same start."""
import numpy as np
import pytest

from oracle import cnn, solver, warm
from oracle import operator as op
from oracle.layout import make_layout
from oracle.solver import Problem

from tests._problems import sharpening_network

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _gauss_psfs(G, P, sigma):
    r = P // 2
    q = np.arange(-r, r + 1)
    yy, xx = np.meshgrid(q, q, indexing="ij")
    h = np.exp(-(yy ** 2 + xx ** 2) / (2 * sigma ** 2))
    return np.broadcast_to(h / h.sum(), (G, G, P, P)).copy()


def star_quadrant_problem(seed=0):
    """120 x 120, 2 x 2 tiles, narrow Gaussian PSFs; point sources only in
    the top-left and bottom-right tiles, a flat background elsewhere."""
    L = make_layout(120, 2, 60, 8, 7, 2)
    rng = np.random.default_rng(seed)
    psfs = _gauss_psfs(2, 7, 0.7)
    xg = np.full(L.X_shape, 0.5)
    for lo, hi in ((8, 58), (72, 118)):
        for _ in range(25):
            i, j = rng.integers(lo, hi, size=2)
            xg[i, j] += 5 + 10 * rng.random()
    y = op.apply_H_global(L, psfs, xg) + 0.002 * rng.standard_normal((120, 120))
    W = 0.5 + rng.random((120, 120))
    return Problem(L, _f32(psfs), _f32(y), _f32(W), lam=0.01, reg_param=0.05, gamma=0.7)


def test_warm_inputs_match_oracle():
    from tests._gpu import context_of
    prob = star_quadrant_problem()
    ctx = context_of(prob)
    frames, scales = ctx.warm_inputs()
    frames = frames.cpu().numpy()
    ins, s_ref = warm.tile_inputs(prob)
    assert np.max(np.abs(np.asarray(scales) - s_ref) / np.asarray(s_ref)) <= 1e-6
    for t, d in enumerate(ctx.tiles):
        f = frames[t]
        sh, sw = d.support_h, d.support_w
        assert np.max(np.abs(f[:sh, :sw] - ins[t])) <= 1e-6 * np.max(np.abs(ins[t]))
        assert not f[sh:, :].any() and not f[:, sw:].any()
    ctx.close()


def test_warm_start_judge_mixes_keep_and_fallback_as_the_oracle():
    """A network that sharpens point sources: its start is kept on the two
    star tiles and falls back on the two flat ones, as the oracle decides;
    kept starts match the oracle's network start (the network is exact in
    bf16, so to fp32 rounding), fallen-back ones the plain start bit for
    bit; then three D-R rounds match the oracle run from its own warm
    start."""
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of, rel_l2
    prob = star_quadrant_problem()
    params = sharpening_network()
    ref_starts, ref_keep, maps = warm.warm_start(prob, params, bf16=True)
    assert any(ref_keep) and not all(ref_keep), ref_keep
    for a, b in maps:
        assert abs(a / b - (1 - warm.MARGIN)) > 0.01      # no decision within fp32 noise of the threshold
    ctx = context_of(prob)
    N = ctx.tiles[0].frame
    net = dl.Net(ctx.n_tiles, N, N, params=cnn.flatten(params).astype(np.float32))
    use, nf = ctx.init_cnn(net)
    assert [bool(k) for k in use] == ref_keep
    assert nf == ref_keep.count(False)
    x0, u0 = ctx.get_state()
    x0 = x0.cpu().numpy()
    assert np.array_equal(x0, u0.cpu().numpy())               # u0 = x0
    x0_tiles = ctx.unpack_support(x0)
    plain = solver.initial_tiles(prob, "observed")
    for t in range(ctx.n_tiles):
        if ref_keep[t]:
            assert rel_l2(x0_tiles[t], ref_starts[t]) <= 1e-5, (t, rel_l2(x0_tiles[t], ref_starts[t]))
        else:
            assert np.array_equal(x0_tiles[t], _f32(plain[t])), t
    # the warm-started solve against the oracle run from its own warm start
    res = ctx.run(3, 5)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, 3, 5, x0=ref_starts)
    err = rel_l2(xh, ref.x_hat)
    print(f"warm-started solve: rel L2 {err:.3e}; kept {int(use.sum())}/{len(use)}")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
    net.close()
    ctx.close()
