"""The grid layout of Section III-C (one block per PSF node spanning three
grid points, half-block overlaps, each block's own PSF) on the GPU against
the oracle: layout, operator, the consensus gather over up to three tiles per
axis, and a full solve."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import solver
from oracle.layout import make_layout
from oracle.solver import Problem
from tests._problems import random_psfs

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def grid_problem(M=256, G=4, P=15, seed=0, gamma=0.7):
    """Observation by the interpolated global operator of the same PSF grid
    (the image formation of Section II-B), deblurred on the grid layout with
    each block's own PSF."""
    L = make_layout(M, G, 0, 0, P, G, model="local", kind="grid")
    rng = np.random.default_rng(seed)
    psfs = _f32(random_psfs(G, G, P, seed + 1))
    Lg = make_layout(M, 1, M, 0, P, G)           # the same PSF grid, one tile: the global operator
    xg = rng.random(Lg.X_shape) * 2
    y = op.apply_H_global(Lg, psfs, xg) + 0.02 * rng.standard_normal((M, M))
    W = 0.5 + rng.random((M, M))
    return Problem(L, psfs, _f32(y), _f32(W), lam=0.02, reg_param=0.05, gamma=gamma, rho=1.0)


def test_grid_layout_matches_oracle():
    from tests._gpu import context_of
    prob = grid_problem()
    L = prob.layout
    ctx = context_of(prob)
    assert ctx.n_tiles == 16
    for t, d in enumerate(ctx.tiles):
        (by0, by1), (bx0, bx1) = L.block(t)
        (sy0, sy1), (sx0, sx1) = L.support(t)
        assert (d.block_y0, d.block_x0, d.block_h, d.block_w) == (by0, bx0, by1 - by0, bx1 - bx0)
        assert (d.support_y0, d.support_x0, d.support_h, d.support_w) == (sy0, sx0, sy1 - sy0, sx1 - sx0)
        assert d.n_terms == 1
    ctx.close()


def test_grid_operator_matches_oracle():
    from tests._gpu import context_of, rel_l2, to_dev
    prob = grid_problem(seed=2)
    L = prob.layout
    ctx = context_of(prob, observe=False)
    rng = np.random.default_rng(3)
    xs = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    ss = [_f32(rng.standard_normal(L.block_shape(t))) for t in range(L.n_tiles)]
    hx = ctx.unpack_block(ctx.apply_H(to_dev(ctx.pack_list_support(xs))).cpu().numpy())
    hts = ctx.unpack_support(ctx.apply_Ht(to_dev(ctx.pack_list_block(ss))).cpu().numpy())
    for t in range(L.n_tiles):
        assert rel_l2(hx[t], op.apply_H(L, prob.psfs, t, xs[t])) <= 1e-5
        assert rel_l2(hts[t], op.apply_Ht(L, prob.psfs, t, ss[t])) <= 1e-5
    ctx.close()


def test_grid_consensus_over_three_tiles_matches_oracle():
    """Near a node, three supports per axis (nine tiles in 2-D) meet."""
    from tests._gpu import context_of, rel_l2, to_dev
    prob = grid_problem(seed=4)
    L = prob.layout
    ctx = context_of(prob)
    rng = np.random.default_rng(5)
    x0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    u0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
    res = ctx.consensus()
    ug = ctx.unpack_support(ctx.get_state()[1].cpu().numpy())
    u_ref, _ = solver.consensus_step(prob, x0, u0)
    for t in range(L.n_tiles):
        assert rel_l2(ug[t], u_ref[t]) <= 1e-6
    assert abs(res - solver.residual(u0, u_ref)) <= 1e-5 * solver.residual(u0, u_ref)
    assert rel_l2(ctx.assemble().cpu().numpy(), solver.assemble(prob, x0)) <= 1e-6
    ctx.close()


def test_grid_solve_matches_oracle():
    """5 D-R rounds of 10 Local-Solver steps on the grid layout: final image
    <= 1e-4, residual history to 1e-3."""
    from tests._gpu import context_of, rel_l2
    prob = grid_problem(seed=6)
    ctx = context_of(prob)
    ctx.init()
    res = ctx.run(5, 10)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, 5, 10)
    err = rel_l2(xh, ref.x_hat)
    print(f"grid layout, 16 tiles, 50 iterations: rel L2 {err:.2e}")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
    ctx.close()


def test_grid_layout_errors():
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import params_of
    prob = grid_problem()
    p = params_of(prob)
    p.model = dl.MODEL_INTERP
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(p, prob.psfs)
    assert e.value.code == -2
    p = params_of(prob)
    p.P = 67                                   # 2r = 66 > the node spacing M / G = 64
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(p, np.broadcast_to(np.full((67, 67), 1.0 / 67 ** 2), (4, 4, 67, 67)).copy())
    assert e.value.code == -2
    import torch
    ctx = dl.Context(params_of(prob), prob.psfs)
    with pytest.raises(dl.DeblurError) as e:
        ctx.blur_global(torch.zeros(ctx.X_shape, dtype=torch.float32, device="cuda"))
    assert e.value.code == -5
    ctx.close()
