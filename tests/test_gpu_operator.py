"""H_t and H_t^T of the HIP library against the FP64 direct-convolution oracle."""
import numpy as np
import pytest

from oracle import operator as op
from oracle.layout import make_layout
from oracle.solver import Problem
from tests._problems import random_psfs

pytestmark = pytest.mark.gpu

CASES = [
    # (M, T, p, o, P, G, model, extra)
    (40, 2, 20, 4, 5, 2, "interp", {}),
    (40, 2, 20, 4, 5, 3, "interp", {}),
    (45, 3, 14, 3, 5, 3, "interp", dict(M_x=38, T_x=2, G_x=2)),   # ragged, non-square
    (40, 2, 20, 4, 5, 2, "local", {}),
    (256, 2, 128, 16, 15, 2, "interp", {}),                          # small workload geometry
    (300, 3, 110, 10, 9, 3, "interp", dict(M_x=290, T_x=3, G_x=2)),  # uneven edge tiles, N = 160
    (600, 2, 300, 20, 21, 2, "interp", {}),                          # N = 640
    (37, 1, 37, 0, 5, 1, "interp", {}),                              # one tile, one PSF
    (50, 1, 50, 0, 7, 3, "interp", {}),                              # one tile, 3 x 3 nodes
    (40, 2, 20, 4, 1, 2, "interp", {}),                              # P = 1: no blur
    (24, 3, 8, 0, 3, 3, "local", {}),                                # zero overlap, 8-px blocks
]


def _problem(M, T, p, o, P, G, model, extra, seed):
    L = make_layout(M, T, p, o, P, G, model=model, **extra)
    psfs = random_psfs(L.ay.G, L.ax.G, P, seed)
    My, Mx = L.ay.M, L.ax.M
    return Problem(L, psfs, np.zeros((My, Mx)), np.ones((My, Mx)))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-P{c[4]}-G{c[5]}-{c[6]}")
def test_apply_H_and_Ht_match_oracle(case):
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _problem(*case, seed=case[0] + case[4])
    ctx = context_of(prob, observe=False)
    L = prob.layout
    rng = np.random.default_rng(1)
    xs = [rng.standard_normal(L.support_shape(t)) for t in range(L.n_tiles)]
    ss = [rng.standard_normal(L.block_shape(t)) for t in range(L.n_tiles)]
    hx = ctx.unpack_block(ctx.apply_H(to_dev(ctx.pack_list_support(xs))).cpu().numpy())
    hts = ctx.unpack_support(ctx.apply_Ht(to_dev(ctx.pack_list_block(ss))).cpu().numpy())
    for t in range(L.n_tiles):
        xf = np.asarray(xs[t], dtype=np.float32).astype(np.float64)
        sf = np.asarray(ss[t], dtype=np.float32).astype(np.float64)
        e1 = rel_l2(hx[t], op.apply_H(L, prob.psfs.astype(np.float32).astype(np.float64), t, xf))
        e2 = rel_l2(hts[t], op.apply_Ht(L, prob.psfs.astype(np.float32).astype(np.float64), t, sf))
        assert e1 <= 1e-5, (t, e1)
        assert e2 <= 1e-5, (t, e2)
    ctx.close()


def test_gpu_adjoint_identity():
    from tests._gpu import context_of, to_dev
    prob = _problem(256, 2, 128, 16, 15, 2, "interp", {}, seed=3)
    ctx = context_of(prob, observe=False)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(ctx.support_total).astype(np.float32)
    s = rng.standard_normal(ctx.block_total).astype(np.float32)
    hx = ctx.apply_H(to_dev(x)).cpu().numpy().astype(np.float64)
    hts = ctx.apply_Ht(to_dev(s)).cpu().numpy().astype(np.float64)
    lhs, rhs = np.dot(hx, s), np.dot(x, hts)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(hx) * np.linalg.norm(s)
    ctx.close()


def test_blur_global_matches_oracle():
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _problem(300, 3, 110, 10, 9, 3, "interp", dict(M_x=290, T_x=3, G_x=2), seed=5)
    ctx = context_of(prob, observe=False)
    xg = np.random.default_rng(4).random(prob.layout.X_shape)
    y = ctx.blur_global(to_dev(xg)).cpu().numpy()
    ref = op.apply_H_global(prob.layout, prob.psfs.astype(np.float32).astype(np.float64),
                            xg.astype(np.float32).astype(np.float64))
    assert rel_l2(y, ref) <= 1e-5
    ctx.close()


def test_rejects_more_than_three_nodes_per_tile_axis():
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import params_of
    prob = _problem(300, 3, 110, 10, 9, 4, "interp", {}, seed=6)
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(params_of(prob), prob.psfs)
    assert e.value.code == -2 and "3 PSF nodes" in str(e.value)
