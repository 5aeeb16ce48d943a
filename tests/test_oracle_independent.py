"""Pin of the oracle's independent baseline (the paper's 'independent'
method of Section IV: each block deblurred on its own, the blocks blended
with omega): without the consensus step each tile runs the proximal-point
method on its own f_t, so its limit is the minimiser of the tile's own
problem."""
import numpy as np

from oracle import minimiser, solver
from oracle.layout import make_layout
from oracle.solver import Problem
from tests._problems import tiny_problem


def test_independent_limit_is_each_tiles_own_minimiser():
    # one PSF node: the interpolation weight is 1 everywhere, so a tile's
    # operator is the plain valid convolution of its support, the operator
    # of a one-tile problem on the tile's block
    P = tiny_problem(M=16, T=2, p=8, o=2, P=3, G=1, seed=11, lam=0.05, reg_param=0.5, gamma=1.0)
    P.y = P.y - 0.4                                   # positivity active
    res = solver.solve(P, n_outer=1500, n_inner=10, consensus=False)
    L = P.layout
    for t in range(L.n_tiles):
        (y0, y1), (x0, x1) = L.block(t)
        Lt = make_layout(y1 - y0, 1, y1 - y0, 0, 3, 1, M_x=x1 - x0, T_x=1, G_x=1)
        Pt = Problem(Lt, P.psfs, P.y[y0:y1, x0:x1], P.W[y0:y1, x0:x1], lam=P.lam, reg=P.reg,
                     reg_param=P.reg_param, gamma=P.gamma, positivity=P.positivity, bc=P.bc)
        xstar, kkt = minimiser.minimise(Pt, tol=1e-14)
        assert kkt < 1e-11
        xt = res.x[t]
        assert np.max(np.abs(xt - Lt.restrict(xstar, 0))) <= 1e-8 * np.max(np.abs(xstar))
    # and the output blends the tiles with omega
    assert np.allclose(res.x_hat, solver.assemble(P, res.x), rtol=0, atol=0)


def test_independent_differs_from_consensus():
    P = tiny_problem(M=16, T=2, p=8, o=2, P=3, G=2, seed=12)
    a = solver.solve(P, 30, 5).x_hat
    b = solver.solve(P, 30, 5, consensus=False).x_hat
    assert np.max(np.abs(a - b)) > 1e-3
