"""The oracle against small worked examples derived by hand (tests/golden/)."""
import math
import os

import numpy as np

from oracle import prior
from oracle.layout import AxisLayout

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.setdefault(line[0], []).append([float(v) for v in line[1:]])
    return rows


def test_axis_layout_worked_example():
    g = _read("axis_layout_M40_T2_p20_o4_r2_G2.txt")
    A = AxisLayout(M=40, T=2, p=20, o=4, r=2, G=2)
    for a, s, e in g["block"]:
        assert A.block(int(a)) == (int(s), int(e))
    for a, s, e in g["support"]:
        assert A.support(int(a)) == (int(s), int(e))
    for row in g["omega"]:
        a, w = int(row[0]), np.array(row[1:])
        assert np.array_equal(A.omega(a), w)          # dyadic values: exact
    coords = np.array(g["coords"][0])
    for row in g["tent"]:
        k, w = int(row[0]), np.array(row[1:])
        assert np.allclose(A.tent(k, coords), w, rtol=0, atol=1e-15)


def test_grid_axis_layout_worked_example():
    g = _read("axis_grid_M12_G3_r1.txt")
    A = AxisLayout(M=12, T=3, p=0, o=0, r=1, G=3, kind="grid")
    for a, s, e in g["block"]:
        assert A.block(int(a)) == (int(s), int(e))
    for a, s, e in g["support"]:
        assert A.support(int(a)) == (int(s), int(e))
    for key, coord in (("omega6", 6), ("omega3", 3), ("omegam1", -1)):
        for a, w in g[key]:
            s0, _ = A.support(int(a))
            assert abs(A.omega(int(a))[coord - s0] - w) <= 1e-15, (key, a)


def test_smoothed_tv_worked_example():
    g = _read("smoothed_tv_2x2.txt")
    x = np.array(g["x"][0]).reshape(2, 2)
    eps = g["eps"][0][0]
    for bc in ("neumann", "circular"):
        pairs = np.array(g[bc + "_pairs"][0]).reshape(4, 2)
        by_hand = sum(math.sqrt(gh * gh + gv * gv + eps * eps) - eps for gh, gv in pairs)
        assert abs(by_hand - g[bc][0][0]) <= 1e-14
        assert abs(prior.value(x, "tv", eps, bc) - by_hand) <= 1e-13


def _layout(My, Mx, T, p, o, P, G):
    from oracle.layout import make_layout
    return make_layout(My, T, p, o, P, G, M_x=Mx)


def _problem_on(L, y, lam=0.0, gamma=1.0):
    from oracle.solver import Problem
    return Problem(L, np.ones((L.ay.G, L.ax.G, 2 * L.r + 1, 2 * L.r + 1)) / (2 * L.r + 1) ** 2, y,
                   np.ones_like(y), lam=lam, gamma=gamma, operator=object())


def test_initial_tiles_ragged_worked_example():
    from oracle import solver
    g = _read("initial_tiles_ragged_M9x10_T2_p4_o1_r1.txt")
    L = _layout(9, 10, 2, 4, 1, 3, 1)
    i, j = np.meshgrid(np.arange(9), np.arange(10), indexing="ij")
    prob = _problem_on(L, (10.0 * i + j - 20.0))
    x0 = solver.initial_tiles(prob, "observed")
    for t, h, w in g["shape"]:
        assert x0[int(t)].shape == (int(h), int(w))
    for t, m, c, v in g["x0"]:
        assert x0[int(t)][int(m), int(c)] == v, (t, m, c)
    # every tile starts from one common image on X
    r = L.r
    img = np.full(L.X_shape, np.nan)
    for t in range(L.n_tiles):
        (y0, y1), (xa, xb) = L.support(t)
        sl = img[y0 + r:y1 + r, xa + r:xb + r]
        seen = ~np.isnan(sl)
        assert np.array_equal(sl[seen], x0[t][seen])
        img[y0 + r:y1 + r, xa + r:xb + r] = x0[t]


def test_residual_worked_example():
    from oracle import solver
    g = _read("residual_2tiles.txt")
    u_old = [np.array(g["u_old0"][0]).reshape(2, 2), np.array(g["u_old1"][0]).reshape(1, 1)]
    u_new = [np.array(g["u_new0"][0]).reshape(2, 2), np.array(g["u_new1"][0]).reshape(1, 1)]
    assert abs(solver.residual(u_old, u_new) - g["residual"][0][0]) <= 1e-15
    assert solver.residual(u_new, u_new) == 0.0


def test_warm_inputs_worked_example():
    from oracle import warm
    g = _read("warm_inputs_M8_T2_p4_o0_r1.txt")
    L = _layout(8, 8, 2, 4, 0, 3, 1)
    i, j = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    prob = _problem_on(L, 10.0 * i + j - 20.0)
    ins, scales = warm.tile_inputs(prob)
    for t, s in g["scale"]:
        assert scales[int(t)] == s
    for t, m, c, v in g["input"]:
        assert abs(ins[int(t)][int(m), int(c)] - v) <= 1e-15 * abs(v), (t, m, c)
    prob_neg = _problem_on(L, -np.ones((8, 8)))
    ins, scales = warm.tile_inputs(prob_neg)
    assert all(s == g["floor_scale"][0][0] for s in scales)
    assert all(np.all(a == g["floor_input"][0][0]) for a in ins)


def test_gradient_map_worked_example():
    from oracle import solver, warm
    from oracle.solver import Problem
    g = _read("gradient_map_delta_psf.txt")
    L = _layout(3, 3, 1, 3, 0, 1, 1)
    y = np.array(g["y"][0]).reshape(3, 3)
    prob = Problem(L, np.ones((1, 1, 1, 1)), y, np.ones((3, 3)), lam=0.0, gamma=1.0)
    tau = solver.step_size(prob, 0)
    assert tau == g["tau"][0][0]
    plain = np.maximum(y, 0.0)
    zero, one = np.zeros((3, 3)), np.ones((3, 3))
    assert warm.gradient_map(prob, 0, plain, tau) == g["map_plain"][0][0]
    assert abs(warm.gradient_map(prob, 0, zero, tau) - g["map_zero"][0][0]) <= 1e-15
    assert abs(warm.gradient_map(prob, 0, one, tau) - g["map_one"][0][0]) <= 1e-15
    for key, net, pl in (("judge_zero_vs_plain", zero, plain), ("judge_plain_vs_zero", plain, zero),
                         ("judge_one_vs_zero", one, zero)):
        starts, keep, _ = warm.judge(prob, [net], [pl])
        assert keep == [bool(g[key][0][0])], key
        assert np.array_equal(starts[0], net if keep[0] else pl)


def test_adam_worked_example():
    from oracle import cnn
    g = _read("adam_3steps.txt")
    b1, b2, eps, lr, w0 = g["params"][0]
    w, m, v = np.array([w0]), np.zeros(1), np.zeros(1)
    for k, (gk, wk) in enumerate(zip(g["grads"][0], g["w"][0]), start=1):
        w, m, v = cnn.adam_step(w, np.array([gk]), m, v, k, lr, b1=b1, b2=b2, eps=eps)
        assert abs(w[0] - wk) <= 1e-15, (k, w[0], wk)
