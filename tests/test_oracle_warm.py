"""Pins of the warm-start oracle (tile transform and fallback judge) beyond
the worked examples in tests/golden/."""
import numpy as np

from oracle import cnn, minimiser, solver, warm
from tests._problems import tiny_problem


def _identity_net(seed=0):
    p = cnn.init_params(seed)
    p[3] = (np.zeros_like(p[3][0]), np.zeros_like(p[3][1]))
    return p


def test_identity_network_gives_the_plain_start_and_falls_back():
    """A network that returns its input gives max(0, s_t * y / s_t) = the
    plain start; the margin then makes every tile fall back."""
    prob = tiny_problem(M=16, T=2, p=8, o=2, P=3, G=2, seed=3)
    prob.y = prob.y - 0.4                       # some negative observations
    x_net = warm.network_start(prob, _identity_net(), bf16=False)
    x_plain = solver.initial_tiles(prob, "observed")
    for a, b in zip(x_net, x_plain):
        assert np.allclose(a, b, rtol=1e-15, atol=0)
    starts, keep, maps = warm.warm_start(prob, _identity_net(), bf16=False)
    assert not any(keep)
    for s, b in zip(starts, x_plain):
        assert np.array_equal(s, b)


def test_gradient_map_vanishes_only_at_the_tile_minimiser():
    """One tile: the consensus problem is the tile's own cost, whose
    projected-Newton minimiser is a zero of the gradient map; a perturbed
    point is not."""
    prob = tiny_problem(M=6, T=1, p=6, o=0, P=3, G=1, seed=5, lam=0.05, reg_param=0.5)
    prob.y = prob.y - 0.5                       # active positivity constraints
    xstar, kkt = minimiser.minimise(prob, tol=1e-13)
    tau = solver.step_size(prob, 0)
    assert np.any(xstar == 0.0)
    assert warm.gradient_map(prob, 0, xstar, tau) <= 1e-10
    rng = np.random.default_rng(0)
    moved = np.maximum(xstar + 0.05 * rng.standard_normal(xstar.shape), 0.0)
    assert warm.gradient_map(prob, 0, moved, tau) > 1e-3


def test_judge_prefers_the_start_closer_to_stationarity():
    """Of a tile's minimiser and its plain start, the judge keeps the
    minimiser (map 0), and never keeps a start whose map is larger."""
    prob = tiny_problem(M=6, T=1, p=6, o=0, P=3, G=1, seed=6, lam=0.05, reg_param=0.5)
    xstar, _ = minimiser.minimise(prob, tol=1e-13)
    plain = solver.initial_tiles(prob, "observed")
    starts, keep, maps = warm.judge(prob, [xstar], plain)
    assert keep == [True] and maps[0][0] < maps[0][1]
    starts, keep, maps = warm.judge(prob, plain, [xstar])
    assert keep == [False] and np.array_equal(starts[0], xstar)


def test_scale_invariance_of_the_transform():
    """The input is y / s_t, so scaling the observation by c > 0 leaves the
    network input unchanged and scales the start by c."""
    prob = tiny_problem(M=16, T=2, p=8, o=2, P=3, G=2, seed=4)
    rng = np.random.default_rng(1)
    p = cnn.init_params(2, scale_last=0.3)
    p = [(W, 0.05 * rng.standard_normal(b.shape)) for W, b in p]
    ins1, s1 = warm.tile_inputs(prob)
    x1 = warm.network_start(prob, p, bf16=False)
    prob.y = prob.y * 8.0
    ins2, s2 = warm.tile_inputs(prob)
    x2 = warm.network_start(prob, p, bf16=False)
    for t in range(prob.n_tiles):
        assert np.allclose(ins1[t], ins2[t], rtol=1e-14, atol=0)
        assert abs(s2[t] - 8.0 * s1[t]) <= 1e-14 * s2[t]
        assert np.allclose(x2[t], 8.0 * x1[t], rtol=1e-13, atol=1e-13)
