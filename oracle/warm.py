"""Learned warm start: the tile transform around the network and the
per-tile fallback judge (FP64).  TEST INFRASTRUCTURE ONLY.

The paper has no learned part; its Algorithm 1 leaves the starting point
open (u^(0) is only "initialised").  The warm start here sets that starting
point x^0 = u^0 per tile and nothing else, so Algorithm 1 runs unchanged
after it.  It is defined as follows.

Tile transform (tile t with block B_t and support P_t = B_t dilated by r):

    s_t        = max(1e-6, mean over B_t of max(y, 0))          (tile scale)
    yhat_t(i)  = y(c(i)) / s_t  for i in P_t                     (network input)
    x0_t       = max(0, s_t * net(yhat_t))                       (network start)

where c(i) is the nearest observed pixel (each coordinate clamped into
[0, M)), and net is the residual network of ``oracle.cnn`` evaluated on the
support-sized image with zero padding outside it.

Fallback judge.  The plain start is x0_plain = max(y(c(i)), 0) (the
'observed' start of ``oracle.solver.initial_tiles``).  For a start x the
gradient map of tile t is

    G_t(x) = || x - P(x - tau_t grad f_t(x)) ||

with P the projection onto x >= 0 (identity without positivity), tau_t the
Local-Solver step 1/L_t, and grad f_t the gradient of the tile's smooth
cost 1/2 ||y_t - H_t x||^2_W + lambda phi(D x).  G_t is zero exactly at the
minimisers of f_t + iota_{>=0}, so it measures how far a start is from
stationarity.  The network start of tile t is kept only if both maps are
finite and G_t(x_net) <= (1 - margin) G_t(x_plain) with margin = 1e-3;
otherwise the tile starts from x0_plain.  The margin makes a network that
returns its input (whose start equals the plain one up to rounding) fall
back.

This module shares no code with the HIP library; it uses the oracle's own
operator, prior, solver and network.

Parity pins (tests/test_oracle_warm.py and tests/golden/): the tile scale and
network input on a hand-derived 2 x 2 layout, the gradient map on a
delta-PSF tile derived by hand, stationarity (G = 0) at a tile minimiser
from the dense minimiser, and the identity network falling back on every
tile.
"""
from __future__ import annotations

import numpy as np

from . import cnn
from . import solver

SCALE_FLOOR = 1e-6
MARGIN = 1e-3


def _nearest_observed(problem, t):
    """y at the nearest observed pixel of every support pixel of tile t."""
    L = problem.layout
    (y0, y1), (x0, x1) = L.support(t)
    iy = np.clip(np.arange(y0, y1), 0, L.ay.M - 1)
    ix = np.clip(np.arange(x0, x1), 0, L.ax.M - 1)
    return problem.y[np.ix_(iy, ix)]


def tile_scale(problem, t):
    """s_t = max(1e-6, mean over the block of max(y, 0))."""
    blk = problem.y_t(t)
    return max(SCALE_FLOOR, float(np.mean(np.maximum(blk, 0.0))))


def tile_inputs(problem):
    """Network inputs y(nearest observed pixel) / s_t on each support, and
    the scales s_t."""
    scales = [tile_scale(problem, t) for t in range(problem.n_tiles)]
    ins = [_nearest_observed(problem, t) / scales[t] for t in range(problem.n_tiles)]
    return ins, scales


def network_start_tile(problem, net_params, t, bf16=True):
    """x0_t = max(0, s_t * net(yhat_t)) of one tile."""
    s = tile_scale(problem, t)
    o, _ = cnn.forward(net_params, (_nearest_observed(problem, t) / s)[None], bf16=bf16)
    return np.maximum(s * o[0], 0.0)


def network_start(problem, net_params, bf16=True, tile_map=None):
    """x0_t = max(0, s_t * net(yhat_t)) per tile.  net_params: list of (W, b)
    of ``oracle.cnn``; bf16 rounds where the GPU network stores BF16.
    ``tile_map`` (optional) evaluates the tiles: it takes a list of argument
    tuples (net_params, t, bf16) of :func:`network_start_tile` after
    ``problem`` and returns the results in order."""
    jobs = [(net_params, t, bf16) for t in range(problem.n_tiles)]
    if tile_map is None:
        return [network_start_tile(problem, *j) for j in jobs]
    return list(tile_map(jobs))


def gradient_map(problem, t, x, tau):
    """G_t(x) = ||x - P(x - tau grad f_t(x))||; the prox term of the
    Local-Solver's objective vanishes at u = x, so its gradient is that of
    f_t's smooth part."""
    g = solver.prox_gradient(problem, t, x, x)
    z = x - tau * g
    if problem.positivity:
        z = np.maximum(z, 0.0)
    return float(np.linalg.norm(x - z))


def judge(problem, x_net, x_plain, taus=None, margin=MARGIN):
    """Per-tile choice between the network start and the plain start.

    Returns (starts, keep, maps): the chosen starts, keep[t] = True where the
    network's start was kept, and maps[t] = (G_t(x_net), G_t(x_plain))."""
    if taus is None:
        taus = [solver.step_size(problem, t) for t in range(problem.n_tiles)]
    starts, keep, maps = [], [], []
    for t in range(problem.n_tiles):
        a = gradient_map(problem, t, x_net[t], taus[t])
        b = gradient_map(problem, t, x_plain[t], taus[t])
        k = bool(np.isfinite(a) and np.isfinite(b) and a <= (1.0 - margin) * b)
        starts.append((x_net[t] if k else x_plain[t]).copy())
        keep.append(k)
        maps.append((a, b))
    return starts, keep, maps


def warm_start(problem, net_params, bf16=True, taus=None, margin=MARGIN, tile_map=None):
    """The whole warm start: network starts, plain starts, per-tile judge.
    Returns (starts, keep, maps) as :func:`judge`."""
    x_net = network_start(problem, net_params, bf16=bf16, tile_map=tile_map)
    x_plain = solver.initial_tiles(problem, "observed")
    return judge(problem, x_net, x_plain, taus, margin)
