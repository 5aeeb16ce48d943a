"""Distributed D-R deblurring solver (Algorithm 1), FP64 reference.

Per tile t the local cost is (Section III-A)

    f_t(x) = 1/2 ||y_t - H_t x||^2_{W_t} + lambda phi(D x) + iota_{>=0}(x).

Algorithm 1 iterates, with metric alpha_t = gamma omega_t (Section III-B):

    x_t  <- prox_{alpha_t^-1, f_t}(u_t)                 (Local-Solver)
    zbar <- sum_t alpha_t (2 x_t - u_t) / sum_t alpha_t  (the Lemma: weighted
                                                          average over the
                                                          tiles covering a pixel)
    u_t  <- u_t + rho (zbar|_t - x_t)

The Local-Solver is inexact and warm-started from the previous x_t (Section
IV-B allows any fast method and inexact prox steps).  Here it is projected
gradient on the prox objective f_t(w) + 1/2 ||w - u_t||^2_{alpha_t}:

    g = H_t^T W_t (H_t w - y_t) + lambda grad phi(w) + alpha_t (w - u_t)
    w <- max(0, w - tau_t g),

with tau_t = 1/L_t and L_t = max(W_t) max(H_t 1) + lambda L_phi + gamma
max(omega_t), an upper bound on the Lipschitz constant of the gradient
(max(H_t 1) is the largest row sum of H_t; its column sums are at most 1 for
non-negative unit-sum PSFs and tents summing to one, so ||H_t||^2 <= max(H_t 1)).

A second Local-Solver (method "fista") takes the same gradient steps with
Nesterov momentum, as in FISTA (Beck and Teboulle, 2009, the accelerated
proximal-gradient method the paper cites among fast first-order solvers):

    w_j = max(0, y_j - tau_t g(y_j)),
    y_{j+1} = w_j + beta_j (w_j - w_{j-1}),  beta_j = (s_j - 1) / s_{j+1},
    s_1 = 1,  s_{j+1} = (1 + sqrt(1 + 4 s_j^2)) / 2,

restarted at every call from y_1 = w_0 = the warm start.  The run returns
w_n, so the last step's momentum (which would only move the unused y_{n+1})
is taken as 0.

The paper's own Local-Solver (Section IV-B) is VMLM-B, a limited-memory
variable-metric (BFGS) method with bound constraints whose step length comes
from a line search (method "vmlmb").  Each iteration, from w with gradient g:

    F    = the free variables: all but those with w_i <= 0 and g_i > 0
           (every variable without positivity)
    d    = -F . B (F . g)         B the limited-memory inverse BFGS matrix of
                                  the last m pairs (s_i, y_i) (two-loop
                                  recursion, initial scaling <s, y>/<y, y> of
                                  the newest pair, 1 with no pair)
    w(a) = P(w + a d),  a = tau_t with no pair, else 1, halved until
           f(w(a)) - f(w) <= c1 <g, w(a) - w>           (c1 = 1e-4, Armijo)
    s    = w(a) - w,  y = g(w(a)) - g,  kept if <s, y> > 0 (else the memory
           is cleared), the oldest pair dropped beyond m = 5.

The change f(w(a)) - f(w) of the prox objective is evaluated through its
exact expansion in D = w(a) - w (prox_objective_change), which has no
cancellation: a difference of two objective values would stop the line
search once the decrease falls below the rounding of the values themselves.
B is positive definite (every kept pair has <s, y> > 0), so d is a descent
direction whenever F . g != 0; with no pair the step is the projected
gradient step of length tau_t, which satisfies the Armijo test by the
descent lemma.  If 30 halvings fail (rounding), the iteration takes no step
and clears the memory.  The memory starts empty at every call (each round's
Local-Solver run is a fresh VMLM-B run warm-started from x_t).

One "iteration" is one Local-Solver step on every tile; consensus runs
after every n_inner of them.  The residual is the D-R fixed-point residual
||u^{k+1} - u^k|| / ||u^{k+1}|| over all tiles.  The output image is
sum_t omega_t x_t on X.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import prior
from .operator import DirectOperator


@dataclasses.dataclass
class Problem:
    layout: object
    psfs: np.ndarray           # [G_y, G_x, P, P]
    y: np.ndarray              # observed image [M_y, M_x]
    W: np.ndarray              # inverse-variance weights [M_y, M_x]
    lam: float = 1e-3
    reg: str = "tv"            # "tv" | "huber"
    reg_param: float = 1e-3    # eps for tv, delta for huber
    bc: str = "neumann"        # "neumann" | "circular"
    gamma: float = 0.4
    rho: float = 1.0
    positivity: bool = True
    operator: object = None    # DirectOperator (default) or FFTOperator

    def __post_init__(self):
        if self.operator is None:
            self.operator = DirectOperator(self.layout, self.psfs)

    @property
    def n_tiles(self):
        return self.layout.n_tiles

    def y_t(self, t):
        return self.layout.block_of(self.y, t)

    def W_t(self, t):
        return self.layout.block_of(self.W, t)

    def alpha_t(self, t):
        return self.gamma * self.layout.omega(t)

    def H(self, t, x):
        return self.operator.apply_H(t, x)

    def Ht(self, t, s):
        return self.operator.apply_Ht(t, s)


def row_sum_bound(problem, t):
    """max over B_t of H_t 1 (the largest row sum of H_t)."""
    ones = np.ones(problem.layout.support_shape(t))
    return float(np.max(problem.H(t, ones)))


def step_size(problem, t):
    """tau_t = 1 / L_t (see module docstring)."""
    L = (float(np.max(problem.W_t(t))) * row_sum_bound(problem, t)
         + problem.lam * prior.lipschitz(problem.reg, problem.reg_param)
         + float(np.max(problem.alpha_t(t))))
    return 1.0 / L


def prox_objective(problem, t, w, u):
    """f_t(w) + 1/2 ||w - u||^2_alpha (the Local-Solver's target)."""
    d = problem.H(t, w) - problem.y_t(t)
    data = 0.5 * float(np.sum(problem.W_t(t) * d * d))
    reg = problem.lam * prior.value(w, problem.reg, problem.reg_param, problem.bc)
    e = w - u
    return data + reg + 0.5 * float(np.sum(problem.alpha_t(t) * e * e))


def prox_objective_change(problem, t, w, u, dw, r=None):
    """prox_objective(w + dw) - prox_objective(w) by its exact expansion:
    with r = H_t w - y_t and e = H_t dw,
      1/2 sum W (r + e)^2 - 1/2 sum W r^2 = sum W e (r + e/2),
      1/2 sum alpha (w + dw - u)^2 - 1/2 sum alpha (w - u)^2
          = sum alpha dw (w - u + dw/2),
    and the regulariser's change per pixel (prior.value_change)."""
    if r is None:
        r = problem.H(t, w) - problem.y_t(t)
    e = problem.H(t, dw)
    data = float(np.sum(problem.W_t(t) * e * (r + 0.5 * e)))
    reg = problem.lam * prior.value_change(w, dw, problem.reg, problem.reg_param, problem.bc)
    metric = float(np.sum(problem.alpha_t(t) * dw * (w - u + 0.5 * dw)))
    return data + reg + metric


def prox_gradient(problem, t, w, u):
    """Gradient of the smooth part of the prox objective at w."""
    r = problem.W_t(t) * (problem.H(t, w) - problem.y_t(t))
    g = problem.Ht(t, r)
    g = g + problem.lam * prior.gradient(w, problem.reg, problem.reg_param, problem.bc)
    return g + problem.alpha_t(t) * (w - u)


def fista_momentum(n_inner):
    """Momentum factors beta_1 .. beta_n of an n-step FISTA run (the module
    docstring): s_1 = 1, s_{j+1} = (1 + sqrt(1 + 4 s_j^2)) / 2, beta_j =
    (s_j - 1) / s_{j+1}, with beta_n = 0 (the run ends on w_n)."""
    beta = []
    s = 1.0
    for j in range(n_inner):
        s_next = (1.0 + np.sqrt(1.0 + 4.0 * s * s)) / 2.0
        beta.append((s - 1.0) / s_next if j + 1 < n_inner else 0.0)
        s = s_next
    return beta


VMLMB_MEMORY = 5
ARMIJO_C1 = 1e-4
MAX_BACKTRACKS = 30


def free_mask(problem, w, g):
    """1 on the free variables of the bound w >= 0, 0 on the active ones
    (w_i <= 0 with g_i > 0, where the projected step stays on the bound)."""
    if not problem.positivity:
        return np.ones_like(w)
    return np.where((w <= 0.0) & (g > 0.0), 0.0, 1.0)


def lbfgs_apply(pairs, q):
    """B q for the limited-memory inverse BFGS matrix B of `pairs` (oldest
    first, each (s, y) with <s, y> > 0), by the two-loop recursion: the
    newest pair first, then the initial matrix <s, y>/<y, y> I of the newest
    pair (I with no pair), then the pairs oldest first."""
    q = q.copy()
    coef = []
    for s, y in reversed(pairs):
        a = float(np.sum(s * q)) / float(np.sum(s * y))
        q -= a * y
        coef.append(a)
    if pairs:
        s, y = pairs[-1]
        q *= float(np.sum(s * y)) / float(np.sum(y * y))
    for (s, y), a in zip(pairs, reversed(coef)):
        b = float(np.sum(y * q)) / float(np.sum(s * y))
        q += (a - b) * s
    return q


def vmlmb(problem, t, w0, u, n_iter, tau, memory=VMLMB_MEMORY, history=None):
    """n_iter VMLM-B iterations on the prox subproblem of tile t from w0
    (module docstring).  history, if a list, receives per iteration
    (prox objective after it, accepted step length or 0, number of halvings,
    number of pairs in memory after it)."""
    w = w0.copy()
    g = prox_gradient(problem, t, w, u)
    f = prox_objective(problem, t, w, u)
    pairs = []
    for _ in range(n_iter):
        F = free_mask(problem, w, g)
        d = -F * lbfgs_apply(pairs, F * g)
        a = tau if not pairs else 1.0
        accepted, halvings = False, 0
        r = problem.H(t, w) - problem.y_t(t)
        for _ in range(MAX_BACKTRACKS):
            wa = w + a * d
            if problem.positivity:
                wa = np.maximum(wa, 0.0)
            df = prox_objective_change(problem, t, w, u, wa - w, r)
            if df <= ARMIJO_C1 * float(np.sum(g * (wa - w))):
                accepted = True
                break
            a *= 0.5
            halvings += 1
        if not accepted:
            pairs = []
            if history is not None:
                history.append((f, 0.0, halvings, 0))
            continue
        ga = prox_gradient(problem, t, wa, u)
        s, y = wa - w, ga - g
        if float(np.sum(s * y)) > 0.0:
            pairs = (pairs + [(s, y)])[-memory:]
        else:
            pairs = []
        w, g, f = wa, ga, f + df
        if history is not None:
            history.append((f, a, halvings, len(pairs)))
    return w


def local_solve(problem, t, w0, u, n_inner, tau=None, method="pg"):
    """n_inner steps on the prox subproblem of tile t: projected gradient
    ("pg"), its accelerated form ("fista") or VMLM-B ("vmlmb"); see the
    module docstring."""
    tau = step_size(problem, t) if tau is None else tau
    if method == "vmlmb":
        return vmlmb(problem, t, w0, u, n_inner, tau)
    if method == "pg":
        w = w0.copy()
        for _ in range(n_inner):
            w = w - tau * prox_gradient(problem, t, w, u)
            if problem.positivity:
                w = np.maximum(w, 0.0)
        return w
    if method != "fista":
        raise ValueError(method)
    w_prev = w0.copy()
    y = w0.copy()
    w = w0.copy()
    for beta in fista_momentum(n_inner):
        w = y - tau * prox_gradient(problem, t, y, u)
        if problem.positivity:
            w = np.maximum(w, 0.0)
        y = w + beta * (w - w_prev)
        w_prev = w
    return w


def initial_tiles(problem, mode="observed", tiles=None):
    """x^0 per tile ('zero' or 'observed'); u^0 = x^0.  ``tiles`` (default:
    all) lists the tiles to return, in that order.

    'observed': max(y, 0) read at the nearest observed pixel (coordinates
    clamped into [0, M)), so all tiles start from one common image on X.
    """
    L = problem.layout
    out = []
    for t in (range(problem.n_tiles) if tiles is None else tiles):
        shape = L.support_shape(t)
        if mode == "zero":
            out.append(np.zeros(shape))
            continue
        if mode != "observed":
            raise ValueError(mode)
        (y0, y1), (x0, x1) = L.support(t)
        iy = np.clip(np.arange(y0, y1), 0, L.ay.M - 1)
        ix = np.clip(np.arange(x0, x1), 0, L.ax.M - 1)
        out.append(np.maximum(problem.y[np.ix_(iy, ix)], 0.0))
    return out


def consensus_average(problem, v_tiles):
    """zbar on X: the alpha-weighted average of the tiles covering each pixel
    (the Lemma of Section III-B).  Returns (zbar, coverage count)."""
    L = problem.layout
    r = L.r
    num = np.zeros(L.X_shape)
    den = np.zeros(L.X_shape)
    cnt = np.zeros(L.X_shape, dtype=np.int64)
    for t in range(problem.n_tiles):
        (y0, y1), (x0, x1) = L.support(t)
        a = problem.alpha_t(t)
        sl = (slice(y0 + r, y1 + r), slice(x0 + r, x1 + r))
        num[sl] += a * v_tiles[t]
        den[sl] += a
        cnt[sl] += 1
    return num / den, cnt


def consensus_step(problem, x_tiles, u_tiles):
    """One consensus + dual update; returns (new u tiles, zbar)."""
    v = [2.0 * x - u for x, u in zip(x_tiles, u_tiles)]
    zbar, _ = consensus_average(problem, v)
    out = []
    for t in range(problem.n_tiles):
        out.append(u_tiles[t] + problem.rho * (problem.layout.restrict(zbar, t) - x_tiles[t]))
    return out, zbar


def residual(u_old, u_new):
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(u_new, u_old))
    den = sum(float(np.sum(a * a)) for a in u_new)
    return float(np.sqrt(num / den)) if den > 0 else 0.0


def assemble(problem, x_tiles):
    """x_hat = sum_t omega_t x_t on X (the consensus image at convergence)."""
    L = problem.layout
    r = L.r
    out = np.zeros(L.X_shape)
    for t in range(problem.n_tiles):
        (y0, y1), (x0, x1) = L.support(t)
        out[y0 + r:y1 + r, x0 + r:x1 + r] += L.omega(t) * x_tiles[t]
    return out


@dataclasses.dataclass
class Result:
    x: list
    u: list
    residuals: list
    x_hat: np.ndarray


def solve(problem, n_outer, n_inner=10, init="observed", x0=None, inner_growth=0,
          consensus=True, callback=None, local_solver="pg", tile_map=None):
    """Algorithm 1 with n_inner(k) = n_inner + inner_growth * k Local-Solver steps.

    ``consensus=False`` skips the consensus step (the paper's 'independent'
    baseline: each tile is deblurred on its own and the tiles are blended
    with omega at the end).  ``local_solver`` is "pg", "fista" or "vmlmb"; a FISTA
    run restarts in every round, as does a "vmlmb" run (empty memory).
    ``tile_map`` (optional) runs the round's
    independent local solves: it takes a list of argument tuples of
    :func:`local_solve` after ``problem`` and returns their results in
    order (the default calls local_solve on each in turn).
    """
    if tile_map is None:
        tile_map = lambda jobs: [local_solve(problem, *j) for j in jobs]   # noqa: E731
    x = [a.copy() for a in (x0 if x0 is not None else initial_tiles(problem, init))]
    u = [a.copy() for a in x]
    taus = [step_size(problem, t) for t in range(problem.n_tiles)]
    res = []
    for k in range(n_outer):
        n_k = n_inner + inner_growth * k
        x = list(tile_map([(t, x[t], u[t], n_k, taus[t], local_solver) for t in range(problem.n_tiles)]))
        if consensus:
            u_new, _ = consensus_step(problem, x, u)
        else:
            # Independent tiles: each runs the proximal-point method on its own
            # f_t (u <- x), which converges to argmin f_t.
            u_new = [a.copy() for a in x]
        res.append(residual(u, u_new))
        u = u_new
        if callback is not None:
            callback(k, x, u)
    return Result(x, u, res, assemble(problem, x))
