"""Result oracle: direct solutions of the consensus problem Eq. (4).

Consensus (x_1, ..., x_N) in C means x_t = S_t x for one image x on X, so
Eq. (4) equals

    min_{x >= 0} F(x) = sum_t [ 1/2 ||y_t - H_t S_t x||^2_{W_t} + lambda phi(D S_t x) ].

This is not the centralised problem Eq. (3): data in overlaps are counted in
every covering tile and the prior is a sum over tiles (Section II-B).  The
D-R iteration converges to its minimiser (Section III-B, with summable prox
errors), so these solvers pin the iterative oracle's limit.  They are meant
for images of a few hundred pixels only.
"""
from __future__ import annotations

import numpy as np

from . import prior


def global_objective(problem, x):
    L = problem.layout
    total = 0.0
    for t in range(L.n_tiles):
        xt = L.restrict(x, t)
        d = problem.H(t, xt) - problem.y_t(t)
        total += 0.5 * float(np.sum(problem.W_t(t) * d * d))
        total += problem.lam * prior.value(xt, problem.reg, problem.reg_param, problem.bc)
    return total


def global_gradient(problem, x):
    L = problem.layout
    r = L.r
    g = np.zeros_like(x)
    for t in range(L.n_tiles):
        xt = L.restrict(x, t)
        gt = problem.Ht(t, problem.W_t(t) * (problem.H(t, xt) - problem.y_t(t)))
        gt = gt + problem.lam * prior.gradient(xt, problem.reg, problem.reg_param, problem.bc)
        (y0, y1), (x0, x1) = L.support(t)
        g[y0 + r:y1 + r, x0 + r:x1 + r] += gt
    return g


def dense_matrix(fn, in_shape):
    """Matrix of a linear map, built column by column from unit inputs."""
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(fn(e.reshape(in_shape))).ravel())
    return np.stack(cols, axis=1)


def _tv_hessian(x, problem, shape):
    """Dense Hessian of lambda * phi(D x) on one support (TV or Huber)."""
    Dh = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[0], shape)
    Dv = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[1], shape)
    gh, gv = prior.forward_diff(x, problem.bc)
    gh, gv = gh.ravel(), gv.ravel()
    if problem.reg == "tv":
        m = np.sqrt(gh * gh + gv * gv + problem.reg_param ** 2)
        a = 1.0 / m - gh * gh / m ** 3
        b = -gh * gv / m ** 3
        c = 1.0 / m - gv * gv / m ** 3
    else:
        n = np.sqrt(gh * gh + gv * gv)
        d = problem.reg_param
        inside = n <= d
        ns = np.maximum(n, 1e-300)
        a = np.where(inside, 1.0, d / ns - d * gh * gh / ns ** 3)
        b = np.where(inside, 0.0, -d * gh * gv / ns ** 3)
        c = np.where(inside, 1.0, d / ns - d * gv * gv / ns ** 3)
    Hs = (Dh.T @ (a[:, None] * Dh) + Dh.T @ (b[:, None] * Dv)
          + Dv.T @ (b[:, None] * Dh) + Dv.T @ (c[:, None] * Dv))
    return problem.lam * Hs


def global_hessian(problem, x):
    """Dense Hessian of F at x (F is smooth; positivity handled outside)."""
    L = problem.layout
    shape = L.X_shape
    n = int(np.prod(shape))
    Hess = np.zeros((n, n))
    for t in range(L.n_tiles):
        sshape = L.support_shape(t)
        S = dense_matrix(lambda z: L.restrict(z, t), shape)
        Ht = dense_matrix(lambda z: problem.H(t, z), sshape)
        Wt = problem.W_t(t).ravel()
        At = Ht.T @ (Wt[:, None] * Ht) + _tv_hessian(L.restrict(x, t), problem, sshape)
        Hess += S.T @ At @ S
    return Hess


def minimise(problem, max_iter=200, tol=1e-13, x0=None):
    """Projected Newton (Bertsekas) on F with x >= 0, dense Hessians.

    Each step fixes the pixels at the bound whose gradient pushes outward,
    takes a Newton step on the others and backtracks along the projection
    arc (Armijo).  Stops when ||x - P(x - grad F(x))|| <= tol * max(1,
    ||grad F(0)||).  Returns (x, kkt residual).
    """
    L = problem.layout
    shape = L.X_shape
    proj = (lambda z: np.maximum(z, 0.0)) if problem.positivity else (lambda z: z)
    x = np.zeros(shape) if x0 is None else proj(x0.copy())
    scale = max(1.0, float(np.linalg.norm(global_gradient(problem, np.zeros(shape)))))
    kkt = np.inf
    for _ in range(max_iter):
        g = global_gradient(problem, x)
        kkt = float(np.linalg.norm(x - proj(x - g)))
        if kkt <= tol * scale:
            break
        gv, xv = g.ravel(), x.ravel()
        active = (xv <= 1e-14) & (gv > 0) if problem.positivity else np.zeros(xv.size, bool)
        free = ~active
        Hs = global_hessian(problem, x)
        d = np.zeros_like(xv)
        d[free] = -np.linalg.solve(Hs[np.ix_(free, free)], gv[free])
        d[active] = -gv[active]
        f0 = global_objective(problem, x)
        step = 1.0
        while True:
            xn = proj(x + step * d.reshape(shape))
            if global_objective(problem, xn) <= f0 + 1e-4 * float(np.sum(g * (xn - x))) or step < 1e-12:
                break
            step *= 0.5
        x = xn
    return x, kkt


def quadratic_solution(problem):
    """Dense solve of Eq. (4) for a quadratic prior and no positivity.

    Requires reg == 'huber' with a delta so large that phi = 1/2 ||D x||^2
    on the data; then grad F = 0 is the linear system
    (sum_t S_t^T (H_t^T W_t H_t + lambda D^T D) S_t) x = sum_t S_t^T H_t^T W_t y_t.
    """
    L = problem.layout
    shape = L.X_shape
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    b = np.zeros(n)
    for t in range(L.n_tiles):
        sshape = L.support_shape(t)
        Ht = dense_matrix(lambda z: problem.H(t, z), sshape)
        Dh = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[0], sshape)
        Dv = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[1], sshape)
        S = dense_matrix(lambda z: L.restrict(z, t), shape)
        Wt = problem.W_t(t).ravel()
        At = Ht.T @ (Wt[:, None] * Ht) + problem.lam * (Dh.T @ Dh + Dv.T @ Dv)
        A += S.T @ At @ S
        b += S.T @ (Ht.T @ (Wt * problem.y_t(t).ravel()))
    return np.linalg.solve(A, b).reshape(shape)


def prox_quadratic_solution(problem, t, u):
    """Dense solve of the prox subproblem of tile t for a quadratic prior and
    no positivity: (H^T W H + lambda D^T D + diag alpha) w = H^T W y + alpha u."""
    sshape = problem.layout.support_shape(t)
    Ht = dense_matrix(lambda z: problem.H(t, z), sshape)
    Dh = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[0], sshape)
    Dv = dense_matrix(lambda z: prior.forward_diff(z, problem.bc)[1], sshape)
    Wt = problem.W_t(t).ravel()
    al = problem.alpha_t(t).ravel()
    A = Ht.T @ (Wt[:, None] * Ht) + problem.lam * (Dh.T @ Dh + Dv.T @ Dv) + np.diag(al)
    b = Ht.T @ (Wt * problem.y_t(t).ravel()) + al * u.ravel()
    return np.linalg.solve(A, b).reshape(sshape)
