"""Pins of the Local-Solver, the consensus step and the D-R iteration."""
import numpy as np
import pytest

from oracle import minimiser, solver
from oracle.minimiser import dense_matrix
from tests._problems import tiny_problem


def test_step_size_bounds_lipschitz():
    P = tiny_problem()
    for t in range(P.n_tiles):
        shape = P.layout.support_shape(t)
        A = dense_matrix(lambda z: P.Ht(t, P.W_t(t) * P.H(t, z)), shape)
        lam_data = np.linalg.eigvalsh(0.5 * (A + A.T)).max()
        # TV Hessian bound 8 lambda / eps, plus the metric term
        L_true = lam_data + P.lam * 8.0 / P.reg_param + P.alpha_t(t).max()
        assert 1.0 / solver.step_size(P, t) >= lam_data + P.alpha_t(t).max() - 1e-12
        assert 1.0 / solver.step_size(P, t) >= L_true * (1 - 1e-12)


def test_local_solver_monotone():
    P = tiny_problem(seed=1)
    rng = np.random.default_rng(0)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        w = rng.random(P.layout.support_shape(t))
        tau = solver.step_size(P, t)
        prev = solver.prox_objective(P, t, w, u)
        for _ in range(30):
            w = solver.local_solve(P, t, w, u, 1, tau)
            cur = solver.prox_objective(P, t, w, u)
            assert cur <= prev + 1e-13
            prev = cur


def test_local_solver_limit_is_closed_form():
    # lambda phi = 1/2 lambda ||D x||^2 (Huber with huge delta), no positivity:
    # the prox solution solves (H^T W H + lambda D^T D + diag alpha) w = H^T W y + alpha u.
    P = tiny_problem(seed=2, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=2.0)
    rng = np.random.default_rng(1)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        ref = minimiser.prox_quadratic_solution(P, t, u)
        w = solver.local_solve(P, t, np.zeros_like(u), u, 1500)
        assert np.max(np.abs(w - ref)) <= 1e-10 * max(1, np.max(np.abs(ref)))


def test_local_solver_kkt_with_positivity():
    P = tiny_problem(seed=3, gamma=2.0)
    rng = np.random.default_rng(2)
    t = 0
    u = rng.standard_normal(P.layout.support_shape(t))      # pushes some pixels to zero
    w = solver.local_solve(P, t, np.zeros_like(u), u, 3000)
    g = solver.prox_gradient(P, t, w, u)
    assert np.all(w >= 0)
    assert (w == 0).any()
    assert np.max(np.abs(np.where(w > 0, g, 0))) <= 1e-9
    assert np.min(np.where(w == 0, g, 0)) >= -1e-9


def test_consensus_is_weighted_projection():
    P = tiny_problem(M=18, T=3, p=6, o=2, P=3, G=3, seed=4)
    L = P.layout
    rng = np.random.default_rng(3)
    v = [rng.standard_normal(L.support_shape(t)) for t in range(P.n_tiles)]
    zbar, cnt = solver.consensus_average(P, v)
    assert cnt.max() == 4
    # Independent route: weighted least squares min_x sum_t ||sqrt(alpha_t)(S_t x - v_t)||^2
    rows, rhs = [], []
    for t in range(P.n_tiles):
        S = dense_matrix(lambda z: L.restrict(z, t), L.X_shape)
        sa = np.sqrt(P.alpha_t(t).ravel())
        rows.append(sa[:, None] * S)
        rhs.append(sa * v[t].ravel())
    xls = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0].reshape(L.X_shape)
    assert np.max(np.abs(xls - zbar)) <= 1e-13
    # projection properties: idempotent, lands in C, V-orthogonal residual
    z_t = [L.restrict(zbar, t) for t in range(P.n_tiles)]
    z2, _ = solver.consensus_average(P, z_t)
    assert np.max(np.abs(z2 - zbar)) <= 1e-14
    c = rng.standard_normal(L.X_shape)
    ip = sum(np.sum(P.alpha_t(t) * (v[t] - z_t[t]) * (L.restrict(c, t) - z_t[t])) for t in range(P.n_tiles))
    assert abs(ip) <= 1e-12


def test_single_tile_is_proximal_point_to_minimiser():
    # N = 1: consensus is the identity, D-R is the proximal-point method and
    # converges to argmin f.  Data shifted down so positivity is active.
    P = tiny_problem(M=10, T=1, p=10, o=0, P=3, G=2, seed=5, lam=0.05, reg_param=0.5, gamma=0.25)
    P.y = P.y - 0.45
    res = solver.solve(P, n_outer=250, n_inner=10)
    xstar, kkt = minimiser.minimise(P, tol=1e-14)
    assert kkt < 1e-11
    assert (xstar == 0).sum() > 5
    assert np.max(np.abs(res.x_hat - xstar)) <= 1e-9 * np.max(np.abs(xstar))


def test_dr_limit_quadratic_matches_dense_solve():
    P = tiny_problem(seed=6, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=1.0)
    res = solver.solve(P, n_outer=600, n_inner=10)
    ref = minimiser.quadratic_solution(P)
    assert res.residuals[-1] < 1e-12
    assert np.max(np.abs(res.x_hat - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_dr_limit_tv_positivity_matches_minimiser():
    # 2 x 2 tiles, smoothed TV, positivity active on part of the image: the
    # D-R limit is the minimiser of the consensus problem Eq. (4).
    P = tiny_problem(seed=7, lam=0.05, reg_param=0.5, gamma=1.0)
    P.y = P.y - 0.45
    res = solver.solve(P, n_outer=300, n_inner=10)
    xstar, kkt = minimiser.minimise(P, tol=1e-14)
    assert kkt < 1e-11
    assert (xstar == 0).sum() > 20
    assert np.max(np.abs(res.x_hat - xstar)) <= 1e-9 * np.max(np.abs(xstar))
    # at convergence all tiles agree on their overlaps
    L = P.layout
    for t in range(P.n_tiles):
        assert np.max(np.abs(res.x[t] - L.restrict(res.x_hat, t))) <= 1e-9


def test_residual_decreases_on_small_workload_shape():
    P = tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=8, lam=1e-3, reg_param=1e-2)
    res = solver.solve(P, n_outer=30, n_inner=10)
    assert res.residuals[-1] < 0.1 * res.residuals[0]


# ---------------------------------------------------------------------------
# FISTA Local-Solver (accelerated projected gradient)
# ---------------------------------------------------------------------------

def test_fista_momentum_sequence():
    # Beck-Teboulle: s_1 = 1 and s_j >= (j + 1) / 2, so beta_j = (s_j - 1) / s_{j+1}
    # lies in [0, 1); the first step has no momentum, and the last is set to 0.
    beta = solver.fista_momentum(50)
    assert beta[0] == 0.0 and beta[-1] == 0.0
    s = 1.0
    for j, b in enumerate(beta[:-1], start=1):
        assert s >= (j + 1) / 2 - 1e-12
        s_next = (1 + np.sqrt(1 + 4 * s * s)) / 2
        assert 0.0 <= b < 1.0
        s = s_next
    assert all(beta[j] < beta[j + 1] for j in range(len(beta) - 2))
    assert solver.fista_momentum(1) == [0.0] and solver.fista_momentum(2) == [0.0, 0.0]


def test_fista_short_runs_are_projected_gradient():
    # with one or two steps every momentum factor is 0: the runs are plain projected gradient
    P = tiny_problem(seed=4, gamma=1.0)
    rng = np.random.default_rng(5)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        w0 = rng.random(P.layout.support_shape(t))
        for n in (1, 2):
            a = solver.local_solve(P, t, w0, u, n, method="fista")
            b = solver.local_solve(P, t, w0, u, n, method="pg")
            assert np.array_equal(a, b)


def test_fista_limit_is_closed_form():
    P = tiny_problem(seed=2, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=2.0)
    rng = np.random.default_rng(1)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        ref = minimiser.prox_quadratic_solution(P, t, u)
        w = solver.local_solve(P, t, np.zeros_like(u), u, 1600, method="fista")
        assert np.max(np.abs(w - ref)) <= 1e-10 * max(1, np.max(np.abs(ref)))


def test_fista_rate_bound():
    # Beck-Teboulle, Theorem 4.4: F(w_k) - F* <= 2 L ||w_0 - w*||^2 / (k + 1)^2 for
    # any L >= the gradient's Lipschitz constant (here 1 / tau_t), on the
    # quadratic prox problem whose minimiser is known in closed form.
    P = tiny_problem(seed=2, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=2.0)
    rng = np.random.default_rng(3)
    t = 1
    u = rng.random(P.layout.support_shape(t))
    w0 = rng.random(P.layout.support_shape(t))
    ref = minimiser.prox_quadratic_solution(P, t, u)
    tau = solver.step_size(P, t)
    F_star = solver.prox_objective(P, t, ref, u)
    d0 = float(np.sum((w0 - ref) ** 2))
    gaps = []
    for k in (1, 2, 4, 8, 16, 32, 64, 128):
        w = solver.local_solve(P, t, w0, u, k, tau, method="fista")
        gap = solver.prox_objective(P, t, w, u) - F_star
        assert -1e-9 <= gap <= 2.0 / tau * d0 / (k + 1) ** 2
        gaps.append(gap)
    # and at 32 steps it is ahead of plain projected gradient
    w_pg = solver.local_solve(P, t, w0, u, 32, tau, method="pg")
    assert gaps[5] < solver.prox_objective(P, t, w_pg, u) - F_star


def test_fista_kkt_with_positivity():
    P = tiny_problem(seed=3, gamma=2.0)
    rng = np.random.default_rng(2)
    t = 0
    u = rng.standard_normal(P.layout.support_shape(t))
    w = solver.local_solve(P, t, np.zeros_like(u), u, 3000, method="fista")
    g = solver.prox_gradient(P, t, w, u)
    assert np.all(w >= 0) and (w == 0).any()
    assert np.max(np.abs(np.where(w > 0, g, 0))) <= 1e-9
    assert np.min(np.where(w == 0, g, 0)) >= -1e-9


def test_fista_dr_limit_matches_minimiser():
    # the D-R limit does not depend on the Local-Solver: with FISTA it is
    # still the minimiser of the consensus problem Eq. (4)
    P = tiny_problem(seed=7, lam=0.05, reg_param=0.5, gamma=1.0)
    P.y = P.y - 0.45
    res = solver.solve(P, n_outer=300, n_inner=10, local_solver="fista")
    xstar, kkt = minimiser.minimise(P, tol=1e-14)
    assert kkt < 1e-11
    assert np.max(np.abs(res.x_hat - xstar)) <= 1e-9 * np.max(np.abs(xstar))
    with_one = [solver.solve(P, 3, 1, local_solver=m).x_hat for m in ("pg", "fista")]
    assert np.array_equal(with_one[0], with_one[1])
