"""Pins of the VMLM-B Local-Solver of the oracle (the paper's limited-memory
variable-metric method with bound constraints, Section IV-B)."""
import numpy as np

from oracle import minimiser, solver
from oracle.minimiser import dense_matrix
from tests._problems import tiny_problem


def _bfgs_inverse(pairs, n):
    """The inverse BFGS matrix of `pairs` built densely by the update
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T (Nocedal and Wright,
    Eq. 6.17) from H0 = (<s, y>/<y, y> of the newest pair) I."""
    if not pairs:
        return np.eye(n)
    s, y = pairs[-1]
    H = float(s @ y) / float(y @ y) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / float(s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def test_two_loop_recursion_is_the_inverse_bfgs_matrix():
    rng = np.random.default_rng(0)
    n = 12
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)                    # SPD: <s, A s> > 0
    for m in (0, 1, 3, 5):
        pairs = []
        for _ in range(m):
            s = rng.standard_normal(n)
            pairs.append((s, A @ s))
        q = rng.standard_normal(n)
        got = solver.lbfgs_apply([(s.reshape(3, 4), y.reshape(3, 4)) for s, y in pairs], q.reshape(3, 4))
        ref = _bfgs_inverse(pairs, n) @ q
        assert np.allclose(got.ravel(), ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_secant_condition_of_the_newest_pair():
    # B y = s for the newest pair (the secant equation)
    rng = np.random.default_rng(1)
    A = np.diag(rng.random(20) + 0.5)
    pairs = [(s, A @ s) for s in rng.standard_normal((4, 20))]
    s, y = pairs[-1]
    assert np.allclose(solver.lbfgs_apply(pairs, y), s, rtol=1e-12, atol=1e-12)


def test_first_iteration_is_the_projected_gradient_step():
    # no pair: d = -F g with step tau_t, which the descent lemma accepts at once
    P = tiny_problem(seed=4)
    rng = np.random.default_rng(3)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        w0 = rng.random(P.layout.support_shape(t))
        tau = solver.step_size(P, t)
        hist = []
        a = solver.vmlmb(P, t, w0, u, 1, tau, history=hist)
        b = solver.local_solve(P, t, w0, u, 1, tau, method="pg")
        assert np.array_equal(a, b)
        assert hist[0][1] == tau and hist[0][2] == 0 and hist[0][3] == 1


def test_monotone_and_memory_bounded():
    P = tiny_problem(seed=5)
    rng = np.random.default_rng(4)
    t = 1
    u = rng.random(P.layout.support_shape(t))
    w0 = rng.random(P.layout.support_shape(t))
    hist = []
    solver.vmlmb(P, t, w0, u, 40, solver.step_size(P, t), history=hist)
    f = [solver.prox_objective(P, t, w0, u)] + [h[0] for h in hist]
    assert all(b <= a + 1e-14 * abs(a) for a, b in zip(f, f[1:]))
    assert max(h[3] for h in hist) == solver.VMLMB_MEMORY
    assert any(h[1] == 1.0 for h in hist)          # quasi-Newton steps taken at full length


def test_limit_is_closed_form():
    # quadratic prox objective (Huber with huge delta), no positivity:
    # (H^T W H + lambda D^T D + diag alpha) w = H^T W y + alpha u
    P = tiny_problem(seed=2, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=2.0)
    rng = np.random.default_rng(1)
    for t in range(P.n_tiles):
        u = rng.random(P.layout.support_shape(t))
        ref = minimiser.prox_quadratic_solution(P, t, u)
        w = solver.local_solve(P, t, np.zeros_like(u), u, 300, method="vmlmb")
        assert np.max(np.abs(w - ref)) <= 1e-10 * max(1, np.max(np.abs(ref)))


def test_faster_than_projected_gradient_on_the_quadratic():
    P = tiny_problem(seed=2, reg="huber", reg_param=1e12, positivity=False, lam=0.05, gamma=2.0)
    rng = np.random.default_rng(5)
    t = 0
    u = rng.random(P.layout.support_shape(t))
    ref = minimiser.prox_quadratic_solution(P, t, u)
    err = {m: np.max(np.abs(solver.local_solve(P, t, np.zeros_like(u), u, 30, method=m) - ref))
           for m in ("pg", "vmlmb")}
    assert err["vmlmb"] < 0.1 * err["pg"], err


def test_kkt_with_positivity_and_tv():
    P = tiny_problem(seed=3, gamma=2.0)
    rng = np.random.default_rng(2)
    t = 0
    u = rng.standard_normal(P.layout.support_shape(t))      # pushes some pixels to zero
    w = solver.local_solve(P, t, np.zeros_like(u), u, 400, method="vmlmb")
    g = solver.prox_gradient(P, t, w, u)
    assert np.all(w >= 0) and (w == 0).any()
    assert np.max(np.abs(np.where(w > 0, g, 0))) <= 1e-9
    assert np.min(np.where(w == 0, g, 0)) >= -1e-9


def test_free_mask_and_descent_direction():
    P = tiny_problem(seed=6)
    rng = np.random.default_rng(6)
    t = 0
    shape = P.layout.support_shape(t)
    w = np.maximum(rng.standard_normal(shape), 0.0)
    u = rng.random(shape)
    g = solver.prox_gradient(P, t, w, u)
    F = solver.free_mask(P, w, g)
    assert np.array_equal(F == 0, (w <= 0) & (g > 0))
    n = w.size
    A = rng.standard_normal((n, n))
    A = A @ A.T + np.eye(n)
    pairs = [(s.reshape(shape), (A @ s).reshape(shape)) for s in rng.standard_normal((3, n))]
    d = -F * solver.lbfgs_apply(pairs, F * g)
    assert float(np.sum(d * g)) < 0.0
    assert not d[F == 0].any()


def test_dr_limit_matches_minimiser():
    # the D-R limit does not depend on the Local-Solver
    P = tiny_problem(seed=7, lam=0.05, reg_param=0.5, gamma=1.0)
    P.y = P.y - 0.45
    res = solver.solve(P, n_outer=300, n_inner=5, local_solver="vmlmb")
    xstar, kkt = minimiser.minimise(P, tol=1e-14)
    assert kkt < 1e-11
    assert np.max(np.abs(res.x_hat - xstar)) <= 1e-9 * np.max(np.abs(xstar))


def test_objective_change_is_the_difference_of_objectives():
    rng = np.random.default_rng(8)
    for kw in (dict(), dict(reg="huber", reg_param=0.3), dict(bc="circular"), dict(reg="huber", reg_param=0.05)):
        P = tiny_problem(seed=9, **kw)
        for t in range(P.n_tiles):
            shape = P.layout.support_shape(t)
            w, u, dw = rng.random(shape), rng.random(shape), 0.3 * rng.standard_normal(shape)
            ref = solver.prox_objective(P, t, w + dw, u) - solver.prox_objective(P, t, w, u)
            got = solver.prox_objective_change(P, t, w, u, dw)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (kw, got, ref)


def test_objective_change_keeps_its_relative_accuracy_for_tiny_steps():
    # the difference of two objective values loses every digit for a step of
    # 1e-9; the expansion does not: it is linear in dw to first order
    P = tiny_problem(seed=10)
    rng = np.random.default_rng(9)
    t = 0
    shape = P.layout.support_shape(t)
    w, u, dw = rng.random(shape), rng.random(shape), rng.standard_normal(shape)
    g = solver.prox_gradient(P, t, w, u)
    for h in (1e-6, 1e-9, 1e-12):
        got = solver.prox_objective_change(P, t, w, u, h * dw)
        assert abs(got / (h * float(np.sum(g * dw))) - 1.0) <= 1e-3
