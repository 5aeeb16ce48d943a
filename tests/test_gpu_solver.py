"""Local-Solver, consensus and full D-R solves of the HIP library against the oracle."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import solver
from oracle.layout import make_layout
from oracle.solver import Problem
from paper_1705_06603_amd import workloads
from tests._problems import tiny_problem

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _as_f32_problem(prob):
    """Same problem with PSFs, y and W rounded to fp32 (what the GPU receives)."""
    return Problem(prob.layout, _f32(prob.psfs), _f32(prob.y), _f32(prob.W), lam=prob.lam, reg=prob.reg,
                   reg_param=prob.reg_param, bc=prob.bc, gamma=prob.gamma, rho=prob.rho,
                   positivity=prob.positivity)


def small_workload_problem():
    w = workloads.WORKLOADS["small"]
    scene, psfs = workloads.make_workload(w)
    L = make_layout(w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    blurred = op.apply_H_global(L, psfs, scene)
    y, W = workloads.observe(blurred, w.noise, w.seed)
    return _as_f32_problem(Problem(L, psfs, y, W, lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)), w


def _mid_problem(reg="tv", bc="neumann", model="interp", seed=0):
    L = make_layout(120, 2, 60, 8, 7, 2, model=model)
    rng = np.random.default_rng(seed)
    psfs = rng.random((2, 2, 7, 7)) ** 2
    psfs /= psfs.sum(axis=(2, 3), keepdims=True)
    xg = rng.random(L.X_shape) * 2
    y = op.apply_H_global(L, psfs, xg) + 0.05 * rng.standard_normal((120, 120)) - 0.3
    W = 0.5 + rng.random((120, 120))
    return _as_f32_problem(Problem(L, psfs, y, W, lam=0.05, reg=reg, reg_param=0.05 if reg == "tv" else 0.2,
                                   bc=bc, gamma=0.7, rho=1.0))


def test_step_sizes_match_oracle():
    from tests._gpu import context_of
    prob = _mid_problem()
    ctx = context_of(prob)
    tau = ctx.step_sizes()
    ref = np.array([solver.step_size(prob, t) for t in range(prob.n_tiles)])
    assert np.max(np.abs(tau - ref) / ref) <= 1e-5
    ctx.close()


@pytest.mark.parametrize("reg,bc,model", [("tv", "neumann", "interp"), ("huber", "circular", "interp"),
                                          ("tv", "neumann", "local"), ("huber", "neumann", "interp"),
                                          ("tv", "circular", "interp")])
def test_inner_steps_match_oracle(reg, bc, model):
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _mid_problem(reg, bc, model, seed=1)
    ctx = context_of(prob)
    L = prob.layout
    rng = np.random.default_rng(3)
    x0 = [rng.random(L.support_shape(t)) for t in range(L.n_tiles)]
    u0 = [rng.random(L.support_shape(t)) for t in range(L.n_tiles)]
    ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
    tau = ctx.step_sizes()
    for n in (1, 3):
        ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
        ctx.solve_tiles(n)
        xg, ug = ctx.get_state()
        xg = ctx.unpack_support(xg.cpu().numpy())
        for t in range(L.n_tiles):
            ref = solver.local_solve(prob, t, _f32(x0[t]), _f32(u0[t]), n, float(tau[t]))
            assert rel_l2(xg[t], ref) <= 1e-5 * n, (n, t, rel_l2(xg[t], ref))
    ctx.close()


def test_consensus_matches_oracle():
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _mid_problem(seed=2)
    ctx = context_of(prob)
    L = prob.layout
    rng = np.random.default_rng(5)
    x0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    u0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
    res = ctx.consensus()
    _, ug = ctx.get_state()
    ug = ctx.unpack_support(ug.cpu().numpy())
    u_ref, _ = solver.consensus_step(prob, x0, u0)
    for t in range(L.n_tiles):
        assert rel_l2(ug[t], u_ref[t]) <= 1e-6
    assert abs(res - solver.residual(u0, u_ref)) <= 1e-5 * solver.residual(u0, u_ref)
    xh = ctx.assemble().cpu().numpy()
    assert rel_l2(xh, solver.assemble(prob, x0)) <= 1e-6
    ctx.close()


def test_objective_matches_oracle():
    from tests._gpu import context_of, to_dev
    prob = _mid_problem(seed=4)
    ctx = context_of(prob)
    L = prob.layout
    rng = np.random.default_rng(6)
    x0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    u0 = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
    d, r, p = ctx.objective()
    ref = sum(solver.prox_objective(prob, t, x0[t], u0[t]) for t in range(L.n_tiles))
    assert abs((d + r + p) - ref) <= 1e-5 * ref
    ctx.close()


def test_small_workload_solve_matches_oracle():
    """256 x 256, 2 x 2 tiles, 50 iterations (5 rounds of 10): final image <= 1e-4."""
    from tests._gpu import context_of, rel_l2
    prob, w = small_workload_problem()
    ctx = context_of(prob)
    ctx.init()
    res_gpu = ctx.run(w.n_outer, w.n_inner)
    xh = ctx.assemble().cpu().numpy()
    taus = ctx.step_sizes()
    ref = solver.solve(prob, w.n_outer, w.n_inner)
    err = rel_l2(xh, ref.x_hat)
    print(f"small workload: rel L2 {err:.3e}, residuals gpu {res_gpu[-1]:.3e} oracle {ref.residuals[-1]:.3e}")
    assert err <= 1e-4
    assert np.allclose(res_gpu, ref.residuals, rtol=1e-3, atol=0)
    ctx.close()


def test_run_graph_equals_step_by_step():
    from tests._gpu import context_of
    prob = _mid_problem(seed=7)
    a = context_of(prob)
    b = context_of(prob)
    a.init()
    b.init()
    ra = a.run(3, 5)
    rb = []
    for _ in range(3):
        b.solve_tiles(5)
        rb.append(b.consensus())
    xa, ua = a.get_state()
    xb, ub = b.get_state()
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    assert np.array_equal(ua.cpu().numpy(), ub.cpu().numpy())
    assert ra == rb
    a.close()
    b.close()


def test_tiny_problem_reaches_minimiser():
    """D-R on the GPU converges to the same consensus minimiser as the oracle."""
    from tests._gpu import context_of, rel_l2
    from oracle import minimiser
    prob = tiny_problem(seed=7, lam=0.05, reg_param=0.5, gamma=1.0)
    prob.y = prob.y - 0.45
    prob = _as_f32_problem(prob)
    ctx = context_of(prob)
    ctx.init()
    res = ctx.run(400, 10, tol=1e-7)
    xh = ctx.assemble().cpu().numpy()
    xstar, kkt = minimiser.minimise(prob, tol=1e-12)
    assert rel_l2(xh, xstar) <= 1e-4, rel_l2(xh, xstar)
    ctx.close()


def test_growing_schedule_matches_oracle():
    """The paper's growing inexact schedule (round k runs n + g k steps): the
    GPU run against the oracle with the same schedule, and one schedule split
    over two calls equals it in one call."""
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of, rel_l2
    prob = _mid_problem(seed=4)
    ctx = context_of(prob)
    ctx.init()
    res = ctx.run(3, 2, growth=2)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, 3, 2, inner_growth=2)      # rounds of 2, 4 and 6 steps
    assert rel_l2(xh, ref.x_hat) <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
    ctx.init()
    res_a = ctx.run(2, 2, growth=2)
    res_b = ctx.run(1, 2, growth=2, first_round=2)
    assert res_a + res_b == res
    assert np.array_equal(ctx.assemble().cpu().numpy(), xh)
    with pytest.raises(dl.DeblurError) as e:
        ctx.run(1, 4, growth=2)                          # growth not a multiple of n_inner
    assert e.value.code == -1
    ctx.close()
