"""The FISTA Local-Solver of the HIP library against the oracle's."""
import numpy as np
import pytest

from oracle import solver
from tests._problems import tiny_problem
from tests.test_gpu_solver import _f32, _mid_problem, small_workload_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("reg,bc", [("tv", "neumann"), ("huber", "circular"), ("huber", "neumann")])
def test_fista_inner_steps_match_oracle(reg, bc):
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _mid_problem(reg, bc, seed=11)
    ctx = context_of(prob, local_solver="fista")
    L = prob.layout
    rng = np.random.default_rng(12)
    x0 = [rng.random(L.support_shape(t)) for t in range(L.n_tiles)]
    u0 = [rng.random(L.support_shape(t)) for t in range(L.n_tiles)]
    tau = ctx.step_sizes()
    worst = 0.0
    for n in (1, 3, 6):
        ctx.set_state(to_dev(ctx.pack_list_support(x0)), to_dev(ctx.pack_list_support(u0)))
        ctx.solve_tiles(n)
        xg = ctx.unpack_support(ctx.get_state()[0].cpu().numpy())
        for t in range(L.n_tiles):
            ref = solver.local_solve(prob, t, _f32(x0[t]), _f32(u0[t]), n, float(tau[t]), "fista")
            err = rel_l2(xg[t], ref)
            worst = max(worst, err / n)
            assert err <= 1e-5 * n, (n, t, err)
            # FISTA and plain projected gradient part ways after two steps
            if n == 6:
                pg = solver.local_solve(prob, t, _f32(x0[t]), _f32(u0[t]), n, float(tau[t]), "pg")
                assert rel_l2(ref, pg) > 100 * rel_l2(xg[t], ref)
    print(f"FISTA inner steps ({reg}/{bc}): worst rel L2 per step {worst:.2e}")
    ctx.close()


def test_fista_small_workload_solve_matches_oracle():
    """256 x 256, 2 x 2 tiles, 5 rounds of 10 FISTA steps: final image <= 1e-4."""
    from tests._gpu import context_of, rel_l2
    prob, w = small_workload_problem()
    ctx = context_of(prob, local_solver="fista")
    ctx.init()
    res_gpu = ctx.run(w.n_outer, w.n_inner)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, w.n_outer, w.n_inner, local_solver="fista")
    err = rel_l2(xh, ref.x_hat)
    print(f"small workload, FISTA: rel L2 {err:.3e}, residuals gpu {res_gpu[-1]:.3e} oracle {ref.residuals[-1]:.3e}")
    assert err <= 1e-4
    assert np.allclose(res_gpu, ref.residuals, rtol=1e-3, atol=0)
    ctx.close()


def test_fista_two_step_rounds_equal_projected_gradient():
    """With two steps per round every momentum factor is 0."""
    from tests._gpu import context_of, rel_l2
    prob = _mid_problem(seed=13)
    out = []
    for m in ("pg", "fista"):
        ctx = context_of(prob, local_solver=m)
        ctx.init()
        res = ctx.run(3, 2)
        out.append((ctx.assemble().cpu().numpy(), res))
        ctx.close()
    assert rel_l2(out[1][0], out[0][0]) <= 1e-6
    assert np.allclose(out[1][1], out[0][1], rtol=1e-5)


def test_fista_tile_groups_give_identical_iterates():
    from tests._gpu import context_of, to_dev
    prob = _mid_problem(seed=14)
    ctx = context_of(prob, local_solver="fista")
    rng = np.random.default_rng(15)
    x0 = rng.random(ctx.support_total).astype(np.float32)
    u0 = rng.random(ctx.support_total).astype(np.float32)
    out = []
    for groups in (1, 2, 4):
        ctx.set_plan(tile_groups=groups)
        ctx.set_state(to_dev(x0), to_dev(u0))
        res = ctx.run(2, 5)
        x, u = ctx.get_state()
        out.append((x.cpu().numpy(), u.cpu().numpy(), res))
    for o in out[1:]:
        assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[1], out[0][1]) and o[2] == out[0][2]
    ctx.close()


def test_fista_rejects_the_growing_schedule():
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of
    prob = tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=16)
    ctx = context_of(prob, local_solver="fista")
    ctx.init()
    with pytest.raises(dl.DeblurError) as e:
        ctx.run(2, 2, growth=2)
    assert e.value.code == -1
    ctx.close()


def test_fista_context_warm_start_matches_projected_gradient_context():
    """The warm-start judge takes one step with no momentum, so a FISTA
    context keeps the same tiles and starts from the same state."""
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of
    from tests.test_gpu_cnn import _params
    prob = _mid_problem(seed=17)
    out = []
    for m in ("pg", "fista"):
        ctx = context_of(prob, local_solver=m)
        N = ctx.tiles[0].frame
        net = dl.Net(ctx.n_tiles, N, N, params=_params(21))
        use, nf = ctx.init_cnn(net)
        x, u = ctx.get_state()
        out.append((use.copy(), nf, x.cpu().numpy(), u.cpu().numpy()))
        net.close()
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2]) and np.array_equal(out[0][3], out[1][3])
