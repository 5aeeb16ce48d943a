"""The independent baseline of the HIP library (params.independent: no
consensus, u_t <- x_t each round, the tiles blended with omega) against the
oracle's solve without consensus."""
import numpy as np
import pytest

from oracle import solver
from tests.test_gpu_solver import _mid_problem, small_workload_problem

pytestmark = pytest.mark.gpu


def test_independent_rounds_match_oracle():
    from tests._gpu import context_of, rel_l2
    prob = _mid_problem(seed=5)
    ctx = context_of(prob, independent=True)
    ctx.init()
    res = ctx.run(4, 5)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, 4, 5, consensus=False)
    err = rel_l2(xh, ref.x_hat)
    print(f"independent, 4 rounds of 5: rel L2 {err:.2e}")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
    # the consensus step alone is u <- x
    x, u = ctx.get_state()
    assert np.array_equal(x.cpu().numpy(), u.cpu().numpy())
    ctx.close()


def test_independent_small_workload_matches_oracle():
    """256 x 256, 2 x 2 tiles, 50 iterations without consensus."""
    from tests._gpu import context_of, rel_l2
    prob, w = small_workload_problem()
    ctx = context_of(prob, independent=True)
    ctx.init()
    res = ctx.run(w.n_outer, w.n_inner)
    xh = ctx.assemble().cpu().numpy()
    ref = solver.solve(prob, w.n_outer, w.n_inner, consensus=False)
    err = rel_l2(xh, ref.x_hat)
    print(f"independent small workload: rel L2 {err:.2e}")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
    ctx.close()


def test_independent_flag_is_validated():
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import params_of
    prob = _mid_problem(seed=5)
    p = params_of(prob)
    p.independent = 2
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(p, prob.psfs)
    assert e.value.code == -1
