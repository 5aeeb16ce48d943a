"""Degenerate settings and error paths of the HIP tile solver against the oracle."""
import numpy as np
import pytest

from oracle import solver
from tests._problems import tiny_problem

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _f32_problem(prob):
    prob.psfs, prob.y, prob.W = _f32(prob.psfs), _f32(prob.y), _f32(prob.W)
    return prob


def _gpu_solve(prob, n_outer, n_inner):
    from tests._gpu import context_of
    ctx = context_of(prob)
    ctx.init()
    res = ctx.run(n_outer, n_inner)
    xh = ctx.assemble().cpu().numpy().astype(np.float64)
    ctx.close()
    return xh, res


@pytest.mark.parametrize("kw", [
    dict(lam=0.0, positivity=False, rho=1.5, gamma=0.05),      # no prior, no constraint, over-relaxed
    dict(lam=0.05, positivity=True, rho=0.5, gamma=2.0),       # under-relaxed, large metric
    dict(M=30, T=1, p=30, o=0, P=5, G=3, lam=0.02),            # a single tile (the proximal-point method)
    dict(M=24, T=3, p=8, o=0, P=3, G=3, model="local"),        # zero overlap, LOCAL
], ids=["lam0-nopos-rho1.5", "rho0.5-gamma2", "one-tile", "local-o0"])
def test_degenerate_settings_match_oracle(kw):
    from tests._gpu import rel_l2
    rho = kw.pop("rho", 1.0)
    M, T, p, o, P, G = (kw.pop(k, d) for k, d in (("M", 40), ("T", 2), ("p", 20), ("o", 4), ("P", 5), ("G", 2)))
    prob = _f32_problem(tiny_problem(M=M, T=T, p=p, o=o, P=P, G=G, seed=7, **kw))
    prob.rho = rho
    xh, res = _gpu_solve(prob, 3, 4)
    ref = solver.solve(prob, 3, 4)
    assert rel_l2(xh, ref.x_hat) <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=1e-7)


def test_consensus_only_rounds_match_oracle():
    """n_inner = 0: each round is the consensus and dual update alone, from a
    state with x != u (x stays fixed, u moves)."""
    from tests._gpu import context_of, rel_l2, to_dev
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=3))
    L = prob.layout
    rng = np.random.default_rng(8)
    x = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    u = [_f32(rng.random(L.support_shape(t))) for t in range(L.n_tiles)]
    ctx = context_of(prob)
    ctx.set_state(to_dev(ctx.pack_list_support(x)), to_dev(ctx.pack_list_support(u)))
    res = ctx.run(2, 0)
    xg, ug = (ctx.unpack_support(a.cpu().numpy()) for a in ctx.get_state())
    ctx.close()
    ref_res = []
    for _ in range(2):
        u_new, _ = solver.consensus_step(prob, x, u)
        ref_res.append(solver.residual(u, u_new))
        u = u_new
    for t in range(L.n_tiles):
        assert np.array_equal(xg[t], x[t].astype(np.float32))
        assert rel_l2(ug[t], u[t]) <= 1e-6
    assert np.allclose(res, ref_res, rtol=1e-4)


def test_zero_rounds_leave_the_state_unchanged():
    from tests._gpu import context_of
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=4))
    ctx = context_of(prob)
    ctx.init()
    x0, u0 = (a.cpu().numpy() for a in ctx.get_state())
    assert ctx.run(0, 10) == []
    x1, u1 = (a.cpu().numpy() for a in ctx.get_state())
    assert np.array_equal(x0, x1) and np.array_equal(u0, u1)
    ctx.close()


def test_error_paths():
    import torch
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of, params_of
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=5))
    ctx = context_of(prob, observe=False)
    with pytest.raises(dl.DeblurError) as e:          # no state yet
        ctx.run(1, 1)
    assert e.value.code == -5
    y = torch.zeros((40, 40), dtype=torch.float32, device="cuda")
    w = torch.full((40, 40), float("nan"), dtype=torch.float32, device="cuda")
    with pytest.raises(dl.DeblurError) as e:          # non-finite weights
        ctx.set_observation(y, w)
    assert e.value.code == -1
    with pytest.raises(dl.DeblurError) as e:          # init from a given state without one
        ctx.set_observation(y, torch.ones_like(y))
        ctx.init(dl.INIT_GIVEN, None)
    assert e.value.code == -1
    ctx.close()
    # geometry the library cannot tile: overlap + 2r beyond the pitch
    bad = params_of(prob)
    bad.overlap = 18
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(bad, prob.psfs)
    assert e.value.code == -2
    # even PSF size
    bad = params_of(prob)
    bad.P = 4
    with pytest.raises(dl.DeblurError) as e:
        dl.Context(bad, np.ones((2, 2, 4, 4)) / 16)
    assert e.value.code == -1


def test_psf_contract_is_enforced_through_the_gpu_binding():
    """A PSF that is negative somewhere or does not sum to 1 is rejected at
    creation (the step sizes assume unit-sum non-negative PSFs)."""
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import params_of
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=8))
    for k, change in ((1, 2.0), (3, -1.0)):
        psfs = prob.psfs.copy()
        psfs.reshape(4, 5, 5)[k] *= change
        with pytest.raises(dl.DeblurError) as e:
            dl.Context(params_of(prob), psfs)
        assert e.value.code == -1 and f"node {k}" in str(e.value), str(e.value)


def test_state_carries_the_round_index():
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=6))
    ctx = context_of(prob)
    ctx.init()
    assert ctx.state_round() == 0
    ctx.run(3, 2)
    assert ctx.state_round() == 3
    ctx.consensus()
    assert ctx.state_round() == 4
    x, u = ctx.get_state()
    ctx.set_state(x, u, round=7)
    assert ctx.state_round() == 7
    ctx.run(2, 2, growth=2, first_round=ctx.state_round())
    assert ctx.state_round() == 9
    ctx.init()
    assert ctx.state_round() == 0
    with pytest.raises(dl.DeblurError) as e:
        ctx.set_state(x, u, round=-1)
    assert e.value.code == -1
    ctx.close()


def test_nonfinite_error_names_the_diverged_tile():
    """A non-finite value planted (from the host) in one tile's x spreads to
    the neighbours' u through the consensus step; the error names the tile
    whose x is non-finite."""
    from paper_1705_06603_amd import _lib as dl
    from tests._gpu import context_of, to_dev
    prob = _f32_problem(tiny_problem(M=40, T=2, p=20, o=4, P=5, G=2, seed=7))
    ctx = context_of(prob)
    ctx.init()
    x, u = (a.cpu().numpy() for a in ctx.get_state())
    d = ctx.tiles[2]
    x[d.x_offset + 3] = np.nan
    ctx.set_state(to_dev(x), to_dev(u))
    with pytest.raises(dl.DeblurError) as e:
        ctx.run(1, 1)
    msg = str(e.value)
    assert e.value.code == -6 and "non-finite x in 1 tile(s): 2 (row 1, column 0)" in msg, msg
    ctx.close()
