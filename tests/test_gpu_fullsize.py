"""Parity at full workload sizes on sampled tiles the oracle computes one by one.

The observation is written by the oracle only on the blocks of the sampled
tiles' neighbourhoods (the only data a single D-R round can reach); it is
zero elsewhere, which does not affect the sampled tiles.  The oracle uses its
FP64 FFT backend, itself pinned to the direct convolution.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle import solver
from oracle.layout import make_layout
from oracle.solver import Problem
from paper_1705_06603_amd import workloads

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _neighbourhood(L, tiles):
    out = set()
    for t in tiles:
        a, b = L.tile_ab(t)
        for da in (-1, 0, 1):
            for db in (-1, 0, 1):
                aa, bb = a + da, b + db
                if 0 <= aa < L.ay.T and 0 <= bb < L.ax.T:
                    out.add(aa * L.ax.T + bb)
    return sorted(out)


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _one_round_map(name, frame, sampled, rounds_before, plan=None, local_solver="pg"):
    """One-step map parity: the GPU state after ``rounds_before`` graph-captured
    D-R rounds is fed to the FP64 oracle, which runs one more round (n_inner
    Local-Solver steps + consensus + dual update, Algorithm 1) on the sampled
    tiles and their neighbours; the GPU's next state must agree.  ``plan``
    (launch-plan fields) selects the launch shapes, as the benchmark's
    autotuner does."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    w = workloads.WORKLOADS[name]
    scene, psfs = workloads.make_workload(w)
    psfs = _f32(psfs)
    L = make_layout(w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    need = _neighbourhood(L, sampled)
    two = _neighbourhood(L, need)                    # the init of the neighbours reads y around them
    F = op.FFTOperator(L, psfs, N=frame)
    rng = np.random.default_rng(77)
    y = np.zeros((w.M, w.M), dtype=np.float32)
    W = np.ones((w.M, w.M), dtype=np.float32)
    for t in two:
        (y0, y1), (x0, x1) = L.block(t)
        blk = F.apply_H(t, L.restrict(scene, t))
        y[y0:y1, x0:x1] = blk + 0.01 * rng.standard_normal(blk.shape)
        W[y0:y1, x0:x1] = 0.5 + rng.random(blk.shape)
    y, W = y.astype(np.float64), W.astype(np.float64)
    prob = Problem(L, psfs, y, W, lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho, operator=F)
    params = dl.make_params(w.M, w.tiles, w.pitch, w.overlap, w.grid, w.psf_size, lam=w.lam, reg_param=w.eps,
                            gamma=w.gamma, rho=w.rho,
                            local_solver=dl.SOLVER_FISTA if local_solver == "fista" else dl.SOLVER_PG)
    ctx = dl.Context(params, psfs)
    assert ctx.tiles[0].frame == frame
    if plan:
        ctx.set_plan(**plan)
    ctx.set_observation(torch.tensor(y.astype(np.float32), device="cuda"),
                        torch.tensor(W.astype(np.float32), device="cuda"))
    ctx.init()
    if rounds_before:
        ctx.run(rounds_before, w.n_inner)
    xk, uk = ctx.get_state()
    xk = [a.astype(np.float64) for a in ctx.unpack_support(xk.cpu().numpy())]
    uk = [a.astype(np.float64) for a in ctx.unpack_support(uk.cpu().numpy())]
    res = ctx.run(1, w.n_inner)
    x1, u1 = ctx.get_state()
    x1 = ctx.unpack_support(x1.cpu().numpy())
    u1 = ctx.unpack_support(u1.cpu().numpy())
    tau = ctx.step_sizes()
    v = [np.zeros(L.support_shape(t)) for t in range(L.n_tiles)]
    xs = {}
    for t in need:
        ref_tau = solver.step_size(prob, t)
        assert abs(tau[t] - ref_tau) <= 1e-5 * ref_tau
        xs[t] = solver.local_solve(prob, t, xk[t], uk[t], w.n_inner, float(tau[t]), local_solver)
        v[t] = 2.0 * xs[t] - uk[t]
    zbar, _ = solver.consensus_average(prob, v)
    for t in sampled:
        u_ref = uk[t] + w.rho * (L.restrict(zbar, t) - xs[t])
        ex, eu = _rel(x1[t], xs[t]), _rel(u1[t], u_ref)
        # the change over the round, which the rounding of x itself does not hide
        edx = _rel(x1[t] - xk[t], xs[t] - xk[t])
        print(f"{name} tile {t}: x {ex:.2e} u {eu:.2e} dx {edx:.2e}")
        assert ex <= 1e-5 and eu <= 1e-5
        assert edx <= 1e-4
    assert np.isfinite(res[0])
    ctx.close()


def test_batched_workload_one_round_map_on_sampled_tiles():
    """2048 x 2048, 8 x 8 tiles, 31 x 31 Moffat grid, frame 320; corner, edge,
    interior and far-corner tiles, first round and a later round."""
    _one_round_map("batched", 320, [0, 3, 4 * 8 + 5, 63], 0)
    # launch shapes the autotuner picks for this workload: 2-wave workgroups,
    # two or four concurrent tile groups
    _one_round_map("batched", 320, [0, 4 * 8 + 5], 3,
                   plan=dict(col_waves=2, row_waves=2, tile_order=2, tile_groups=2))
    _one_round_map("batched", 320, [3, 63], 1, plan=dict(col_waves=2, row_waves=2, tile_order=0, tile_groups=4))


def test_batched_workload_fista_round_on_sampled_tiles():
    """The FISTA Local-Solver at full size: one round of 10 accelerated steps
    on the batched workload, in the benchmark's launch shapes."""
    _one_round_map("batched", 320, [0, 4 * 8 + 5, 63], 2, local_solver="fista",
                   plan=dict(col_waves=2, row_waves=2, tile_order=2, tile_groups=4))


def test_large_workload_one_round_map_on_sampled_tiles():
    """8192 x 8192, 16 x 16 tiles of 512-576 px, 63 x 63 Moffat grid, frame 640."""
    _one_round_map("large", 640, [0, 16 * 8 + 9, 255], 2, plan=dict(tile_groups=4))


def test_combined_workload_one_round_map_on_sampled_tiles():
    """16384 x 16384, 32 x 32 tiles, 63 x 63 Moffat grid (1024 tiles in one batch)."""
    _one_round_map("combined", 640, [33 * 5, 1023], 1)


def test_large_workload_operator_on_sampled_tiles():
    """8192 x 8192, 16 x 16 tiles of 512-576 px, 63 x 63 Moffat grid, frame 640."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    w = workloads.WORKLOADS["large"]
    psfs = _f32(workloads.moffat_psf_grid(w.grid, w.psf_size, rotate=True))
    L = make_layout(w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    params = dl.make_params(w.M, w.tiles, w.pitch, w.overlap, w.grid, w.psf_size, lam=w.lam, reg_param=w.eps,
                            gamma=w.gamma, rho=w.rho)
    ctx = dl.Context(params, psfs)
    assert ctx.tiles[0].frame == 640
    rng = np.random.default_rng(5)
    x = rng.random(ctx.support_total, dtype=np.float32)
    s = rng.standard_normal(ctx.block_total, dtype=np.float32)
    hx = ctx.apply_H(torch.tensor(x, device="cuda")).cpu().numpy()
    hts = ctx.apply_Ht(torch.tensor(s, device="cuda")).cpu().numpy()
    F = op.FFTOperator(L, psfs, N=640)
    for t in [0, 7, 15, 16 * 8 + 9, 255]:
        d = ctx.tiles[t]
        xt = x[d.x_offset:d.x_offset + d.support_h * d.support_w].reshape(d.support_h, d.support_w)
        st = s[d.y_offset:d.y_offset + d.block_h * d.block_w].reshape(d.block_h, d.block_w)
        got_h = hx[d.y_offset:d.y_offset + d.block_h * d.block_w].reshape(d.block_h, d.block_w)
        got_t = hts[d.x_offset:d.x_offset + d.support_h * d.support_w].reshape(d.support_h, d.support_w)
        e1 = _rel(got_h, F.apply_H(t, xt.astype(np.float64)))
        e2 = _rel(got_t, F.apply_Ht(t, st.astype(np.float64)))
        print(f"tile {t} ({d.block_h}x{d.block_w}, K={d.n_terms}): H {e1:.2e} Ht {e2:.2e}")
        assert e1 <= 1e-5 and e2 <= 1e-5
    ctx.close()
