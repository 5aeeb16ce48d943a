"""Final-image parity at the batched workload's full size: 2048 x 2048
observed pixels in 8 x 8 tiles (32-px overlap, uneven edge tiles), 8 x 8 grid
of 31 x 31 Moffat PSFs, Poisson + read noise, smoothed TV with positivity,
200 iterations (20 D-R rounds of 10 Local-Solver steps), in the launch
configuration the benchmark times (autotuned plan, graph-captured rounds).

The plain-start solve and a warm-started solve (network start with the
per-tile fallback judge, then the same rounds) each run on the GPU and in the
FP64 oracle, whose per-tile work runs on the host's cores through its FFT
backend (pinned equal to direct convolution on these tile shapes in
tests/test_oracle_fullsize.py).  The final images x_hat = sum_t omega_t x_t
must agree to 1e-4 relative L2, the residual histories to 1e-3 relative.

The observation is made by the oracle: the workload's scene blurred tile by
tile with the oracle's operator (the tile operator is the exact restriction
of the global one, so overlapping blocks agree), then the workload's seeded
noise and weights."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import solver, warm
from oracle.layout import make_layout
from oracle.solver import Problem
from paper_1705_06603_amd import workloads
from tests._oracle_pool import OraclePool
from tests._problems import sharpening_network

pytestmark = pytest.mark.gpu

FRAME = 320


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def batched():
    print("final-image parity: building the batched workload (oracle blur)", flush=True)
    w = workloads.WORKLOADS["batched"]
    scene, psfs = workloads.make_workload(w)
    psfs = _f32(psfs)                      # the library holds the PSFs in fp32
    geom = (w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    L = make_layout(*geom)
    F = op.FFTOperator(L, psfs, FRAME)
    blurred = np.zeros((w.M, w.M))
    for t in range(L.n_tiles):
        (y0, y1), (x0, x1) = L.block(t)
        blurred[y0:y1, x0:x1] = F.apply_H(t, L.restrict(scene, t))
    y, W = workloads.observe(blurred, w.noise, w.seed)
    y, W = _f32(y), _f32(W)
    prior = dict(lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)
    prob = Problem(L, psfs, y, W, operator=F, **prior)
    pool = OraclePool(geom, psfs, y, W, prior, frame=FRAME)
    yield w, prob, pool
    pool.close()


def _gpu_context(w, prob):
    """A context as the benchmark builds it: autotuned launch plan, the
    workload's prior, the observation in HBM."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    params = dl.make_params(w.M, w.tiles, w.pitch, w.overlap, w.grid, w.psf_size,
                            lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)
    plan, _ = dl.autotune(params, prob.psfs, n_inner=w.n_inner, reps=5)
    params.fft_size = plan.frame
    ctx = dl.Context(params, prob.psfs)
    ctx.set_plan(plan)
    ctx.set_observation(torch.tensor(prob.y, dtype=torch.float32, device="cuda").contiguous(),
                        torch.tensor(prob.W, dtype=torch.float32, device="cuda").contiguous())
    return ctx, plan


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_plain_solve_final_image_matches_oracle(batched):
    w, prob, pool = batched
    ctx, plan = _gpu_context(w, prob)
    print(f"final-image parity, plain start: GPU solve under plan {plan.as_dict()}", flush=True)
    ctx.init()
    res = ctx.run(w.n_outer, w.n_inner)
    xh = ctx.assemble().cpu().numpy()
    ctx.close()
    print("final-image parity, plain start: oracle solve on the host", flush=True)
    ref = solver.solve(prob, w.n_outer, w.n_inner, tile_map=pool.local)
    err = _rel(xh, ref.x_hat)
    print(f"plain start: final image rel L2 {err:.3e}; residual {res[-1]:.4e} (oracle {ref.residuals[-1]:.4e})")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)


def test_warm_started_solve_final_image_matches_oracle(batched):
    """The network has bf16-exact weights (x - relu(Lap x) / 4: it softens
    the peaks of the noise and is kept on every tile by the judge), so the
    GPU's and the oracle's network starts agree to about fp32 rounding; each
    side then takes its own per-tile decisions and runs its own 200
    iterations."""
    from paper_1705_06603_amd import _lib as dl
    from oracle import cnn
    w, prob, pool = batched
    params = sharpening_network(kappa=-0.25, theta=0.0)
    print("final-image parity, warm start: oracle network starts and judge", flush=True)
    starts, keep, maps = warm.warm_start(prob, params, bf16=True, tile_map=pool.network)
    # no decision within fp32 noise of the threshold: both sides then decide alike
    for t, (a, b) in enumerate(maps):
        assert abs(a / b - (1 - warm.MARGIN)) > 1e-4, (t, a, b)
    ctx, plan = _gpu_context(w, prob)
    N = ctx.tiles[0].frame
    net = dl.Net(ctx.n_tiles, N, N, params=cnn.flatten(params).astype(np.float32), inference_only=True)
    use, nf = ctx.init_cnn(net)
    print(f"warm start: {int(use.sum())}/{len(use)} tiles keep the network start (oracle {sum(keep)})",
          flush=True)
    assert [bool(k) for k in use] == keep
    x0 = ctx.unpack_support(ctx.get_state()[0].cpu().numpy())
    start_err = max(_rel(x0[t], starts[t]) for t in range(ctx.n_tiles))
    # fp32 against fp64 sums can round a few bf16 activations apart at the
    # brightest stars: the starts agree to ~2e-5, well inside the network's
    # own tolerance
    assert start_err <= 1e-4, start_err
    res = ctx.run(w.n_outer, w.n_inner)
    xh = ctx.assemble().cpu().numpy()
    net.close()
    ctx.close()
    print("final-image parity, warm start: oracle solve on the host", flush=True)
    ref = solver.solve(prob, w.n_outer, w.n_inner, x0=starts, tile_map=pool.local)
    err = _rel(xh, ref.x_hat)
    print(f"warm start: starts rel L2 <= {start_err:.2e}; final image rel L2 {err:.3e}; "
          f"residual {res[-1]:.4e} (oracle {ref.residuals[-1]:.4e})")
    assert err <= 1e-4
    assert np.allclose(res, ref.residuals, rtol=1e-3, atol=0)
