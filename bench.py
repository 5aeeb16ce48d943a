"""Benchmark of the batched tile solve on one MI355X.

Default workload (the largest single-GPU configuration): 16384 x 16384
observed image in 32 x 32 tiles (64-px overlap), 32 x 32 grid of 63 x 63
Moffat PSFs, Poisson + read noise, smoothed TV, positivity.  One step = one
warm-started solve: the CNN warm start on all 1024 tiles (one launch per
layer) with the per-tile fallback judge, 20 graph-captured D-R rounds of 10
Local-Solver steps (200 iterations), output assembly.  Inputs (observation,
weights, PSF spectra, network weights) are resident in HBM before the timed
region starts.  `--workload batched|large` times the other configurations
(plain start) the same way.

The convergence section (time to residual 1e-4, warm start vs plain start)
runs on the 2048 x 2048 batched workload, where the warm-start network is
trained on converged plain-solver pairs of fresh scenes.

Prints one JSON line (see the keys below).  --gpus N > 1 is rejected: the
solver runs every tile of the image on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpixel-iterations/s of tile solve; time to 1e-4 residual, warm-start vs plain"
UNIT = "Mpixel-iterations/s"
KERNELS_PER_STEP = ("col_H", "row_resid", "col_Ht", "row_update")


def kernel_source_hash():
    """Hash of the frame kernels' code (fft_core.h + kernels.h) with comments
    and blank lines removed, so that recorded counters stay matched to the
    code they were taken on across comment-only edits."""
    import re
    h = hashlib.sha256()
    for f in ("fft_core.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1705_06603_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


WORKLOAD_TEXT = {
    "batched": "batched: 2048x2048 image, 8x8 tiles (32-px overlap, uneven edge tiles), 8x8 grid of 31x31 "
               "Moffat PSFs, Poisson+read noise, smoothed TV + positivity, 200 iterations (20 D-R rounds x 10 "
               "Local-Solver steps), plain start, one solve per step",
    "large": "large: 8192x8192 image, 16x16 tiles of 512-576 px (64-px overlap), 16x16 grid of 63x63 Moffat "
             "PSFs with field-dependent FWHM and rotation, Poisson+read noise, smoothed TV + positivity, 300 "
             "iterations (30 D-R rounds x 10 Local-Solver steps), plain start, one solve per step",
    "combined": "combined: 16384x16384 image, 32x32 tiles of 512 px + 64-px overlap, 32x32 grid of 63x63 Moffat "
                "PSFs, Poisson+read noise, smoothed TV + positivity; CNN warm start on all 1024 tiles (all "
                "four layers in one fused launch) with per-tile fallback, then 200 iterations (20 D-R rounds x 10 "
                "Local-Solver steps), one warm-started solve per step",
}

# Weights of the batched workload's warm-start network (written by the
# training entry point of paper_1705_06603_amd.train).
WARM_WEIGHTS = os.path.join(ROOT, "paper_1705_06603_amd", "weights", "warm_batched.npy")

# Workloads whose timed step starts from the network (the others from the
# plain observed start).
WARM_WORKLOADS = ("combined",)


def parse_plan(text):
    """'frame,col_waves,row_waves,order[,tile_groups]' with order a name or number."""
    from paper_1705_06603_amd import _lib as dl
    parts = text.split(",")
    f, cw, rw, order = parts[:4]
    names = {v: k for k, v in dl.ORDER_NAMES.items()}
    pl = dl.Plan()
    pl.frame, pl.col_waves, pl.row_waves = int(f), int(cw), int(rw)
    pl.tile_order = names[order] if order in names else int(order)
    pl.tile_groups = int(parts[4]) if len(parts) > 4 else 1
    return pl


def build_workload(name="batched", tune=True, plan=None, tune_reps=None):
    """Scene, PSFs and the noisy observation of a workload, on a context whose
    launch plan comes from the library's autotuner (or is given).

    The blur is applied by the HIP library itself (deblur_blur_global);
    noise and weights come from the seeded generators."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    from paper_1705_06603_amd import workloads

    w = workloads.WORKLOADS[name]
    scene, psfs = workloads.make_workload(w)
    params = dl.make_params(w.M, w.tiles, w.pitch, w.overlap, w.grid, w.psf_size,
                            lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)
    trials = []
    if plan is None and tune:
        # timed rounds per plan: fewer on the large images, where one round
        # already spans tens of milliseconds
        reps = tune_reps if tune_reps else (5 if w.M <= 2048 else 1)
        plan, trials = dl.autotune(params, psfs, n_inner=w.n_inner, reps=reps)
    if plan is not None:
        params.fft_size = plan.frame
    ctx = dl.Context(params, psfs)
    if plan is not None:
        ctx.set_plan(plan)
    x_dev = torch.tensor(scene.astype(np.float32), device="cuda")
    blurred = ctx.blur_global(x_dev).cpu().numpy().astype(np.float64)
    del x_dev
    y, W = workloads.observe(blurred, w.noise, w.seed)
    del blurred
    ctx.set_observation(torch.tensor(y.astype(np.float32), device="cuda"),
                        torch.tensor(W.astype(np.float32), device="cuda"))
    return ctx, w, scene, psfs, y, W, trials


def solver_context(ctx, psfs, y, W, local_solver):
    """A second context on the same workload, observation and launch plan,
    with another Local-Solver."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    params = dl.Params.from_buffer_copy(ctx.params)
    params.local_solver = local_solver
    params.fft_size = ctx.tiles[0].frame
    fctx = dl.Context(params, psfs)
    fctx.set_plan(ctx.plan())
    fctx.set_observation(torch.tensor(y.astype(np.float32), device="cuda"),
                         torch.tensor(W.astype(np.float32), device="cuda"))
    return fctx


def tile_bytes(ctx):
    """Compulsory bytes per launch of each kernel: every input read once,
    every output written once, each PSF node spectrum read once.

    With N the frame and HP = (N/2) N complex64 = 4 N^2 bytes a packed
    half-plane, per tile with K_x column masks:
      col_H      : (K_x + 1) HP               (Z_kx in, Yc out)
      row_resid  : 2 HP + 8 N^2               (Yc in, Rr out, (y, W) frame in)
      col_Ht     : (1 + K_x) HP               (Rr in, G_kx out)
      row_update : 2 K_x HP + 12 N^2          (G_kx in, Z_kx out, x and u in, x out)
      consensus  : 12 bytes per (tile, support pixel): x, u in, u out
    plus, for col_H and col_Ht, every PSF node spectrum once (HP each).
    """
    N = ctx.tiles[0].frame
    HP = 4 * N * N
    out = dict(col_H=0, row_resid=0, col_Ht=0, row_update=0, consensus=0)
    for d in ctx.tiles:
        kx = d.n_terms_x
        out["col_H"] += (kx + 1) * HP
        out["row_resid"] += 2 * HP + 8 * N * N
        out["col_Ht"] += (1 + kx) * HP
        out["row_update"] += 2 * kx * HP + 12 * N * N
        out["consensus"] += 12 * d.support_h * d.support_w
    nodes = ctx.params.G_y * ctx.params.G_x
    out["col_H"] += nodes * HP
    out["col_Ht"] += nodes * HP
    return out


def step_floor_bytes(ctx):
    """The method's algorithmic HBM floor of one inner iteration (one
    Local-Solver step on every tile): per support pixel, x, u, y and W read
    and x written (20 B), plus 8 B of PSF spectrum per term for H and for
    H^T (8 K_t B), summed over the tiles."""
    total = 0
    for d in ctx.tiles:
        total += (20 + 8 * d.n_terms_y * d.n_terms_x) * d.support_h * d.support_w
    return total


def kernel_variant(ctx, kernel):
    """Launch shape of one kernel family under the context's plan."""
    pl = ctx.plan()
    if kernel in ("col_H", "col_Ht"):
        return {"frame": pl.frame, "waves": pl.col_waves, "tile_order": pl.tile_order}
    if kernel == "consensus":
        return {"frame": pl.frame}
    return {"frame": pl.frame, "waves": pl.row_waves}


def measured_traffic(ctx, workload, kernel):
    """HBM bytes per launch of kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter summary (one entry per launch shape measured), if it
    was taken on the current kernel sources and the same launch shape; else
    None."""
    tfile = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.json")
    if not os.path.exists(tfile):
        return None
    with open(tfile) as fh:
        tj = json.load(fh)
    if tj.get("kernel_source_hash") != kernel_source_hash():
        return None
    entries = tj.get("kernels", {}).get(kernel) or []
    if isinstance(entries, dict):
        entries = [entries]
    want = kernel_variant(ctx, kernel)
    for k in entries:
        if k.get("variant") == want:
            return k.get("bytes_per_launch")
    return None


def _oracle_tile_steps(job):
    """Worker of cpu_baseline: one Local-Solver step of the FP64 oracle on each
    of the given tiles in turn until the time budget is spent.  The
    observation, weights and PSFs come from .npy files, memory-mapped, so a
    worker reads only its tiles' blocks."""
    from oracle import operator as op
    from oracle import solver
    from oracle.layout import make_layout
    from oracle.solver import Problem
    from threadpoolctl import threadpool_limits
    geom, prior, paths, backend, frame, tiles, budget_s = job
    threadpool_limits(1)          # one thread per worker process
    y, W, psfs = (np.load(p, mmap_mode="r") for p in paths)
    psfs = np.asarray(psfs, dtype=np.float64)
    L = make_layout(*geom)
    operator = op.FFTOperator(L, psfs, frame) if backend == "fft" else None
    prob = Problem(L, psfs, y, W, operator=operator, **prior)
    el, steps = 0.0, 0
    t_start = time.perf_counter()
    for t in itertools.cycle(tiles):   # the worker's tiles, again until the budget is spent
        x0 = solver.initial_tiles(prob, "observed", tiles=[t])[0]   # setup, not timed
        tau = solver.step_size(prob, t)                              # setup, not timed
        ts = time.perf_counter()
        solver.local_solve(prob, t, x0, x0, 1, tau)
        el += time.perf_counter() - ts
        steps += 1
        if time.perf_counter() - t_start > budget_s:
            break
    return steps, el


def baseline_procs():
    """Worker processes for the CPU baseline: the host CPUs this process may
    run on, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def start_baseline_pool(procs):
    """Fork the CPU baseline's workers.  Called before anything touches the
    GPU, so the children are plain copies of a host-only process; they sit idle
    until cpu_baseline hands them work."""
    import multiprocessing as mp
    return mp.get_context("fork").Pool(procs)


def cpu_baseline(pool, procs, psfs, y, W, w, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload, on the
    host's cores.  First one worker alone (the one-process rate), then
    `procs` worker processes of one thread each, every one doing Local-Solver
    steps on its share of seeded sampled tiles for about budget_s seconds;
    the whole-image rate is the sum of the workers' rates, extrapolated by
    tile count.  The oracle's operator is direct convolution; for the 63 x 63
    PSFs its FP64 FFT backend (pinned equal to direct convolution) is used,
    as one direct-convolution tile step there takes about a minute."""
    import shutil
    import tempfile

    import scipy.fft
    from oracle.layout import make_layout

    geom = (w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    L = make_layout(*geom)
    backend = "direct" if w.psf_size <= 31 else "fft"
    frame = scipy.fft.next_fast_len(max(max(L.support_shape(t)) for t in range(L.n_tiles)), real=True)
    order = np.random.default_rng(12345).permutation(L.n_tiles)
    prior = dict(lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)
    tmp = tempfile.mkdtemp(prefix="deblur_baseline_")
    try:
        paths = []
        for name, a in (("y", y), ("W", W), ("psfs", psfs)):
            paths.append(os.path.join(tmp, name + ".npy"))
            np.save(paths[-1], np.asarray(a, dtype=np.float32 if name != "psfs" else np.float64))
        one = pool.apply(_oracle_tile_steps, ((geom, prior, paths, backend, frame,
                                               [int(t) for t in order[:8]], budget_s / 2),))
        jobs = [(geom, prior, paths, backend, frame, [int(t) for t in order[k::procs]], budget_s)
                for k in range(procs)]
        out = pool.map(_oracle_tile_steps, jobs, chunksize=1)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    steps = sum(n for n, _ in out)
    tile_steps_per_s = sum(n / el for n, el in out if n)
    per_tile = (w.M * w.M) / L.n_tiles / 1e6
    rate = tile_steps_per_s * per_tile
    rate_one = (one[0] / one[1]) * per_tile if one[0] else None
    kind = ("fp64 direct-convolution oracle" if backend == "direct" else
            f"fp64 oracle with its FFT backend ({frame}x{frame} frames; the direct-convolution form is pinned "
            f"equal to it and takes about a minute per tile step at 63x63 PSFs)")
    return {"value": rate, "unit": UNIT, "cores": procs, "kind": "oracle",
            "one_process_value": rate_one, "cpu_model": cpu_model(),
            "sample": f"1 Local-Solver step (H + H^T + TV gradient + projected update) of the {kind}, "
                      f"{steps} tile-steps over {L.n_tiles} seeded-shuffled tiles of the same workload, in "
                      f"{procs} single-threaded processes for ~{budget_s:.0f} s each (after one process alone "
                      f"for ~{budget_s / 2:.0f} s: {one[0]} tile-steps); whole-image rate = sum of the "
                      f"processes' tile-step rates x (image pixels / tiles)"}


def run_to_tolerance(ctx, w, tol, max_rounds, label, chunk=100, growth=0):
    """D-R rounds until the residual reaches tol (checked every round), in
    chunks of `chunk` rounds with a progress line after each chunk.  With
    growth > 0, round k runs n_inner + growth * k Local-Solver steps."""
    res = []
    while len(res) < max_rounds:
        r = ctx.run(min(chunk, max_rounds - len(res)), w.n_inner, tol=tol, growth=growth, first_round=len(res))
        res += r
        print(f"# {label}: {len(res)} rounds, residual {res[-1]:.3e}", file=sys.stderr, flush=True)
        if res[-1] <= tol:
            break
    return res


def schedule_iterations(w, rounds, growth):
    """Local-Solver iterations in the first `rounds` rounds of a schedule."""
    return sum(w.n_inner + growth * k for k in range(rounds))


def train_network(w, args, scenes, tol, max_rounds, crops_per_tile, label):
    """A warm-start network trained (untimed) on plain-solver pairs of fresh
    scenes (seeds 10000+) of workload w: inputs are the warm-start inputs of a
    tile, targets its plain solution at residual tol."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    from paper_1705_06603_amd import train as tr
    t0 = time.perf_counter()
    tctx, _ = tr.workload_context(w)
    ins, outs = tr.make_pairs(tctx, w, seeds=range(10000, 10000 + scenes), crop=256,
                              crops_per_tile=crops_per_tile, tol=tol, max_rounds=max_rounds)
    tctx.close()
    n_pairs = int(ins.shape[0])
    trainer = dl.Net(16, 256, 256, seed=3)
    losses = tr.train(trainer, ins, outs, steps=args.train_steps, batch=16, lr=2e-3)
    torch.cuda.synchronize()
    del ins, outs
    info = {"workload": w.name, "pairs": n_pairs, "scenes": scenes, "crop": 256,
            "target": f"plain solve to residual {tol:g} (at most {max_rounds} rounds)",
            "steps": args.train_steps, "batch": 16, "loss_first": losses[0], "loss_last": losses[-1],
            "seconds": round(time.perf_counter() - t0, 2)}
    print(f"# {label}: network trained on {n_pairs} pairs in {info['seconds']} s", file=sys.stderr, flush=True)
    return trainer, info


def warm_network(ctx, w, args):
    """The network of the warm-started workload: trained on a 4096 x 4096
    image of the same PSF model and tiling (8 x 8 tiles of 512 px + 64,
    8 x 8 Moffat grid of 63 x 63), then copied into an inference network
    sized for every tile of the image at once."""
    import dataclasses
    from paper_1705_06603_amd import _lib as dl
    tw = dataclasses.replace(w, name=w.name + "-train", M=4096, tiles=8, grid=8)
    trainer, info = train_network(tw, args, scenes=args.train_scenes or 4, tol=1e-3, max_rounds=600,
                                  crops_per_tile=4, label="warm start")
    N = ctx.tiles[0].frame
    net = dl.Net(ctx.n_tiles, N, N, params=trainer.get_params(), inference_only=True)
    trainer.close()
    return net, info


def network_cost(ctx, net):
    """Forward time of the network on every tile of ctx at once, and its MFMA
    utilisation: the network's algorithmic flops (38,016 per pixel: layers
    1 and 4 on the VALU, 2 and 3 on bf16 MFMA) over the launch time, against
    the dense bf16 MFMA peak.  An inference-only network runs the fused
    kernel (one launch, activations in LDS); a trainable one runs layer by
    layer, and then the 32 -> 32 layer alone is reported too."""
    N = ctx.tiles[0].frame
    frames, _ = ctx.warm_inputs()
    B = ctx.n_tiles
    ms_all, ms_mid = net.time_forward(frames, reps=5)
    flop_all = 38016.0 * B * N * N
    out = {"forward_ms_per_batch": round(ms_all, 3), "batch_tiles": B, "frame": N, "fused": ms_mid == 0.0,
           "forward_TFLOPs": round(flop_all / (ms_all * 1e-3) / 1e12, 1), "mfma_bf16_peak_TFLOPs": 2500.0,
           "mfma_utilisation": round(flop_all / (ms_all * 1e-3) / 2.5e15, 4),
           "activation_hbm_bytes": 0 if ms_mid == 0.0 else 3 * 2 * 64.0 * B * N * N}
    if ms_mid > 0.0:
        flop_mid = 2.0 * 9 * 32 * 32 * B * N * N
        # the 32 -> 32 layer reads and writes one bf16 activation map of 32
        # channels: 144 flop per byte, below the bf16 MFMA / HBM balance of
        # 2500 / 8 = 312, so its roofline is the HBM one
        bytes_mid = 2.0 * 32 * 2 * B * N * N
        out.update({"mid_layer_ms": round(ms_mid, 4),
                    "mid_layer_TFLOPs": round(flop_mid / (ms_mid * 1e-3) / 1e12, 1),
                    "mid_layer_mfma_utilisation": round(flop_mid / (ms_mid * 1e-3) / 2.5e15, 4),
                    "mid_layer_algorithmic_bytes": bytes_mid,
                    "mid_layer_GBps": round(bytes_mid / (ms_mid * 1e-3) / 1e9, 1),
                    "mid_layer_hbm_frac": round(bytes_mid / (ms_mid * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    return out


def timed_solves(ctx, w, steps, net=None):
    """ms per solve of `steps` back-to-back solves (init or warm start,
    n_outer graph-captured rounds, assembly) between HIP events on the
    context stream."""
    import torch
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    res = None
    for _ in range(steps):
        if net is not None:
            ctx.init_cnn(net)
        else:
            ctx.init()
        res = ctx.run(w.n_outer, w.n_inner)
        ctx.assemble()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, res


# The lambda sweep of Section IV on a natural-image stand-in: a dead-leaves
# scene with the batched workload's geometry (2048^2, 8 x 8 tiles of pitch
# 256, 32-px overlap), an 8 x 8 grid of 31 x 31 elliptical Gaussian PSFs
# growing radially from FWHM 3.5 px to 8.5 x 6.5 px (the milder of the
# paper's two shift-variant grids), white Gaussian noise of variance 400 on
# a 6000-photon peak (sigma = 1/300 on the unit-peak scene), the Huber prior
# on circular differences with delta = 100 photons (1/60).  In these units
# the paper's lambda (photon scale, W = 1/400) is lambda / 400.
QUALITY = dict(M=2048, tiles=8, pitch=256, overlap=32, grid=8, psf=31, sigma=1.0 / 300.0, delta=1.0 / 60.0,
               gamma=4.0, seed=4, tol=1e-4, max_rounds=400)


def quality_sweep(plan, lams_paper=(1.5625e-5, 3.125e-5, 6.25e-5, 1.25e-4, 2.5e-4, 5e-4, 1e-3),
                  overlaps=(0, 16, 32, 64)):
    """Image quality against the ground truth over a range of lambda, for
    the proposed method and the independent baseline (no consensus, tiles
    blended with omega), as Section IV compares them, then over the block
    overlap at the proposed method's best lambda (the paper's SNR/SSIM vs
    overlap plots).  Each solve runs D-R rounds of 10 Local-Solver steps
    until the residual reaches 1e-4 (at most 400 rounds); SNR and SSIM of
    the observed crop of x_hat against the scene."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    from paper_1705_06603_amd import quality, workloads
    q = QUALITY
    M, r = q["M"], q["psf"] // 2
    scene = workloads.dead_leaves((M + 2 * r, M + 2 * r), q["seed"])
    psfs = workloads.gaussian_psf_grid_radial(q["grid"], q["psf"])

    def params(lam, independent, overlap=q["overlap"]):
        p = dl.make_params(M, q["tiles"], q["pitch"], overlap, q["grid"], q["psf"], reg=dl.REG_HUBER,
                           bc=dl.BC_CIRCULAR, lam=lam, reg_param=q["delta"], gamma=q["gamma"],
                           independent=independent)
        if overlap == q["overlap"]:
            p.fft_size = plan.frame
        return p

    c = dl.Context(params(1e-3, False), psfs)
    blurred = c.blur_global(torch.tensor(scene.astype(np.float32), device="cuda")).cpu().numpy()
    c.close()
    y, W = workloads.observe(blurred.astype(np.float64), "gaussian", q["seed"], sigma=q["sigma"])
    truth = scene[r:r + M, r:r + M]
    yd = torch.tensor(y.astype(np.float32), device="cuda")
    Wd = torch.tensor(W.astype(np.float32), device="cuda")

    def solve(lam, independent, overlap=q["overlap"]):
        c = dl.Context(params(lam, independent, overlap), psfs)
        if overlap == q["overlap"]:
            c.set_plan(plan)
        c.set_observation(yd, Wd)
        c.init()
        res = []
        while len(res) < q["max_rounds"]:
            res += c.run(min(100, q["max_rounds"] - len(res)), 10, tol=q["tol"])
            if res[-1] <= q["tol"]:
                break
        xh = c.assemble().cpu().numpy()[r:r + M, r:r + M]
        c.close()
        return {"snr_db": round(quality.snr_db(xh, truth), 4), "ssim": round(quality.ssim(xh, truth), 4),
                "rounds": len(res), "residual": res[-1]}

    out = {"scene": "dead leaves (r^-3 disk radii 2-160 px, grey levels U(0.05, 1)), seed %d" % q["seed"],
           "psfs": "8 x 8 elliptical Gaussians 31 x 31, FWHM 3.5 -> 8.5 x 6.5 px radially",
           "noise": "Gaussian, sigma = 1/300 of the peak (variance 400 at 6000 photons), W = 1",
           "prior": "Huber, delta = 1/60 of the peak (100 photons), circular differences",
           "stop": "residual <= %g or %d D-R rounds of 10 steps" % (q["tol"], q["max_rounds"]),
           "metric_region": "observed crop, against the scene",
           "observed": {"snr_db": round(quality.snr_db(y, truth), 4), "ssim": round(quality.ssim(y, truth), 4)},
           "lambda_paper_units": list(lams_paper), "lambda": [400.0 * l for l in lams_paper],
           "proposed": [], "independent": []}
    for lp in lams_paper:
        for label, ind in (("proposed", False), ("independent", True)):
            out[label].append(solve(400.0 * lp, ind))
    for label in ("proposed", "independent"):
        b = max(range(len(lams_paper)), key=lambda i: out[label][i]["snr_db"])
        out["best_" + label] = dict(out[label][b], lambda_paper_units=lams_paper[b])
    lp = out["best_proposed"]["lambda_paper_units"]
    out["overlap_sweep"] = {"lambda_paper_units": lp, "overlap": list(overlaps),
                            "proposed": [solve(400.0 * lp, False, o) for o in overlaps],
                            "independent": [solve(400.0 * lp, True, o) for o in overlaps]}
    print("# quality sweep done", file=sys.stderr, flush=True)
    return out


def convergence(args):
    """On the batched workload (2048 x 2048): time and iterations to a D-R
    residual of 1e-4 from the plain start, from the network's warm start
    (with per-tile fallback), with the growing schedule, with the FISTA
    Local-Solver and with the VMLM-B Local-Solver (fixed and growing
    schedule, the latter the paper's own configuration); plus the FISTA and
    VMLM-B solve throughput.  The network is trained first (untimed) on
    converged plain-solver pairs (residual 1e-4) of fresh scenes (seeds
    10000+), held out from the benchmark scene (seed 2)."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    print("# convergence: batched workload", file=sys.stderr, flush=True)
    ctx, w, scene, psfs, y, W, _ = build_workload("batched", tune=not args.no_autotune)
    N = ctx.tiles[0].frame
    if os.path.exists(WARM_WEIGHTS) and not args.train_in_bench:
        # the network of the batched workload's configuration: trained by
        # `python -m paper_1705_06603_amd.train` on 20,032 converged pairs
        params = np.load(WARM_WEIGHTS, allow_pickle=False)
        with open(WARM_WEIGHTS + ".json") as fh:
            info = dict(json.load(fh), weights=os.path.relpath(WARM_WEIGHTS, ROOT))
        net = dl.Net(ctx.n_tiles, N, N, params=params, inference_only=True)
    else:
        trainer, info = train_network(w, args, scenes=args.train_scenes or 8, tol=1e-4, max_rounds=2000,
                                      crops_per_tile=1, label="convergence")
        net = dl.Net(ctx.n_tiles, N, N, params=trainer.get_params(), inference_only=True)
        trainer.close()
    out = {"workload": WORKLOAD_TEXT["batched"], "tol": 1e-4, "n_inner": w.n_inner, "gamma": w.gamma,
           "plan": ctx.plan().as_dict(), "training": info}
    fctx = solver_context(ctx, psfs, y, W, dl.SOLVER_FISTA)
    vctx = solver_context(ctx, psfs, y, W, dl.SOLVER_VMLMB)
    iters = w.n_outer * w.n_inner
    pms, _ = timed_solves(ctx, w, 1)
    pms, _ = timed_solves(ctx, w, 20)
    timed_solves(fctx, w, 1)
    fms, _ = timed_solves(fctx, w, 20)
    fk = fctx.time_kernels(reps=20)
    out["fista_throughput"] = {"ms_per_solve": round(fms, 3),
                               "value": round((w.M * w.M) * iters / (fms * 1e-3) / 1e6, 2),
                               "plain_ms_per_solve": round(pms, 3),
                               "plain_value": round((w.M * w.M) * iters / (pms * 1e-3) / 1e6, 2),
                               "unit": UNIT, "row_update_ms": round(fk["row_update"], 5)}
    timed_solves(vctx, w, 1)
    vms, _ = timed_solves(vctx, w, 5)
    out["vmlmb_throughput"] = {"ms_per_solve": round(vms, 3),
                               "value": round((w.M * w.M) * iters / (vms * 1e-3) / 1e6, 2), "unit": UNIT,
                               "note": "eager launches, one 4-byte readback per line-search trial"}
    stream = torch.cuda.current_stream()
    growing = ("plain_growing", "vmlmb_growing")
    for label in ("plain", "warm", "plain_growing", "plain_fista", "plain_vmlmb", "vmlmb_growing"):
        growth = w.n_inner if label in growing else 0
        c = fctx if label == "plain_fista" else vctx if "vmlmb" in label else ctx
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if label == "warm":
            _, nf = ctx.init_cnn(net)
        else:
            c.init()
            nf = None
        res = run_to_tolerance(c, w, 1e-4, args.max_rounds if not growth else 60, label,
                               chunk=100 if not growth else 5, growth=growth)
        e1.record(stream)
        torch.cuda.synchronize()
        reached = res[-1] <= 1e-4
        first = lambda th: next((schedule_iterations(w, i + 1, growth) for i, r in enumerate(res) if r <= th), None)
        out[label] = {"reached": bool(reached),
                      "iterations": schedule_iterations(w, len(res), growth) if reached else None,
                      "ms": round(e0.elapsed_time(e1), 2) if reached else None,
                      "ms_run": round(e0.elapsed_time(e1), 2), "rounds_run": len(res),
                      "final_residual": res[-1], "iterations_to_1e-3": first(1e-3),
                      "iterations_to_1e-2": first(1e-2)}
        if label == "warm":
            out[label]["fallback_tiles"] = nf
    out["network"] = network_cost(ctx, net)
    net.close()
    fctx.close()
    vctx.close()
    out["quality_sweep"] = quality_sweep(ctx.plan())
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=16.0)
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the context's default launch plan")
    ap.add_argument("--plan", default=None, help="fixed launch plan 'frame,col_waves,row_waves,order[,groups]' "
                                                 "(order: column_major | tile_major | heavy_first; groups 1, 2 or 4)")
    ap.add_argument("--workload", default="combined", choices=sorted(WORKLOAD_TEXT),
                    help="combined (16384^2, warm-started) is the headline configuration; the others are "
                         "reported the same way from the plain start")
    ap.add_argument("--plain-start", action="store_true", help="time the combined workload from the plain start")
    ap.add_argument("--max-rounds", type=int, default=1500)
    ap.add_argument("--train-scenes", type=int, default=0,
                    help="training scenes (0: 8 for the convergence network, 4 for the warm-start network)")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--train-in-bench", action="store_true",
                    help="train the batched workload's network here instead of loading its stored weights")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs all tiles on one GPU; --gpus must be 1"}))
        sys.exit(2)
    want_baseline = not (args.no_cpu_baseline or args.copy_calibration)
    procs = baseline_procs()
    pool = start_baseline_pool(procs) if want_baseline else None

    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_direction": a.numel() * 4}))
        return

    print(f"# building workload {args.workload}", file=sys.stderr, flush=True)
    ctx, w, scene, psfs, y, W, trials = build_workload(args.workload, tune=not args.no_autotune,
                                                       plan=parse_plan(args.plan) if args.plan else None)
    del scene
    n_outer, n_inner = w.n_outer, w.n_inner
    warm = args.workload in WARM_WORKLOADS and not args.plain_start
    net, net_info = warm_network(ctx, w, args) if warm else (None, None)
    stream = torch.cuda.current_stream()
    nf_last = []

    def step():
        if warm:
            _, nf = ctx.init_cnn(net)
            nf_last[:] = [nf]
        else:
            ctx.init()
        res = ctx.run(n_outer, n_inner)
        ctx.assemble()
        return res

    print("# warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    print(f"# timed: {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    e0.record(stream)
    res = None
    for _ in range(args.steps):
        res = step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    iters = n_outer * n_inner
    value = (w.M * w.M) * iters * args.steps / (ms_total * 1e-3) / 1e6
    print(f"# timed: {ms_per_step:.2f} ms per step, {value:.1f} {UNIT}", file=sys.stderr, flush=True)

    # Per-kernel launch durations (HIP events on the context stream, every
    # launch covering all tiles) and the HBM roofline of the inner iteration:
    # the method's algorithmic floor per iteration over the four frame
    # kernels' summed launch time.
    kms = ctx.time_kernels(reps=20 if w.M <= 2048 else 5)
    kb = tile_bytes(ctx)
    step_ms = sum(kms[k] for k in KERNELS_PER_STEP)
    floor = step_floor_bytes(ctx)
    achieved = floor / (step_ms * 1e-3) / 1e9
    counters = [measured_traffic(ctx, args.workload, k) for k in KERNELS_PER_STEP]
    traffic = sum(counters) if all(c is not None for c in counters) else None
    dom = max(KERNELS_PER_STEP, key=lambda k: kms[k])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "inner iteration: " + " + ".join(KERNELS_PER_STEP),
                "kernel_ms": round(step_ms, 5), "algorithmic_bytes_per_launch": floor,
                "algorithmic_bytes_rule": "sum over tiles of (20 + 8 K_t) B per support pixel",
                "frac_from_ms_per_step": round(floor * iters / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "dominant_kernel": {"name": dom, "ms": round(kms[dom], 5), "design_bytes": kb[dom],
                                    "design_GBps": round(kb[dom] / (kms[dom] * 1e-3) / 1e9, 1),
                                    "design_frac": round(kb[dom] / (kms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                    "traffic": counters[KERNELS_PER_STEP.index(dom)]},
                "all_kernels_ms": {k: round(v, 5) for k, v in kms.items()},
                "all_kernels_design_GBps": {k: round(kb[k] / (kms[k] * 1e-3) / 1e9, 1) for k in kms}}
    if traffic is not None:
        # the HBM bytes the counters saw, over the same kernel time: how busy
        # HBM is, beside the algorithmic rate above
        roofline["traffic_GBps"] = round(traffic / (step_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        roofline["all_kernels_traffic_GBps"] = {k: round(c / (kms[k] * 1e-3) / 1e9, 1)
                                                for k, c in zip(KERNELS_PER_STEP, counters)}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload] if warm or args.workload != "combined"
                   else WORKLOAD_TEXT[args.workload].replace("CNN warm start on all 1024 tiles (one launch per "
                                                             "layer) with per-tile fallback, then ", "plain start, "),
                   "global_pixels": w.M * w.M, "iterations": iters, "tiles": ctx.n_tiles,
                   "fft_frame": ctx.tiles[0].frame, "parallelism": "single GPU, all tiles batched",
                   "plan": ctx.plan().as_dict()},
        "final_residual": res[-1] if res else None,
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    if warm:
        out["warm_start"] = {"fallback_tiles": nf_last[0] if nf_last else None, "training": net_info,
                             "network": network_cost(ctx, net)}
        net.close()
    if trials:
        dflt = trials[0]   # the tuner measures a new context's own plan first
        best = min(trials, key=lambda t: t.us_per_iter)
        out["autotune"] = {"plans_measured": len(trials), "frames": sorted({t.frame for t in trials}),
                           "best": best.as_dict(), "default": dflt.as_dict(),
                           "worst_us_per_iter": round(max(t.us_per_iter for t in trials), 2)}
    ctx.close()
    torch.cuda.empty_cache()
    if not args.no_convergence:
        out["convergence"] = convergence(args)
    if pool is not None:
        print(f"# cpu baseline ({procs} processes)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pool, procs, psfs, y, W, w, args.cpu_budget)
        pool.close()
        pool.join()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
