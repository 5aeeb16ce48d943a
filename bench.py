"""Benchmark of the batched tile solve on one MI355X.

One step = one full solve of the batched workload: 2048 x 2048 observed
image in 8 x 8 tiles (32-px overlap, uneven edge tiles), 8 x 8 grid of 31 x 31
Moffat PSFs, Poisson + read noise, smoothed TV, positivity, 200 Local-Solver
iterations (20 D-R rounds of 10), i.e. init -> 20 graph-captured rounds ->
output assembly.  Inputs (observation, weights, PSF spectra) are resident in
HBM before the timed region starts.

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
               "Local-Solver steps), one solve per step",
    "large": "large: 8192x8192 image, 16x16 tiles of 512-576 px (64-px overlap), 16x16 grid of 63x63 Moffat "
             "PSFs with field-dependent FWHM and rotation, Poisson+read noise, smoothed TV + positivity, 300 "
             "iterations (30 D-R rounds x 10 Local-Solver steps), one solve per step",
    "combined": "combined: 16384x16384 image, 32x32 tiles (64-px overlap), 32x32 grid of 63x63 Moffat PSFs, "
                "Poisson+read noise, smoothed TV + positivity, 300 iterations (30 D-R rounds x 10 "
                "Local-Solver steps), one solve per step",
}


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


def build_workload(name="batched", tune=True, plan=None):
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
        plan, trials = dl.autotune(params, psfs, n_inner=w.n_inner, reps=5)
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


def fista_context(ctx, psfs, y, W):
    """A second context on the same workload, observation and launch plan,
    with the FISTA Local-Solver."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    params = dl.Params.from_buffer_copy(ctx.params)
    params.local_solver = dl.SOLVER_FISTA
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
    of the given tiles in turn until the time budget is spent."""
    from oracle import solver
    from oracle.layout import make_layout
    from oracle.solver import Problem
    from threadpoolctl import threadpool_limits
    geom, prior, y, W, psfs, tiles, budget_s = job
    threadpool_limits(1)          # one thread per worker process
    L = make_layout(*geom)
    prob = Problem(L, psfs, y, W, **prior)
    x0 = solver.initial_tiles(prob, "observed")
    el, steps = 0.0, 0
    t_start = time.perf_counter()
    for t in itertools.cycle(tiles):   # the worker's tiles, again until the budget is spent
        tau = solver.step_size(prob, t)          # setup, not timed
        ts = time.perf_counter()
        solver.local_solve(prob, t, x0[t], x0[t], 1, tau)
        el += time.perf_counter() - ts
        steps += 1
        if time.perf_counter() - t_start > budget_s:
            break
    return steps, el


def baseline_procs():
    """Worker processes for the CPU baseline: the host CPUs this process may
    run on, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def start_baseline_pool(procs):
    """Fork the CPU baseline's workers.  Called before anything touches the
    GPU, so the children are plain copies of a host-only process; they sit idle
    until cpu_baseline hands them work."""
    import multiprocessing as mp
    return mp.get_context("fork").Pool(procs)


def cpu_baseline(pool, procs, psfs, y, W, w, budget_s=20.0):
    """The FP64 oracle (direct convolution) on a bounded sample of the same
    workload, on the host's cores: `procs` worker processes of one thread
    each, every one doing Local-Solver steps on its share of seeded sampled
    tiles for about budget_s seconds; the whole-image rate is the sum of the
    workers' rates, extrapolated by tile count."""
    from oracle.layout import make_layout

    geom = (w.M, w.tiles, w.pitch, w.overlap, w.psf_size, w.grid)
    L = make_layout(*geom)
    order = np.random.default_rng(12345).permutation(L.n_tiles)
    prior = dict(lam=w.lam, reg_param=w.eps, gamma=w.gamma, rho=w.rho)
    jobs = [(geom, prior, y, W, psfs, [int(t) for t in order[k::procs]], budget_s) for k in range(procs)]
    out = pool.map(_oracle_tile_steps, jobs, chunksize=1)
    steps = sum(n for n, _ in out)
    tile_steps_per_s = sum(n / el for n, el in out if n)
    rate = (w.M * w.M) * tile_steps_per_s / L.n_tiles / 1e6
    return {"value": rate, "unit": UNIT, "cores": procs, "kind": "oracle",
            "sample": f"1 Local-Solver step (H + H^T + TV gradient + projected update) of the fp64 "
                      f"direct-convolution oracle, {steps} tile-steps over {L.n_tiles} seeded-shuffled tiles, in {procs} "
                      f"single-threaded processes for ~{budget_s:.0f} s each; whole-image rate = sum of the "
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


def convergence(ctx, w, args, fctx=None):
    """Time and iterations to a D-R residual of 1e-4 from the plain start and
    from the network's warm start (with per-tile fallback), same GPU, same
    scene.  The network is trained first (untimed) on plain-solver pairs of
    fresh scenes (seeds 10000+), held out from the benchmark scene; the warm
    start then runs it on all tiles of the image in one launch per layer."""
    import torch
    from paper_1705_06603_amd import _lib as dl
    from paper_1705_06603_amd import train as tr
    N = ctx.tiles[0].frame
    scenes = args.train_scenes if args.train_scenes else (8 if ctx.n_tiles <= 64 else 2)
    t0 = time.perf_counter()
    tctx, _ = tr.workload_context(w)
    ins, outs = tr.make_pairs(tctx, w, seeds=range(10000, 10000 + scenes), crop=256,
                              crops_per_tile=1, n_outer=w.n_outer)
    tctx.close()
    n_pairs = int(ins.shape[0])
    trainer = dl.Net(16, 256, 256, seed=3)
    losses = tr.train(trainer, ins, outs, steps=args.train_steps, batch=16, lr=2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del ins, outs
    # inference network sized for every tile of the image at once
    net = dl.Net(ctx.n_tiles, N, N, params=trainer.get_params(), inference_only=True)
    trainer.close()
    out = {"tol": 1e-4, "n_inner": w.n_inner, "gamma": w.gamma,
           "training": {"pairs": n_pairs, "scenes": scenes, "crop": 256,
                        "steps": args.train_steps, "batch": 16, "loss_first": losses[0], "loss_last": losses[-1],
                        "seconds": round(train_s, 2)}}
    stream = torch.cuda.current_stream()
    # plain and warm start with the fixed schedule; plain start with the
    # paper's growing schedule (n_inner + n_inner k steps in round k); plain
    # start with the FISTA Local-Solver
    labels = ("plain", "warm", "plain_growing") + (("plain_fista",) if fctx is not None else ())
    for label in labels:
        growth = w.n_inner if label == "plain_growing" else 0
        c = fctx if label == "plain_fista" else ctx
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
    # network inference cost (all tiles in one batch) and MFMA utilisation of a 32 -> 32 layer
    frames, _ = ctx.warm_inputs()
    B = ctx.n_tiles
    ms_all, ms_mid = net.time_forward(frames, reps=10)
    flop_mid = 2.0 * 9 * 32 * 32 * B * N * N
    # the 32 -> 32 layer reads and writes one bf16 activation map of 32
    # channels: 144 flop per byte, below the bf16 MFMA / HBM balance of
    # 2500 / 8 = 312, so its roofline is the HBM one
    bytes_mid = 2.0 * 32 * 2 * B * N * N
    out["network"] = {"forward_ms_per_batch": round(ms_all, 3), "batch_tiles": B, "frame": N,
                      "mid_layer_ms": round(ms_mid, 4), "mid_layer_TFLOPs": round(flop_mid / (ms_mid * 1e-3) / 1e12, 1),
                      "mfma_bf16_peak_TFLOPs": 2500.0,
                      "mfma_utilisation": round(flop_mid / (ms_mid * 1e-3) / 2.5e15, 4),
                      "mid_layer_algorithmic_bytes": bytes_mid,
                      "mid_layer_GBps": round(bytes_mid / (ms_mid * 1e-3) / 1e9, 1),
                      "mid_layer_hbm_frac": round(bytes_mid / (ms_mid * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the context's default launch plan")
    ap.add_argument("--plan", default=None, help="fixed launch plan 'frame,col_waves,row_waves,order[,groups]' "
                                                 "(order: column_major | tile_major | heavy_first; groups 1 or 2)")
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOAD_TEXT),
                    help="batched is the headline configuration; the others are reported the same way")
    ap.add_argument("--max-rounds", type=int, default=1500)
    ap.add_argument("--train-scenes", type=int, default=0,
                    help="training scenes (0: 8 for up to 64 tiles, else 2)")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs all tiles on one GPU; --gpus must be 1"}))
        sys.exit(2)
    want_baseline = not (args.no_cpu_baseline or args.copy_calibration) and args.workload == "batched"
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

    print("# building workload", file=sys.stderr, flush=True)
    ctx, w, scene, psfs, y, W, trials = build_workload(args.workload, tune=not args.no_autotune,
                                                       plan=parse_plan(args.plan) if args.plan else None)
    n_outer, n_inner = w.n_outer, w.n_inner
    stream = torch.cuda.current_stream()

    def step():
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
    print("# timed", file=sys.stderr, flush=True)
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

    # Per-kernel launch durations (HIP events on the context stream).
    kms = ctx.time_kernels(reps=20)
    kb = tile_bytes(ctx)
    per_step_ms = {k: kms[k] * iters for k in KERNELS_PER_STEP}
    dom = max(per_step_ms, key=per_step_ms.get)
    achieved = kb[dom] / (kms[dom] * 1e-3) / 1e9
    traffic = measured_traffic(ctx, args.workload, dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "kernel_ms": round(kms[dom], 5),
                "algorithmic_bytes_per_launch": kb[dom],
                "all_kernels_ms": {k: round(v, 5) for k, v in kms.items()},
                "all_kernels_GBps": {k: round(kb[k] / (kms[k] * 1e-3) / 1e9, 1) for k in kms}}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "global_pixels": w.M * w.M, "iterations": iters, "tiles": ctx.n_tiles,
                   "fft_frame": ctx.tiles[0].frame, "parallelism": "single GPU, all tiles batched",
                   "plan": ctx.plan().as_dict()},
        "final_residual": res[-1] if res else None,
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    if trials:
        dflt = trials[0]   # the tuner measures a new context's own plan first
        best = min(trials, key=lambda t: t.us_per_iter)
        out["autotune"] = {"plans_measured": len(trials), "frames": sorted({t.frame for t in trials}),
                           "best": best.as_dict(), "default": dflt.as_dict(),
                           "worst_us_per_iter": round(max(t.us_per_iter for t in trials), 2)}
    if not args.no_convergence:
        # the FISTA Local-Solver on the same workload and plan: its step
        # throughput (same timed solve as above) and, below, its time to 1e-4
        print("# FISTA Local-Solver", file=sys.stderr, flush=True)
        fctx = fista_context(ctx, psfs, y, W)

        def fstep():
            fctx.init()
            fctx.run(n_outer, n_inner)
            fctx.assemble()

        fstep()
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(args.steps):
            fstep()
        f1.record(stream)
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / args.steps
        fk = fctx.time_kernels(reps=20)
        out["fista"] = {"ms_per_step": round(fms, 3),
                        "value": round((w.M * w.M) * iters / (fms * 1e-3) / 1e6, 2), "unit": UNIT,
                        "row_update_ms": round(fk["row_update"], 5)}
        print("# convergence: plain vs warm start vs FISTA", file=sys.stderr, flush=True)
        out["convergence"] = convergence(ctx, w, args, fctx)
        fctx.close()
    if pool is not None:
        print(f"# cpu baseline ({procs} processes)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pool, procs, psfs, y, W, w, args.cpu_budget)
        pool.close()
        pool.join()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
