"""Benchmark of the frequency-Hough hot path on one MI355X.

One step = the whole hot path over one batch: for every sky direction of the
workload, Doppler correction, stripe edges, peak windows, the LDS histogram
tiles with their row sums and per-bin maxima, and sub-band candidate
selection (fh_hough_candidates, persistent schedule).  Inputs (peakmap and
weights) are resident in device memory before the timed region.

Prints one JSON line (metric: Hough cell-updates/s = input peaks x spin-down
rows x sky directions per second).

    python bench.py [--steps K] [--warmup W] [--workload batch-256hz] [--n-sky 1024]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# LDS atomic issue rate of gfx950: one wave64 ds_add_u32 every 4 clocks per
# CU (16 lanes/clk), 256 CUs, 2.4 GHz.  One cell update = one LDS atomic.
LDS_ATOMIC_PEAK_TOPS = 256 * 16 * 2.4e9 / 1e12
WORKLOAD_TEXT = {
    "batch-256hz": "batch-256hz: 1024 sky directions (Fibonacci grid), 1 Hz band at 256 Hz, "
                   "T_FFT 4096 s, 6300 FFTs, ~2.3M peaks, 583 spin-down rows [-1e-8, 1e-9] Hz/s, "
                   "40960 fine bins (K_f 10), FP32 adaptive weights, top-2 per 0.1 Hz sub-band",
    "sky-100hz": "sky-100hz: 1 Hz band at 100 Hz, T_FFT 8192 s, 3140 FFTs, ~2.0M peaks, 118 rows, "
                 "81920 fine bins",
    "large-1024hz": "large-1024hz: 10 Hz at 1024 Hz, T_FFT 1024 s, 25000 FFTs, ~20M peaks, 147 rows",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch-256hz")
    ap.add_argument("--n-sky", type=int, default=None)
    ap.add_argument("--plain-sky", type=int, default=64,
                    help="directions timed with the plain per-sky schedule")
    ap.add_argument("--unweighted", action="store_true")
    ap.add_argument("--tile-bins", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of one direction the CPU oracle computes (0 = auto)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB moved by one plain device copy before the timed steps "
                         "(reference dispatch for hardware byte counters)")
    return ap.parse_args()


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def cpu_baseline(w, rows_arg):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import oracle
    grid = w.grid
    rows = rows_arg or grid.ns
    # size the sample to roughly 10-30 s of CPU work
    t0 = time.perf_counter()
    oracle.hough_map(w.pm, grid, w.sky[0], weights=None if w.weights is None else w.weights.astype("float64"),
                     rows=(0, min(grid.ns, 8)))
    probe = time.perf_counter() - t0
    per_row = probe / min(grid.ns, 8)
    if not rows_arg:
        rows = int(max(8, min(grid.ns, 20.0 / max(per_row, 1e-6))))
    t0 = time.perf_counter()
    oracle.hough_map(w.pm, grid, w.sky[0], weights=None if w.weights is None else w.weights.astype("float64"),
                     rows=(0, rows))
    dt = time.perf_counter() - t0
    updates = w.pm.n_peaks * rows
    return {"value": updates / dt, "unit": "cell-updates/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "1 sky direction, spin-down rows 0..%d of %d, %d peaks (%.3g cell updates, %.1f s)"
                      % (rows - 1, grid.ns, w.pm.n_peaks, updates, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the frequency-Hough path on a "
              "single MI355X (no multi-GPU code path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1407_8333_amd import api, synth

    n_sky = args.n_sky or (1024 if args.workload == "batch-256hz" else
                           (4096 if args.workload == "large-1024hz" else 1))
    w = synth.workload(args.workload, n_sky=n_sky)
    if args.unweighted:
        w.weights = None
    grid, sel = w.grid, w.sel
    cells_per_sky = w.pm.n_peaks * grid.ns
    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    dpm = ctx.upload(w.pm)
    wt = None if w.weights is None else torch.as_tensor(w.weights, device=dev)
    out = torch.empty((n_sky, api.n_subbands(grid, sel), 2, 8), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        api.fh_hough_candidates(ctx, dpm, w.sky, grid, sel, weights=wt, schedule=1,
                                tile_bins=args.tile_bins, out=out)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()

    ctx.profile(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prof = ctx.profile_read()
    ctx.profile(False)
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    total_cells = cells_per_sky * n_sky * args.steps
    value = total_cells / wall

    # plain per-sky schedule on a subset of the same directions
    n_plain = min(args.plain_sky, n_sky)
    plain = None
    if n_plain > 0:
        api.fh_hough_candidates(ctx, dpm, w.sky[:n_plain], grid, sel,
                                weights=None if wt is None else wt, schedule=0,
                                tile_bins=args.tile_bins)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        api.fh_hough_candidates(ctx, dpm, w.sky[:n_plain], grid, sel,
                                weights=None if wt is None else wt, schedule=0,
                                tile_bins=args.tile_bins)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pp = ctx.profile_read()
        ctx.profile(False)
        plain = {"value": cells_per_sky * n_plain / dt, "n_sky": n_plain,
                 "ms_per_sky": dt * 1e3 / n_plain,
                 "tile_kernel_ms_per_launch": pp["tiles_ms"] / max(1, pp["tiles_launches"])}

    tiles_ms_avg = prof["tiles_ms"] / max(1, prof["tiles_launches"])
    cells_per_launch = prof["cell_updates"] / max(1, prof["tiles_launches"])
    achieved = cells_per_launch / (tiles_ms_avg * 1e-3) / 1e12
    plan = ctx.plan(dpm, grid, args.tile_bins)
    res = {
        "metric": "Hough cell-updates/s (peaks x spin-down bins) on 1 GPU",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if wt is not None else "u32 (unweighted counts)",
        "data": "synthetic (seeded Gaussian-noise peakmaps, theta 2.5 local maxima)",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "n_sky": n_sky, "n_fft": w.pm.n_fft, "n_peaks": w.pm.n_peaks,
                   "ns": grid.ns, "nf": grid.nf, "kf": grid.kf,
                   "weighted": wt is not None, "schedule": "persistent",
                   "tile": [plan["tile_rows"], plan["tile_bins"]]},
        "p50_ms_per_step": pct(step_ms, 50),
        "p99_ms_per_step": pct(step_ms, 99),
        "batched_vs_plain": None if plain is None else value / plain["value"],
        "plain": plain,
        "kernel_split_ms_per_step": {"tiles": prof["tiles_ms"] / args.steps,
                                     "front": prof["front_ms"] / args.steps,
                                     "select": prof["select_ms"] / args.steps},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": LDS_ATOMIC_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / LDS_ATOMIC_PEAK_TOPS,
                     "traffic": None,
                     "kernel": "k_tiles_persistent (one op = one ds_add_u32 cell update)",
                     "launch_ms": tiles_ms_avg, "cells_per_launch": cells_per_launch},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_rows)
    dpm.release()
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
