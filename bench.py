"""Benchmark of the frequency-Hough hot path on one MI355X.

One step = the whole hot path over one batch: for every sky direction of the
workload, Doppler correction, stripe edges, peak windows, the LDS histogram
tiles with their row sums and per-bin maxima, and sub-band candidate
selection (fh_hough_candidates, persistent schedule, all directions in one
persistent tile launch, replayed as one captured hipGraph on its own
stream).  Inputs (peakmap and weights) are resident in device memory before
the timed region.

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
# The live probe (libfh_probe.so) measures what a CU sustains.
LDS_ATOMIC_PEAK_TOPS = 256 * 16 * 2.4e9 / 1e12
PROBE_LIB = os.path.join(ROOT, "paper_1407_8333_amd", "libfh_probe.so")
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch-256hz")
    ap.add_argument("--n-sky", type=int, default=None)
    ap.add_argument("--plain-sky", type=int, default=64,
                    help="directions timed with the plain per-sky schedule")
    ap.add_argument("--unweighted", action="store_true")
    ap.add_argument("--tile-bins", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of one direction the CPU oracle computes (0 = auto)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream (for device traces of the lanes)")
    ap.add_argument("--serve-lanes", type=int, default=8)
    ap.add_argument("--overlap-from", default=None,
                    help="print the stream overlap of a rocprofv3 kernel_trace.csv and exit")
    ap.add_argument("--overlap-skip", nargs="*", default=[],
                    help="stream ids left out of --overlap-from (e.g. the input-building stream)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the Poisson serving run (0 disables it)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured serving capacity")
    ap.add_argument("--doppler", default="exact", choices=["exact", "shift"],
                    help="Doppler correction: exact per peak (default) or one shift per FFT")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of hipGraph replays")
    ap.add_argument("--sky-chunk", type=int, default=0,
                    help="directions per persistent launch (0 = library choice: all 1024 in one)")
    ap.add_argument("--variant-steps", type=int, default=3,
                    help="steps timed for each eager / 4-launch variant (0 disables them)")
    ap.add_argument("--large-sky", type=int, default=4096,
                    help="directions of the large-band leg (0 disables it)")
    ap.add_argument("--no-probe", action="store_true", help="skip the LDS-atomic probe")
    ap.add_argument("--shape-sky", type=int, default=128,
                    help="directions per serving shape timed alone (0 disables the per-shape leg)")
    ap.add_argument("--shapes-only", nargs="*", default=None,
                    help="time only the given serving shapes, e.g. 1024:narrow 8192:wide (none = all)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB moved by one plain device copy before the timed steps "
                         "(reference dispatch for hardware byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_tiles_persistent_batch256hz_hbm_bytes.txt")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1407_8333_amd", "csrc",
                             "fh_kernels.hip")


SQ_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                       "k_tiles_persistent_batch256hz_sq_counters.txt")
# VALU issue rate of one CU: 4 SIMDs, each retiring one wave64 VALU
# instruction every 4 clocks, at 2.4 GHz; in wave-instructions per second
VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def committed_field(path, key, workload, n_sky, tile_bins, weighted):
    """A `key = value` figure of a committed rocprofv3 summary, when it was
    taken on this workload and on the current kernel source; None otherwise."""
    import hashlib
    if not (workload == "batch-256hz" and n_sky == 1024 and tile_bins == 2496 and weighted):
        return None
    try:
        fields = {}
        for line in open(path):
            if " = " in line:
                k, v = line.split(" = ", 1)
                fields[k.strip()] = v.strip()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256") != src:
            return None
        return float(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def committed_traffic(workload, n_sky, tile_bins, weighted):
    """HBM bytes per tile launch from the committed byte counters."""
    return committed_field(TRAFFIC_FILE, "traffic_bytes_per_launch", workload, n_sky, tile_bins, weighted)


def valu_cobound(achieved, workload, n_sky, tile_bins, weighted):
    """The tile kernel's VALU co-bound in cell updates/s: the chip's VALU
    issue rate divided by the VALU instructions per cell update (SQ counters
    of the same kernel source)."""
    r = committed_field(SQ_FILE, "valu_instr_per_cell_update", workload, n_sky, tile_bins, weighted)
    if r is None:
        return None
    peak = VALU_WAVE_INSTR_PER_S / r / 1e12
    return {"peak": peak, "unit": "TOP/s", "frac": achieved / peak, "valu_instr_per_cell_update": r}


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def cpu_baseline(w, rows_arg, target_s=20.0):
    """The oracle as it stands, on a bounded sample of the same workload: the
    full map and sub-band candidates of as many sky directions as fit in
    about `target_s` seconds (a slice of the spin-down rows of one direction
    if even one direction takes longer)."""
    import oracle
    grid, sel = w.grid, w.sel
    wts = None if w.weights is None else w.weights
    n_sky_all = len(w.sky)

    def one(k, rows):
        wk = None if wts is None else (wts if wts.ndim == 1 else wts[k]).astype("float64")
        m = oracle.hough_map(w.pm, grid, w.sky[k], weights=wk, rows=(0, rows))
        if rows == grid.ns:
            oracle.candidates(m, sel.width, sel.excl, sel.sep)

    rows = rows_arg or grid.ns
    t0 = time.perf_counter()
    one(0, rows)
    probe = time.perf_counter() - t0
    if not rows_arg and probe > target_s:
        rows = int(max(8, grid.ns * target_s / probe))
    n = 1
    if rows == grid.ns:
        n = int(max(1, min(n_sky_all, round(target_s / max(probe, 1e-6)))))
    t0 = time.perf_counter()
    for k in range(n):
        one(k, rows)
    dt = time.perf_counter() - t0
    updates = w.pm.n_peaks * rows * n
    what = ("%d sky directions, all %d spin-down rows, map + candidates" % (n, grid.ns) if rows == grid.ns
            else "1 sky direction, spin-down rows 0..%d of %d, map only" % (rows - 1, grid.ns))
    return {"value": updates / dt, "unit": "cell-updates/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "%s, %d peaks (%.3g cell updates, %.1f s)" % (what, w.pm.n_peaks, updates, dt)}


def lds_probe():
    """Live LDS-atomic microbenchmark: lanes per shader clock per CU, shader
    clocks per wave-wide atomic and the chip-wide rate for three address
    patterns, for the tile pattern with 3 of each 16-lane group's lanes
    active, and for the tile pattern with ds_add_f32 (libfh_probe.so)."""
    import ctypes
    lib = ctypes.CDLL(PROBE_LIB)
    f = lib.fhp_lds_atomic
    d = ctypes.POINTER(ctypes.c_double)
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, d, d, d, d]
    f.restype = ctypes.c_int
    out = {}
    for mode, name, active in [(0, "conflict_free", 64), (1, "random", 64), (2, "tile_pattern", 64),
                               (6, "tile_pattern_3_of_16_rows", 12), (7, "tile_pattern_f32", 64)]:
        iters = 200 if mode == 7 else 2000  # the float atomics are far slower
        rate, lpc, ms, ghz = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = f(mode, iters, 1024, ctypes.byref(rate), ctypes.byref(lpc), ctypes.byref(ms), ctypes.byref(ghz))
        if rc != 0:
            raise RuntimeError("LDS probe failed with HIP error %d" % rc)
        out[name] = {"lanes_per_clk_per_cu": lpc.value, "tops": rate.value / 1e12, "clock_ghz": ghz.value,
                     "clocks_per_wave_atomic": active / lpc.value if lpc.value > 0 else None}
    return out


def large_band_leg(ctx, n_sky, steps=2):
    """The large-band configuration at full size: 10 Hz at 1024 Hz, T_FFT
    1024 s, 25000 FFTs (~20M peaks), 147 rows, 4096 directions, FP32 weights;
    one warm-up step (autotuning), then `steps` timed steps."""
    import torch

    from paper_1407_8333_amd import api, synth
    w = synth.workload("large-1024hz", n_sky=n_sky)
    dpm = ctx.upload(w.pm)
    wt = torch.as_tensor(w.weights, device="cuda")
    out = torch.empty((n_sky, api.n_subbands(w.grid, w.sel), 2, 8), dtype=torch.int32, device="cuda")
    api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, weights=wt, out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        api.fh_hough_candidates(ctx, dpm, w.sky, w.grid, w.sel, weights=wt, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pr = ctx.profile_read()
    ctx.profile(False)
    plan = ctx.plan(dpm, w.grid, 0)
    dpm.release()
    cells = w.pm.n_peaks * w.grid.ns * n_sky * steps
    launch_ms = pr["tiles_ms"] / max(1, pr["tiles_launches"])
    achieved = pr["cell_updates"] / max(1, pr["tiles_launches"]) / (launch_ms * 1e-3) / 1e12
    return {"workload": WORKLOAD_TEXT["large-1024hz"] + ", %d directions, FP32 weights" % n_sky,
            "n_sky": n_sky, "n_peaks": w.pm.n_peaks, "steps": steps,
            "value": cells / dt, "unit": "cell-updates/s", "ms_per_step": dt * 1e3 / steps,
            "tile_launches_per_step": pr["tiles_launches"] / steps, "tile": [plan["tile_rows"], plan["tile_bins"]],
            "kernel_split_ms_per_step": {"tiles": pr["tiles_ms"] / steps, "front": pr["front_ms"] / steps,
                                         "select": pr["select_ms"] / steps},
            "roofline": {"bound": "lds_atomic", "achieved": achieved, "peak": LDS_ATOMIC_PEAK_TOPS,
                         "unit": "TOP/s", "frac": achieved / LDS_ATOMIC_PEAK_TOPS, "launch_ms": launch_ms}}


def serve_t_fft(f_lo):
    """T_FFT of a band by frequency: [20, 128) Hz 8192 s, [128, 256) 4096 s,
    [256, 512) 2048 s, [512, 1000] 1024 s (every one within the maximum FFT
    length for which a signal stays within one bin, Table I)."""
    return 8192.0 if f_lo < 128 else 4096.0 if f_lo < 256 else 2048.0 if f_lo < 512 else 1024.0


class _BandShape:
    """What synth.make_grid reads of a peakmap: T_FFT, FFT count, times."""

    def __init__(self, t_fft, t):
        self.t_fft, self.t, self.n_fft = t_fft, t, int(t.shape[0])


def build_serving_bands(ctx, f_lo=20, f_hi=1000, seed=77, t_obs_days=149.0):
    """Resident 1 Hz peakmaps of every band [f, f + 1) Hz, f = f_lo .. f_hi - 1,
    of a ~149 d run: Exp(1) equalised spectra drawn on the GPU from a seeded
    generator over the band and its Doppler and spin-down margins, turned into
    peakmaps (local maxima above 2.5) by fh_peakmap_from_spectra."""
    import torch

    from paper_1407_8333_amd import api, synth
    rng = synth.rng_for(seed)
    t_obs = t_obs_days * 86400.0
    shapes = {}
    for t_fft in (8192.0, 4096.0, 2048.0, 1024.0):
        n_fft = int(round(t_obs / (0.5 * t_fft)))
        t = synth.fft_times(n_fft, t_fft)
        shapes[t_fft] = (_BandShape(t_fft, t), synth.detector_velocity(t, rng))
    plan = []
    for f in range(f_lo, f_hi):
        t_fft = serve_t_fft(f)
        n_fft = shapes[t_fft][0].n_fft
        m = synth.band_margin_bins(f + 1.0, t_fft, n_fft, 1e-8)
        k_lo, k_hi = int(f * t_fft) - m, int((f + 1) * t_fft) + m
        plan.append((f, t_fft, n_fft, k_lo, k_hi))
    cap = max(n * (k_hi - k_lo + 2) for _, _, n, k_lo, k_hi in plan)
    buf = torch.empty(cap, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    bands = []
    for f, t_fft, n_fft, k_lo, k_hi in plan:
        nb = k_hi - k_lo + 2  # one guard bin each side
        sp = buf[:n_fft * nb].view(n_fft, nb)
        sp.exponential_(generator=gen)
        shape, v = shapes[t_fft]
        dpm = api.DevicePeakmap.from_spectra(ctx, sp, k_lo - 1, 2.5, shape.t, v, t_fft)
        bands.append((shape, float(f), dpm))
    del buf
    torch.cuda.synchronize()
    return bands


SPIN_DOWN_RANGES = {"narrow": (-1e-9, 1e-10), "wide": (-1e-8, 1e-9)}


def serving_shapes(ctx, which=None, n_sky=128, reps=3, seed=5):
    """Each serving shape alone: the first 1 Hz band of each T_FFT with each
    spin-down range, n_sky random directions, top-2 per 0.1 Hz sub-band.  Per
    shape: ms per call, the tile kernel's ms and its fraction of the
    LDS-atomic peak (peaks x rows x directions / tile time / 9.83e12 /s), the
    front's ms, and the plan (tile width, row blocks run, folded tail rows)."""
    import torch

    from paper_1407_8333_amd import api, synth
    bands = build_serving_bands(ctx)
    first = {}
    for shape, f, dpm in bands:
        first.setdefault(shape.t_fft, (shape, f, dpm))
    rng = synth.rng_for(seed)
    out = []
    for t_fft in (8192.0, 4096.0, 2048.0, 1024.0):
        for name, rg in SPIN_DOWN_RANGES.items():
            if which and "%d:%s" % (t_fft, name) not in which:
                continue
            shape, f, dpm = first[t_fft]
            grid = synth.make_grid(shape, f, f + 1.0, *rg)
            sel = synth.Selection(width=int(round(0.1 * grid.kf * t_fft)))
            sky = synth.sky_uniform(n_sky, rng)
            api.fh_hough_candidates(ctx, dpm, sky, grid, sel)  # autotunes the shape
            torch.cuda.synchronize()
            ctx.profile(True)
            t0 = time.perf_counter()
            for _ in range(reps):
                api.fh_hough_candidates(ctx, dpm, sky, grid, sel)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            pr = ctx.profile_read()
            ctx.profile(False)
            plan = ctx.plan(dpm, grid)
            cells = dpm.n_peaks * grid.ns * n_sky
            tiles_ms = pr["tiles_ms"] / reps
            out.append({"t_fft": t_fft, "range": name, "ns": grid.ns, "n_fft": dpm.n_fft,
                        "n_peaks": dpm.n_peaks, "n_sky": n_sky, "ms": dt * 1e3,
                        "cell_updates_per_s": cells / dt, "tiles_ms": tiles_ms,
                        "tile_frac": cells / (tiles_ms * 1e-3) / (LDS_ATOMIC_PEAK_TOPS * 1e12),
                        "front_ms": pr["front_ms"] / reps, "tile_bins": plan["tile_bins"],
                        "row_blocks": plan["n_row_blocks"],
                        "tail_rows": max(0, grid.ns - 16 * plan["n_row_blocks"])})
    for _, _, dpm in bands:
        dpm.release()
    return out


def serve_bench(ctx, n_req, load, lanes=8, seed=77, burst_n=192):
    """Poisson stream of (band, sky patch, spin-down range) requests through the
    continuous-batching server.  Bands: one of the 980 resident 1 Hz bands of
    20-1000 Hz, uniformly; sky patch: 1-256 random directions, log-uniform in
    the count; spin-down range: [-1e-9, 1e-10] or [-1e-8, 1e-9] Hz/s, equally
    likely.  Capacity is measured on a burst submitted at once; the stream then
    arrives at `load` times that capacity."""
    import numpy as np
    import torch

    from paper_1407_8333_amd import api, synth
    t_build = time.perf_counter()
    bands = build_serving_bands(ctx, seed=seed)
    build_s = time.perf_counter() - t_build
    rng = synth.rng_for(seed + 1)
    ranges = [(-1e-9, 1e-10), (-1e-8, 1e-9)]

    def draw():
        shape, f_lo, dpm = bands[int(rng.integers(len(bands)))]
        grid = synth.make_grid(shape, f_lo, f_lo + 1.0, *ranges[int(rng.integers(2))])
        sel = synth.Selection(width=int(round(0.1 * grid.kf * shape.t_fft)))
        n_sky = int(min(256, max(1, round(2.0 ** rng.uniform(0.0, 8.0)))))
        return dpm, grid, sel, synth.sky_uniform(n_sky, rng)

    def out_for(r):
        return torch.empty((len(r[3]), api.n_subbands(r[1], r[2]), 2, 8), dtype=torch.int32, device="cuda")

    # one search per distinct shape first (T_FFT x spin-down range): tile
    # autotuning on 128 directions, as the serving_shapes leg tunes them
    for t_fft in (8192.0, 4096.0, 2048.0, 1024.0):
        shape, f_lo, dpm = next(b for b in bands if b[0].t_fft == t_fft)
        for rg in ranges:
            grid = synth.make_grid(shape, f_lo, f_lo + 1.0, *rg)
            sel = synth.Selection(width=int(round(0.1 * grid.kf * t_fft)))
            api.fh_hough_candidates(ctx, dpm, synth.sky_uniform(128, rng), grid, sel)
    torch.cuda.synchronize()

    srv = api.Server(ctx, hbm_budget=64 << 30, lanes=lanes)
    # capacity: a burst submitted at once
    burst = [draw() for _ in range(burst_n)]
    outs = [out_for(b) for b in burst]
    t0 = time.perf_counter()
    for b, o in zip(burst, outs):
        srv.submit(b[0], b[3], b[1], b[2], o)
    got, burst_cells = 0, 0
    while got < len(burst):
        for c in srv.poll():
            got += 1
            burst_cells += c["cell_updates"]
    burst_s = time.perf_counter() - t0
    cap = len(burst) / burst_s
    rate = load * cap
    reqs = [draw() for _ in range(n_req)]
    outs = [out_for(r) for r in reqs]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    done = []
    t0 = time.perf_counter()
    k = 0
    while len(done) < n_req:
        now = time.perf_counter() - t0
        while k < n_req and arrivals[k] <= now:
            r = reqs[k]
            srv.submit(r[0], r[3], r[1], r[2], outs[k], tag=k)
            k += 1
        done.extend(srv.poll())
    wall = time.perf_counter() - t0
    srv.close()
    for _, _, d in bands:
        d.release()
    bad = sum(1 for c in done if c["status"] != 0)
    lat = [c["latency_ms"] for c in done]
    dev = [c["device_ms"] for c in done]
    cells = sum(c["cell_updates"] for c in done)
    return {"requests": n_req, "failed": bad, "lanes": lanes, "hbm_budget_gib": 64,
            "arrival_rate_per_s": rate, "capacity_per_s": cap, "load": load,
            "capacity_throughput": burst_cells / burst_s, "burst_requests": burst_n,
            "p50_latency_ms": pct(lat, 50), "p99_latency_ms": pct(lat, 99),
            "mean_queue_ms": float(np.mean([c["queue_ms"] for c in done])),
            "p50_device_ms": pct(dev, 50), "p99_device_ms": pct(dev, 99),
            # mean number of requests on the device at once (device time / wall)
            "mean_requests_on_device": float(sum(dev)) / (wall * 1e3),
            "throughput": cells / wall, "unit": "cell-updates/s", "stream_s": wall,
            "bands": "980 resident 1 Hz bands, 20-1000 Hz (T_FFT 8192 / 4096 / 2048 / 1024 s "
                     "below 128 / 256 / 512 / 1000 Hz), ~149 d, built on the GPU in %.1f s" % build_s,
            "sky_patch": "1-256 random directions, log-uniform count",
            "spin_down_ranges": ranges}


def trace_overlap(path, skip=()):
    """Overlap of kernels from different streams in a rocprofv3 kernel trace
    (kernel_trace.csv): the time during which kernels of two or more streams
    (Stream_Id, else Queue_Id) run at once, against the time any kernel runs.
    Streams in `skip` (e.g. the one that built the inputs) are left out."""
    import csv
    rows = list(csv.DictReader(open(path)))
    key = "Stream_Id" if rows and "Stream_Id" in rows[0] else "Queue_Id"
    rows = [r for r in rows if r[key] not in set(skip)]
    ev = []
    for r in rows:
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        tile = "k_tiles" in r["Kernel_Name"]
        ev.append((a, 1, r[key], tile))
        ev.append((b, -1, r[key], tile))
    ev.sort(key=lambda e: (e[0], e[1]))
    active, tiles = {}, {}
    busy = multi = multi_tiles = 0
    last = ev[0][0] if ev else 0
    for t, d, q, tile in ev:
        dt = t - last
        if active:
            busy += dt
        if len(active) >= 2:
            multi += dt
        if len(tiles) >= 2:
            multi_tiles += dt
        last = t
        active[q] = active.get(q, 0) + d
        if active[q] == 0:
            del active[q]
        if tile:
            tiles[q] = tiles.get(q, 0) + d
            if tiles[q] == 0:
                del tiles[q]
    return {"kernels": len(rows), "streams": sorted({r[key] for r in rows}), "stream_key": key,
            "queues": sorted({r["Queue_Id"] for r in rows}), "skipped_streams": sorted(skip),
            "busy_ms": busy * 1e-6, "two_or_more_streams_ms": multi * 1e-6,
            "two_or_more_streams_frac": multi / busy if busy else 0.0,
            "tile_kernels_of_two_or_more_streams_ms": multi_tiles * 1e-6}


def main():
    args = parse()
    if args.overlap_from:
        print(json.dumps(trace_overlap(args.overlap_from, args.overlap_skip)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the frequency-Hough path on a "
              "single MI355X (no multi-GPU code path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1407_8333_amd import api, synth

    if args.shapes_only is not None:
        ctx = api.Context(0)
        out = {"serving_shapes": serving_shapes(ctx, args.shapes_only, n_sky=args.shape_sky or 128)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return

    if args.serve_only:
        ctx = api.Context(0)
        out = {"serving": serve_bench(ctx, args.serve_requests, args.serve_load, lanes=args.serve_lanes)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return

    n_sky = args.n_sky or (1024 if args.workload == "batch-256hz" else
                           (4096 if args.workload == "large-1024hz" else 1))
    w = synth.workload(args.workload, n_sky=n_sky)
    if args.unweighted:
        w.weights = None
    grid, sel = w.grid, w.sel
    cells_per_sky = w.pm.n_peaks * grid.ns
    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    ctx.set_doppler(args.doppler)
    dpm = ctx.upload(w.pm)
    wt = None if w.weights is None else torch.as_tensor(w.weights, device=dev)
    out = torch.empty((n_sky, api.n_subbands(grid, sel), 2, 8), dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()  # a created stream: graph capture needs one

    def step(graph=not args.no_graph, chunk=args.sky_chunk):
        with torch.cuda.stream(stream):
            api.fh_hough_candidates(ctx, dpm, w.sky, grid, sel, weights=wt, schedule=1,
                                    tile_bins=args.tile_bins, sky_chunk=chunk, use_graph=1 if graph else 0,
                                    out=out, stream=stream)

    def timed(n, **kw):
        """ms per step of n steps (events on the launch stream), after one untimed step."""
        step(**kw)
        stream.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n):
            step(**kw)
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / n

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
    prof_graph = ctx.profile_read()
    ctx.profile(False)
    step_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    total_cells = cells_per_sky * n_sky * args.steps
    value = total_cells / wall
    ctx.check()

    # Kernel timing: a graph replay is one span, so the tile kernel's launch
    # duration comes from the same launch configuration run eagerly, each
    # kernel bracketed by HIP events on the launch stream.
    n_eager = max(3, args.variant_steps)
    step(graph=False)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(n_eager):
        step(graph=False)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / n_eager
    prof = ctx.profile_read()
    ctx.profile(False)
    variants = {"graph_ms_per_step": ms_per_step, "eager_ms_per_step": eager_ms,
                "tile_launches_per_step": prof["tiles_launches"] / n_eager}
    if args.variant_steps > 0 and n_sky > 256:
        variants["eager_4x256_ms_per_step"] = timed(args.variant_steps, graph=False, chunk=256)
        variants["graph_4x256_ms_per_step"] = timed(args.variant_steps, graph=True, chunk=256)

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

    probe = None if args.no_probe else lds_probe()
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
                   "weighted": wt is not None, "schedule": "persistent", "doppler": args.doppler,
                   "tile": [plan["tile_rows"], plan["tile_bins"]],
                   "launch": "one hipGraph replay per step" if not args.no_graph else "eager launches",
                   "tile_launches_per_step": variants["tile_launches_per_step"]},
        "p50_ms_per_step": pct(step_ms, 50),
        "p99_ms_per_step": pct(step_ms, 99),
        "batched_vs_plain": None if plain is None else value / plain["value"],
        "plain": plain,
        "launch_variants": variants,
        "kernel_split_ms_per_step": {"tiles": prof["tiles_ms"] / n_eager,
                                     "front": prof["front_ms"] / n_eager,
                                     "select": prof["select_ms"] / n_eager},
        "roofline": {"bound": "lds_atomic", "achieved": achieved, "peak": LDS_ATOMIC_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / LDS_ATOMIC_PEAK_TOPS,
                     "peak_basis": "16 ds_add_u32 lanes per clock per CU x 256 CUs x 2.4 GHz",
                     "probe": probe,
                     "traffic": committed_traffic(args.workload, n_sky, plan["tile_bins"], wt is not None),
                     "valu_cobound": valu_cobound(achieved, args.workload, n_sky, plan["tile_bins"],
                                                  wt is not None),
                     "kernel": "k_tiles_persistent (one op = one ds_add_u32 cell update)",
                     "launch_ms": tiles_ms_avg, "cells_per_launch": cells_per_launch},
    }
    if args.large_sky > 0 and args.workload == "batch-256hz":
        dpm.release()
        dpm = None
        res["large_band"] = large_band_leg(ctx, args.large_sky)
    if args.shape_sky > 0 and args.workload == "batch-256hz":
        res["serving_shapes"] = serving_shapes(ctx, n_sky=args.shape_sky)
    if args.serve_requests > 0:
        res["serving"] = serve_bench(ctx, args.serve_requests, args.serve_load, lanes=args.serve_lanes)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_rows)
    if dpm is not None:
        dpm.release()
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
