"""bench.py's host side, without a GPU: the one-GPU contract, the stream
overlap read from a kernel trace, and the percentile helper."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Stream_Id",
                                          "Queue_Id"])
        w.writeheader()
        for name, a, b, s in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": b, "Stream_Id": s,
                        "Queue_Id": s})


def test_overlap_of_two_streams(tmp_path):
    """Stream 1 runs [0, 10) and [20, 30) ms, stream 2 runs [5, 25) ms, stream
    9 (skipped) [0, 100) ms: busy 30 ms, two streams at once during [5, 10)
    and [20, 25), i.e. 10 ms; tile kernels of both streams overlap in [5, 10)
    only."""
    ms = 1_000_000
    p = tmp_path / "k_kernel_trace.csv"
    _trace(p, [("k_tiles_persistent<...>", 0, 10 * ms, "1"),
               ("k_front", 20 * ms, 30 * ms, "1"),
               ("k_tiles_persistent<...>", 5 * ms, 25 * ms, "2"),
               ("k_pm_rows", 0, 100 * ms, "9")])
    out = bench.trace_overlap(str(p), skip=["9"])
    assert out["kernels"] == 3 and out["streams"] == ["1", "2"]
    assert out["busy_ms"] == pytest.approx(30.0)
    assert out["two_or_more_streams_ms"] == pytest.approx(10.0)
    assert out["two_or_more_streams_frac"] == pytest.approx(1 / 3)
    assert out["tile_kernels_of_two_or_more_streams_ms"] == pytest.approx(5.0)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--overlap-from", str(p),
                        "--overlap-skip", "9"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    assert json.loads(r.stdout.strip().splitlines()[-1])["two_or_more_streams_ms"] == pytest.approx(10.0)


def test_percentiles():
    xs = list(range(1, 101))
    assert bench.pct(xs, 50) == 51
    assert bench.pct(xs, 99) == 99
    assert bench.pct(xs, 0) == 1 and bench.pct(xs, 100) == 100
    assert bench.pct([], 50) is None
