"""CPU oracle of the frequency-Hough hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code: they agree only through the fixed-point definition written
in ``fh_oracle.c`` (Eqs. fdopp, uno, due, ncount, ncountadap, freqres, sdstep).

Contents
  * ``hough_map``   - direct-fill FP64 Hough map (C, OpenMP over rows)
  * ``candidates``  - exhaustive sub-band candidate scan (C)
  * ``critical_ratio`` - Eq. cr, and its weighted analogue
  * ``brute``       - pure-Python cell-major map for tiny inputs
  * ``stats``       - closed forms of the statistics sections (pins)
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fh_oracle.c")
_LIB = os.path.join(_HERE, "libfh_oracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _open(path):
    """A loaded build of fh_oracle.c with its prototypes attached."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fho_hough_map.argtypes = [i32, P, P, P, P, f64, P, P, i32, i64, i32, i32,
                                  f64, f64, f64, i32, i32, P]
    lib.fho_hough_map.restype = ctypes.c_int
    lib.fho_hough_map_mode.argtypes = [i32, P, P, P, P, f64, P, P, i32, i64, i32, i32,
                                       f64, f64, f64, i32, i32, i32, f64, P]
    lib.fho_hough_map_mode.restype = ctypes.c_int
    lib.fho_shift_center.argtypes = [i32, i32, f64, f64]
    lib.fho_shift_center.restype = i64
    lib.fho_candidates.argtypes = [P, i32, i32, i32, i32, i32, P, P]
    lib.fho_candidates.restype = i32
    lib.fho_row_shifts.argtypes = [i32, P, f64, f64, i32, f64, f64, i32, P]
    lib.fho_row_shifts.restype = None
    lib.fho_left_edges.argtypes = [i32, P, P, P, P, f64, P, i32, i64, f64, f64, f64,
                                   i64, P, P, P]
    lib.fho_left_edges.restype = ctypes.c_int
    lib.fho_inv_doppler.argtypes = [i32, P, P, P]
    lib.fho_inv_doppler.restype = None
    lib.fho_center.argtypes = [i32, i32, f64]
    lib.fho_center.restype = i64
    lib.fho_set_threads.argtypes = [i32]
    lib.fho_set_threads.restype = None
    lib.fho_max_threads.argtypes = []
    lib.fho_max_threads.restype = i32
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            _lib = _open(_LIB)
    return _lib


@contextlib.contextmanager
def _library(path):
    """Route every oracle call through another build of fh_oracle.c while the
    context is open (the mutation test plants mistakes in copies of it)."""
    global _lib
    lib = _open(path)
    with _lock:
        saved, _lib = _lib, lib
    try:
        yield lib
    finally:
        with _lock:
            _lib = saved


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def shift_reference(grid, t_fft: float) -> float:
    """Default reference frequency of the per-FFT shift variant: the centre
    of the map's band, (b0 + nf / 2) / (K_f T_FFT)."""
    return (float(grid.b0) + 0.5 * float(grid.nf)) / (float(grid.kf) * float(t_fft))


def hough_map(pm, grid, nhat, weights=None, rows=None, threads=None, doppler: str = "exact",
              f_ref=None) -> np.ndarray:
    """FP64 Hough map [ns][nf] of one sky direction.

    pm: peakmap (t_fft, t, v, offsets, bins); grid: kf, b0, nf, ns, fdot0,
    dfdot, t0; nhat: unit vector; weights: per-FFT weights or None; rows:
    (lo, hi) to compute a row range only (other rows are returned as 0);
    doppler: "exact" (per peak) or "shift" (per FFT at f_ref, by default the
    band centre).
    """
    lib = _load()
    if threads is not None:
        lib.fho_set_threads(int(threads))
    t = np.ascontiguousarray(pm.t, dtype=np.float64)
    v = np.ascontiguousarray(pm.v, dtype=np.float64).reshape(-1, 3)
    off = np.ascontiguousarray(pm.offsets, dtype=np.int64)
    bins = np.ascontiguousarray(pm.bins, dtype=np.int32)
    n = np.ascontiguousarray(np.asarray(nhat, dtype=np.float64).reshape(3))
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    lo, hi = (0, grid.ns) if rows is None else rows
    out = np.zeros((grid.ns, grid.nf), dtype=np.float64)
    if doppler not in ("exact", "shift"):
        raise ValueError("doppler must be 'exact' or 'shift'")
    fr = shift_reference(grid, pm.t_fft) if f_ref is None else float(f_ref)
    rc = lib.fho_hough_map_mode(int(t.shape[0]), _ptr(off), _ptr(bins), _ptr(t), _ptr(v),
                                float(pm.t_fft), _ptr(n), None if w is None else _ptr(w),
                                int(grid.kf), int(grid.b0), int(grid.nf), int(grid.ns),
                                float(grid.fdot0), float(grid.dfdot), float(grid.t0),
                                int(lo), int(hi), 1 if doppler == "shift" else 0, fr, _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def max_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().fho_max_threads())


def set_threads(n: int) -> None:
    _load().fho_set_threads(int(n))


def row_shifts(pm, grid, s: int):
    """Spin-down shifts G_is of row s for every FFT, int64, in fixed-point fine
    bins (2^16 steps per bin)."""
    lib = _load()
    n = pm.t.shape[0]
    out = np.zeros(n, np.int64)
    t = np.ascontiguousarray(pm.t, dtype=np.float64)
    lib.fho_row_shifts(n, _ptr(t), float(grid.t0), float(pm.t_fft), int(grid.kf),
                       float(grid.fdot0), float(grid.dfdot), int(s), _ptr(out))
    return out


def left_edges(pm, grid, nhat, peaks, rows):
    """Fixed-point left stripe edges L_s of the (peak, row) pairs, int64, by
    the same steps as ``hough_map`` (exact Doppler correction)."""
    lib = _load()
    t = np.ascontiguousarray(pm.t, dtype=np.float64)
    v = np.ascontiguousarray(pm.v, dtype=np.float64).reshape(-1, 3)
    off = np.ascontiguousarray(pm.offsets, dtype=np.int64)
    bins = np.ascontiguousarray(pm.bins, dtype=np.int32)
    n = np.ascontiguousarray(np.asarray(nhat, dtype=np.float64).reshape(3))
    pk = np.ascontiguousarray(peaks, dtype=np.int64)
    rw = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros(pk.shape[0], np.int64)
    rc = lib.fho_left_edges(int(t.shape[0]), _ptr(off), _ptr(bins), _ptr(t), _ptr(v), float(pm.t_fft),
                            _ptr(n), int(grid.kf), int(grid.b0), float(grid.fdot0), float(grid.dfdot),
                            float(grid.t0), int(pk.shape[0]), _ptr(pk), _ptr(rw), _ptr(out))
    if rc != 0:
        raise ValueError("peak index out of range")
    return out


def inv_doppler(pm, nhat):
    lib = _load()
    n = pm.t.shape[0]
    r = np.zeros(n, np.float64)
    v = np.ascontiguousarray(pm.v, dtype=np.float64).reshape(-1, 3)
    nh = np.ascontiguousarray(np.asarray(nhat, dtype=np.float64).reshape(3))
    lib.fho_inv_doppler(n, _ptr(v), _ptr(nh), _ptr(r))
    return r


def shift_center(k, kf, q, r):
    """Corrected centre of the per-FFT shift variant (q: reference in fine bins)."""
    return int(_load().fho_shift_center(int(k), int(kf), float(q), float(r)))


def center(k, kf, r):
    return int(_load().fho_center(int(k), int(kf), float(r)))


def candidates(hmap: np.ndarray, width: int, excl: int = 4, sep: int = 8):
    """Exhaustive sub-band candidates of a [ns][nf] map.

    Returns (idx, val): idx [n_sb, 2, 3] int32 = (valid, bin, row), val [n_sb, 2].
    """
    lib = _load()
    m = np.ascontiguousarray(hmap, dtype=np.float64)
    ns, nf = m.shape
    n_sb = (nf + width - 1) // width
    idx = np.zeros((n_sb, 2, 3), np.int32)
    val = np.zeros((n_sb, 2), np.float64)
    rc = lib.fho_candidates(_ptr(m), ns, nf, int(width), int(excl), int(sep), _ptr(idx), _ptr(val))
    if rc < 0:
        raise ValueError("bad width")
    return idx, val


# the statistics closed forms live in one place, oracle/stats.py (pinned to
# the paper's printed numbers in tests/test_paper_values.py)
from .stats import critical_ratio, critical_ratio_weighted, p0  # noqa: E402,F401
