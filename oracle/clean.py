"""Peakmap cleaning oracle -- TEST INFRASTRUCTURE ONLY (tests, smoke and the
benchmark's CPU baseline may call it; the library never does).

Plain numpy definitions of the cleaning steps of Sec. "Removal of time and
frequency domain disturbances":

* gross histogram and wandering-line veto (subsection on spectral wandering
  lines): peaks counted in cells of dt_h seconds x df_h Hz; every peak of a
  cell holding more than a threshold is removed;
* persistency (subsection on lines of constant frequency, second option):
  the number of FFTs holding a peak at each natural bin;
* robust statistic (appendix "Robust statistic"): median m1 and dispersion
  m2 = median(|x - m1|) / 0.6745 (the printed formula is garbled; this is
  the median absolute deviation it describes, normalised so that m2 is the
  standard deviation of a normal variable);
* veto of natural bins whose statistic exceeds a threshold (persistency
  counts, or the maximum over spin-down rows of the Hough map computed
  without Doppler correction, the third option of that subsection: the map
  itself comes from ``oracle.hough_map`` with a zero sky vector).

Cell geometry (the same definition the library documents): FFT i is in
time cell floor((t_i - t_origin) / dt_h); a peak of natural bin k is in
frequency cell floor(k / (df_h T_FFT)) - c0; cells outside [0, n_t) x
[0, n_f) are not counted and their peaks are never vetoed.
"""
from __future__ import annotations

import math

import numpy as np

ROBUST_C = 0.6745


def gross_geometry(t, k_lo: int, k_hi: int, dt_h: float, df_h: float, t_fft: float):
    """(t_origin, dt_h, n_t, df_h, c0, n_f) covering FFT times t and natural
    bins [k_lo, k_hi)."""
    t = np.asarray(t, dtype=np.float64)
    t_origin = float(t.min())
    n_t = int(math.floor((float(t.max()) - t_origin) / dt_h)) + 1
    B = df_h * t_fft
    c0 = int(math.floor(float(k_lo) / B))
    n_f = int(math.floor(float(k_hi - 1) / B)) - c0 + 1
    return t_origin, dt_h, n_t, df_h, c0, n_f


def _cells(pm, t_origin, dt_h, n_t, df_h, c0, n_f):
    """Per peak: (time cell, frequency cell, inside?)."""
    counts = np.diff(pm.offsets)
    ti = np.floor((np.asarray(pm.t, np.float64) - t_origin) / dt_h).astype(np.int64)
    ct = np.repeat(ti, counts)
    B = df_h * pm.t_fft
    cf = np.floor(pm.bins.astype(np.float64) / B).astype(np.int64) - c0
    inside = (ct >= 0) & (ct < n_t) & (cf >= 0) & (cf < n_f)
    return ct, cf, inside


def gross_histogram(pm, t_origin, dt_h, n_t, df_h, c0, n_f) -> np.ndarray:
    """int64 [n_t][n_f]: peaks per gross cell."""
    ct, cf, inside = _cells(pm, t_origin, dt_h, n_t, df_h, c0, n_f)
    h = np.zeros((n_t, n_f), np.int64)
    np.add.at(h, (ct[inside], cf[inside]), 1)
    return h


def _keep(pm, keep):
    """Peakmap with the peaks where keep is True (order kept)."""
    counts = np.add.reduceat(keep.astype(np.int64), pm.offsets[:-1]) if pm.bins.size else \
        np.zeros(len(pm.t), np.int64)
    # reduceat on an empty segment returns the next element: fix empty FFTs
    counts = np.where(np.diff(pm.offsets) == 0, 0, counts)
    off = np.zeros(len(pm.t) + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return off, pm.bins[keep].astype(np.int32)


def gross_veto(pm, t_origin, dt_h, n_t, df_h, c0, n_f, threshold: float):
    """(offsets, bins) without the peaks whose cell holds more than threshold."""
    h = gross_histogram(pm, t_origin, dt_h, n_t, df_h, c0, n_f)
    ct, cf, inside = _cells(pm, t_origin, dt_h, n_t, df_h, c0, n_f)
    over = np.zeros(pm.bins.shape[0], bool)
    over[inside] = h[ct[inside], cf[inside]] > threshold
    return _keep(pm, ~over)


def gross_expectation(dt_h: float, df_h: float, t_fft: float, p0: float, overlap: float = 0.5):
    """(N, E_H, sigma_H) of a gross cell: N = FFTs per cell x natural bins
    per cell (FFTs interlaced by `overlap`), E_H = N p0,
    sigma_H = sqrt(N p0 (1 - p0))."""
    n = (dt_h / (t_fft * (1.0 - overlap))) * (df_h * t_fft)
    return n, n * p0, math.sqrt(n * p0 * (1.0 - p0))


def bin_counts(pm, k_lo: int, k_hi: int) -> np.ndarray:
    """int64 [k_hi - k_lo]: FFTs holding a peak at each natural bin."""
    b = pm.bins.astype(np.int64)
    b = b[(b >= k_lo) & (b < k_hi)]
    return np.bincount(b - k_lo, minlength=k_hi - k_lo).astype(np.int64)


def median(x) -> float:
    """Median: the middle value, or the mean of the two middle values."""
    s = np.sort(np.asarray(x, dtype=np.float64))
    n = s.size
    if n == 0:
        raise ValueError("median of nothing")
    return float(s[n // 2]) if n % 2 else 0.5 * (float(s[n // 2 - 1]) + float(s[n // 2]))


def robust_stats(x):
    """(m1, m2): median, and median absolute deviation / 0.6745."""
    m1 = median(x)
    m2 = median(np.abs(np.asarray(x, dtype=np.float64) - m1)) / ROBUST_C
    return m1, m2


def veto_bins(pm, k_lo: int, k_hi: int, x, step: int, offset: int, threshold: float):
    """(offsets, bins) without the peaks of natural bins k in [k_lo, k_hi)
    whose statistic x[step (k - k_lo) + offset] (when that index is inside x)
    exceeds threshold."""
    x = np.asarray(x)
    b = pm.bins.astype(np.int64)
    idx = step * (b - k_lo) + offset
    ok = (b >= k_lo) & (b < k_hi) & (idx >= 0) & (idx < x.size)
    over = np.zeros(b.size, bool)
    over[ok] = x[idx[ok]] > threshold
    return _keep(pm, ~over)


def line_counts(hmap) -> np.ndarray:
    """Per fine bin, the largest count over the spin-down rows of a map."""
    return np.asarray(hmap).max(axis=0)
