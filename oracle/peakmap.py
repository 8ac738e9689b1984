"""Peakmap oracle (Sec. "Peakmap", Eq. pm) -- TEST INFRASTRUCTURE ONLY.

R(i, j) = S_P(i, j) / S_AR(i, j), computed bin by bin in float32; bin j of
FFT i is a peak when R > theta and R is strictly larger than both
neighbouring bins.  The first and last bin of each row have only one
neighbour and serve as guards (never peaks).  Row bin j is natural bin k0 + j.
"""
from __future__ import annotations

import numpy as np


def peakmap_from_spectra(sp, sar, k0: int, theta: float):
    """Returns (offsets int64 [N+1], bins int32 [P])."""
    sp = np.asarray(sp, dtype=np.float32)
    R = sp if sar is None else sp / np.asarray(sar, dtype=np.float32)
    th = np.float32(theta)
    n = R.shape[0]
    offsets = np.zeros(n + 1, np.int64)
    bins = []
    for i in range(n):
        row = R[i]
        c, left, right = row[1:-1], row[:-2], row[2:]
        j = np.nonzero((c > th) & (c > left) & (c > right))[0] + 1
        bins.append((k0 + j).astype(np.int32))
        offsets[i + 1] = offsets[i] + j.size
    return offsets, (np.concatenate(bins) if bins else np.zeros(0, np.int32)).astype(np.int32)
