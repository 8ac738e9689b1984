"""Pins of the peakmap oracle (Sec. "Peakmap", Eq. pm and Eq. p0)."""
import math

import numpy as np

from oracle import peakmap, stats


def test_hand_built_rows():
    th = 2.5
    rows = np.array([
        # guard, then: a peak, a plateau (not strict), below threshold max, edge
        [9.0, 1.0, 3.0, 1.0, 4.0, 4.0, 1.0, 2.4, 1.0, 9.0],
        [1.0, 2.6, 2.5, 2.0, 2.0, 3.0, 2.9, 5.0, 1.0, 2.0],
    ], dtype=np.float32)
    off, bins = peakmap.peakmap_from_spectra(rows, None, 100, th)
    assert off.tolist() == [0, 1, 4]
    # row 0: bin 2 (3.0 > 1, 1); bins 4/5 equal (no strict max); bin 7 below theta;
    # bins 0 and 9 are guards.  row 1: bins 1 (2.6), 5 (3.0 > 2.9) and 7 (5.0)
    assert bins.tolist() == [102, 101, 105, 107]


def test_ratio_is_taken_bin_by_bin():
    sp = np.array([[1.0, 6.0, 2.0, 8.0, 1.0]], np.float32)
    sar = np.array([[1.0, 2.0, 1.0, 2.0, 1.0]], np.float32)
    # R = 1, 3, 2, 4, 1: bins 1 and 3 are local maxima above 2.5
    off, bins = peakmap.peakmap_from_spectra(sp, sar, 0, 2.5)
    assert bins.tolist() == [1, 3]


def test_noise_density_matches_p0():
    rng = np.random.Generator(np.random.PCG64(5))
    R = rng.standard_exponential((300, 4000)).astype(np.float32)
    off, bins = peakmap.peakmap_from_spectra(R, None, 0, 2.5)
    m = 300 * (4000 - 2)
    q = stats.p0(2.5)
    assert abs(off[-1] - m * q) < 5 * math.sqrt(m * q * (1 - q))
