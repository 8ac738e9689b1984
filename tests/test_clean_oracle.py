"""Pins of the cleaning oracle (Sec. "Removal of time and frequency domain
disturbances" and the appendix "Robust statistic")."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import clean
from paper_1407_8333_amd import synth


def _golden():
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")):
        if line.startswith("#") or "|" not in line:
            continue
        name, value, _ = [x.strip() for x in line.split("|", 2)]
        g[name] = [float(v) for v in value.split(",")]
    return g


G = _golden()


def test_gross_cell_statistics_match_the_printed_example():
    n, e, sd = clean.gross_expectation(12 * 3600.0, 0.01, 8192.0, 0.0755)
    assert n == pytest.approx(G["gross_points_8192s"][0], rel=0.01)
    assert e == pytest.approx(G["gross_mean_8192s"][0], abs=0.5)
    assert sd == pytest.approx(G["gross_std_8192s"][0], abs=0.05)
    lo, hi = G["gross_threshold_range"]
    assert lo == pytest.approx(e + 2 * sd, abs=1.0) and hi == pytest.approx(e + 3 * sd, abs=1.0)
    # the cell is wide enough for a CW signal: the rotation Doppler band at
    # 128 Hz (|v_rot| / c ~ 1.5e-6) is the printed 1.9e-4 Hz, far below 0.01 Hz
    assert 128.0 * 1.5e-6 == pytest.approx(G["gross_rotation_doppler_128hz"][0], rel=0.02)


def _tiny_pm():
    # 4 FFTs of 100 s at t = 0, 50, 100, 150; natural bins by hand
    t = np.array([0.0, 50.0, 100.0, 150.0])
    segs = [[10, 25, 31], [12], [], [29, 30, 41]]
    off = np.zeros(5, np.int64)
    off[1:] = np.cumsum([len(s) for s in segs])
    bins = np.array([b for s in segs for b in s], np.int32)
    return synth.Peakmap(100.0, t, np.zeros((4, 3)), off, bins)


def test_gross_histogram_by_hand():
    pm = _tiny_pm()
    # cells of 100 s x 0.1 Hz = 10 natural bins: time cells {0,50}->0, {100,150}->1
    geo = clean.gross_geometry(pm.t, 10, 42, 100.0, 0.1, 100.0)
    assert geo == (0.0, 100.0, 2, 0.1, 1, 4)
    h = clean.gross_histogram(pm, *geo)
    want = np.array([[2, 1, 1, 0],    # bins 10, 12 | 25 | 31
                     [0, 1, 1, 1]])   # 29 | 30 | 41
    np.testing.assert_array_equal(h, want)
    off, bins = clean.gross_veto(pm, *geo, threshold=1.5)
    np.testing.assert_array_equal(off, [0, 2, 2, 2, 5])
    np.testing.assert_array_equal(bins, [25, 31, 29, 30, 41])
    # peaks outside the histogram are never vetoed
    off, bins = clean.gross_veto(pm, 0.0, 100.0, 1, 0.1, 1, 1, threshold=0.5)
    np.testing.assert_array_equal(bins, [25, 31, 29, 30, 41])


def test_gross_histogram_counts_every_peak_and_noise_mean():
    rng = synth.rng_for(3)
    pm = synth.make_noise_peakmap(300, 1024.0, 51200, 53248, seed=4, velocity="none")
    geo = clean.gross_geometry(pm.t, pm.k_lo, pm.k_hi, 6 * 3600.0, 0.05, 1024.0)
    h = clean.gross_histogram(pm, *geo)
    assert h.sum() == pm.n_peaks
    # full cells: mean = points per cell x peak density
    inner = h[:-1, 1:-1]
    n_cell = (6 * 3600.0 / 512.0) * (0.05 * 1024.0)
    dens = pm.n_peaks / (pm.n_fft * (pm.k_hi - pm.k_lo))
    assert inner.mean() == pytest.approx(n_cell * dens, rel=0.05)
    del rng


def _wandering_band(seed=10):
    """Noise (T_FFT 1024 s, 400 FFTs, 1 Hz at 100 Hz) plus a line drifting
    0.02 Hz over the run with a peak in every FFT, and a CW signal whose
    peak is present in 10 % of the FFTs (a signal near the detection
    threshold).  Returns (peakmap, line bins, CW bins, FFTs holding the CW)."""
    t_fft, n = 1024.0, 400
    k_lo, k_hi = 102400, 102400 + 1024
    pm = synth.make_noise_peakmap(n, t_fft, k_lo, k_hi, seed=seed)
    t = pm.t
    line = (k_lo + 200 + np.round(np.linspace(0, 0.02 * t_fft, n))).astype(np.int64)
    cw = synth.Injection((k_lo + 700.3) / t_fft, 0.0, np.array([0.0, 0.6, 0.8]))
    kcw = synth.signal_track_bins(t, pm.v, t_fft, cw, 0.5 * (t[0] + t[-1]))[0]
    has_cw = synth.rng_for(seed + 1).random(n) < 0.1
    segs = []
    for i in range(n):
        b = set(pm.bins[pm.offsets[i]:pm.offsets[i + 1]].tolist())
        b.add(int(line[i]))
        if has_cw[i]:
            b.add(int(kcw[i]))
        segs.append(sorted(b))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in segs])
    pm2 = synth.Peakmap(t_fft, t, pm.v, off, np.array([b for s in segs for b in s], np.int32), k_lo, k_hi)
    return pm2, line, kcw, has_cw


def test_wandering_line_is_vetoed_and_a_cw_signal_is_kept():
    """A slowly wandering line fills its gross cells above E_H + 3 sigma_H
    (the paper's choice is 2-3 sigma_H) and is removed; a weak CW signal
    stays in one frequency cell and is kept."""
    pm2, line, kcw, has_cw = _wandering_band()
    n, t_fft = pm2.n_fft, pm2.t_fft
    dt_h, df_h = 6 * 3600.0, 0.01
    geo = clean.gross_geometry(pm2.t, pm2.k_lo, pm2.k_hi, dt_h, df_h, t_fft)
    dens = (pm2.n_peaks - 2 * n) / (n * (pm2.k_hi - pm2.k_lo))
    _, e, sd = clean.gross_expectation(dt_h, df_h, t_fft, dens)
    o2, b2 = clean.gross_veto(pm2, *geo, threshold=e + 3 * sd)
    kept = [set(b2[o2[i]:o2[i + 1]].tolist()) for i in range(n)]
    line_kept = sum(int(line[i]) in kept[i] for i in range(n))
    cw_kept = sum(int(kcw[i]) in kept[i] for i in range(n) if has_cw[i])
    assert line_kept < 0.1 * n
    assert cw_kept >= 0.9 * has_cw.sum()
    # only cells above the threshold lose peaks
    removed = pm2.n_peaks - b2.size
    assert 0 < removed < 0.05 * pm2.n_peaks


def test_robust_statistic_by_hand_and_on_normal_samples():
    assert clean.robust_stats([1, 2, 3, 4, 100]) == (3.0, 1.0 / 0.6745)
    # even count: means of the two middle values; |x - 2.5| = 1.5 0.5 0.5 1.5
    assert clean.robust_stats([4, 1, 3, 2]) == (2.5, 1.0 / 0.6745)
    x = synth.rng_for(1).normal(7.0, 3.0, 200001)
    m1, m2 = clean.robust_stats(x)
    assert m1 == pytest.approx(7.0, abs=0.03) and m2 == pytest.approx(3.0, rel=0.01)
    # a heavy tail moves the mean and the standard deviation, not m1 and m2
    y = np.concatenate([x, np.full(2000, 1e6)])
    m1b, m2b = clean.robust_stats(y)
    assert abs(m1b - m1) < 0.05 and abs(m2b - m2) < 0.05 and np.std(y) > 1e4
    with pytest.raises(ValueError):
        clean.robust_stats([])


def test_persistency_finds_a_constant_line():
    n, t_fft = 500, 1024.0
    pm = synth.make_noise_peakmap(n, t_fft, 10000, 12000, seed=5, velocity="none")
    line_bins = [10500, 11234]
    segs = []
    for i in range(n):
        b = set(pm.bins[pm.offsets[i]:pm.offsets[i + 1]].tolist())
        if i % 5:  # present in 80 % of the FFTs
            b.update(line_bins)
        segs.append(sorted(b))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in segs])
    pm2 = synth.Peakmap(t_fft, pm.t, pm.v, off, np.array([b for s in segs for b in s], np.int32))
    c = clean.bin_counts(pm2, 10001, 11999)
    assert c.sum() == ((pm2.bins >= 10001) & (pm2.bins < 11999)).sum()
    m1, m2 = clean.robust_stats(c)
    dens = pm.n_peaks / (n * 2000)
    assert m1 == pytest.approx(n * dens, rel=0.1)
    assert m2 == pytest.approx(math.sqrt(n * dens * (1 - dens)), rel=0.25)
    thr = m1 + 6 * m2
    assert set((np.nonzero(c > thr)[0] + 10001).tolist()) == set(line_bins)
    o3, b3 = clean.veto_bins(pm2, 10001, 11999, c, 1, 0, thr)
    assert not np.isin(b3, line_bins).any()
    assert b3.size == pm2.n_peaks - c[np.array(line_bins) - 10001].sum()


def test_line_finder_without_doppler():
    """The Hough map without Doppler correction (zero sky vector) puts a
    constant line present in every FFT at N in the zero spin-down row at its
    frequency; a signal whose Doppler shift swings by +-34 bins over the run
    does not reach N/2 anywhere."""
    n, t_fft = 200, 1024.0
    t = synth.fft_times(n, t_fft)
    v = np.zeros((n, 3))
    v[:, 2] = 2e-3 * np.sin(2 * np.pi * np.arange(n) / 50.0)
    k_line = 20480 + 300
    cw = synth.Injection((20480 + 700.4) / t_fft, 0.0, np.array([0.0, 0.6, 0.8]), lam=0.0)
    kcw = synth.signal_track_bins(t, v, t_fft, cw, 0.5 * (t[0] + t[-1]))[0]
    segs = [sorted({k_line, int(kcw[i])}) for i in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in segs])
    pm = synth.Peakmap(t_fft, t, v, off, np.array([b for s in segs for b in s], np.int32))
    dfd = (1.0 / t_fft) / (n * t_fft * 0.5)
    grid = synth.Grid(kf=10, b0=10 * 20480, nf=10 * 1024, ns=3, fdot0=-dfd, dfdot=dfd,
                      t0=0.5 * (t[0] + t[-1]))
    h = oracle.hough_map(pm, grid, np.zeros(3))
    lc = clean.line_counts(h)
    assert h[1, 10 * k_line - grid.b0] == n
    assert lc.max() == n
    assert lc[10 * 700 - 5: 10 * 701 + 5].max() < n / 2
    o, b = clean.veto_bins(pm, 20480, 20480 + 1024, lc, 10, -grid.b0 + 10 * 20480, n / 2)
    assert not (b == k_line).any() and b.size == n
