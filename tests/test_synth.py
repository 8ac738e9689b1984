"""The synthetic generator reproduces the paper's peakmap statistics."""
import math

import numpy as np
import pytest

from oracle import stats
from paper_1407_8333_amd import synth


def test_noise_peak_density_is_p0():
    pm = synth.make_noise_peakmap(400, 1024.0, 100_000, 102_000, seed=3, velocity="none")
    m = 400 * 2000
    q = stats.p0(2.5)
    # binomial expectation m p0 and spread sqrt(m p0 (1-p0)) (Eq. p0 and below)
    assert abs(pm.n_peaks - m * q) < 5 * math.sqrt(m * q * (1 - q))


def test_peaks_are_local_maxima_never_adjacent():
    pm = synth.make_noise_peakmap(50, 1024.0, 1000, 3000, seed=4)
    for i in range(pm.n_fft):
        seg = pm.bins[pm.offsets[i]:pm.offsets[i + 1]]
        assert np.all(np.diff(seg) >= 2)


def test_signal_bin_selection_probability():
    """Signal bins are a local max above theta with the probability of the
    non-central chi^2 model (Eq. noncenchi2)."""
    lam = 1.5
    t_fft = 1024.0
    n = 4000
    inj = synth.Injection(100.0 + 0.3 / t_fft, 0.0, np.array([1.0, 0.0, 0.0]), lam=lam)
    pm = synth.make_noise_peakmap(n, t_fft, 102_300, 102_500, seed=8, velocity="none",
                                  injections=[inj], t0=0.0)
    k = int(round(inj.f0 * t_fft))
    hit = sum(int(np.any(pm.bins[pm.offsets[i]:pm.offsets[i + 1]] == k)) for i in range(n))
    p = stats.p_lambda_exact(2.5, lam)
    assert abs(hit / n - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_velocity_scale_and_sky_norm():
    rng = synth.rng_for(1)
    t = synth.fft_times(1000, 4096.0)
    v = synth.detector_velocity(t, rng)
    sp = np.linalg.norm(v, axis=1)
    assert sp.max() < 1.02e-4 and sp.min() > 0.98e-4
    s = synth.sky_fibonacci(1024)
    np.testing.assert_allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    assert abs(s.mean(axis=0)).max() < 1e-2


def test_named_workload_sizes():
    w = synth.workload("sky-100hz")
    assert w.pm.n_fft == 3140 and w.grid.ns == 118 and w.grid.nf == 81920
    assert 1.9e6 < w.pm.n_peaks < 2.1e6
