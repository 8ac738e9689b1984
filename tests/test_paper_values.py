"""Closed forms of the paper against the numbers it prints (tests/golden/paper_values.txt)."""
import math
import os

import numpy as np
import pytest

from oracle import stats


def _golden():
    out = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, value, _ = [x.strip() for x in line.split("|")]
        vals = [float(x) for x in value.split(",")]
        out[name] = vals if len(vals) > 1 else vals[0]
    return out


G = _golden()


def test_p0_at_theta_2_5():
    assert stats.p0(2.5) == pytest.approx(G["p0_theta_2.5"], abs=5e-5)


def test_local_max_reduces_peaks_by_about_9_percent():
    """The printed "about 9 %" matches the plain threshold giving e^-t / p0 - 1
    = 8.7 % more peaks (the local-max count is 8.0 % lower)."""
    more = 100 * (stats.p_plain_threshold(2.5) / stats.p0(2.5) - 1)
    assert more == pytest.approx(G["localmax_reduction_percent"], abs=0.5)
    assert stats.p0(2.5) / stats.p_plain_threshold(2.5) == pytest.approx(0.920, abs=5e-4)


def test_fft_counts_for_one_year():
    assert stats.n_fft_interlaced(365 * 86400.0, 1024.0) == G["n_fft_1yr_1024s"]
    assert stats.n_fft_interlaced(365 * 86400.0, 8192.0) == G["n_fft_1yr_8192s"]


def test_hough_mean_and_std():
    mu, sd = stats.hough_mean_std(int(G["n_fft_1yr_1024s"]), G["p0_theta_2.5"])
    assert mu == pytest.approx(G["hough_mean_N61594"], abs=0.05)
    assert sd == pytest.approx(G["hough_std_N61594"], abs=0.05)


def test_table3_cr_threshold():
    for pfa, cr in zip(G["table3_pfa"], G["table3_crthr"]):
        assert stats.cr_threshold(pfa, 1.0) == pytest.approx(cr, abs=0.006)


def test_table3_nthr_reading():
    """The printed n_thr column follows N p0 + sigma erfc^-1(2 P_fa) with the
    rounded p0 = 0.0755, i.e. Eq. nthr_gauss without its sqrt(2); with the
    sqrt(2) every entry is larger by 40-110 counts."""
    q = G["p0_theta_2.5"]
    for n, pfa, nthr in zip(G["table3_n_fft"], G["table3_pfa"], G["table3_nthr"]):
        assert stats.n_thr(int(n), pfa, sqrt2=False, q=q) == pytest.approx(nthr, abs=0.6)
        assert stats.n_thr(int(n), pfa, sqrt2=True, q=q) > nthr + 30


def test_p_lambda_small_signal_limit():
    """Eq. plambda_approx is the first-order expansion of the exact integral."""
    th = 2.5
    assert stats.p_lambda_paper_integral(th, 1e-9) == pytest.approx(stats.p0(th), rel=1e-6)
    assert stats.p_lambda_exact(th, 1e-9) == pytest.approx(stats.p0(th), rel=1e-6)
    lam = 1e-3
    d_exact = (stats.p_lambda_paper_integral(th, lam) - stats.p0(th)) / lam
    d_approx = (stats.p_lambda_approx(th, lam) - stats.p0(th)) / lam
    assert d_exact == pytest.approx(d_approx, rel=2e-3)
