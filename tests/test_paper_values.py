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


# ---------------------------------------------------------------------------
# Eq. cr and its weighted form


def test_cr_of_the_printed_mean_and_deviation():
    """Eq. cr with the printed p0 puts the printed mean of the number count at
    CR = 0 and the mean plus one printed deviation at CR = 1 (N = 61594)."""
    n, q = int(G["n_fft_1yr_1024s"]), G["p0_theta_2.5"]
    mu, sd = G["hough_mean_N61594"], G["hough_std_N61594"]
    assert stats.critical_ratio(mu, n, q=q) == pytest.approx(0.0, abs=0.002)
    assert stats.critical_ratio(mu + sd, n, q=q) == pytest.approx(1.0, abs=0.002)
    assert stats.critical_ratio(mu - 2 * sd, n, q=q) == pytest.approx(-2.0, abs=0.004)


def test_cr_of_the_table3_count_thresholds():
    """Table III's n_thr column, read without the sqrt(2) of Eq. nthr_gauss,
    sits at CR = CR_thr / sqrt(2) of the same row (to the integer rounding
    of n_thr: 1/sigma)."""
    q = G["p0_theta_2.5"]
    for n, nthr, crthr in zip(G["table3_n_fft"], G["table3_nthr"], G["table3_crthr"]):
        sigma = math.sqrt(n * q * (1 - q))
        assert stats.critical_ratio(nthr, int(n), q=q) == pytest.approx(crthr / math.sqrt(2.0),
                                                                         abs=1.0 / sigma + 0.01)


def test_weighted_cr_reduces_to_eq_cr_for_unit_weights():
    n = np.array([0.0, 17.0, 75.5, 200.0])
    for n_fft in (1, 200, 61594):
        np.testing.assert_array_equal(stats.critical_ratio_weighted(n, float(n_fft), float(n_fft)),
                                      stats.critical_ratio(n, n_fft))


def test_weighted_cr_is_invariant_to_a_common_weight_scale():
    rng = np.random.default_rng(3)
    w = rng.uniform(0.05, 3.0, 500)
    n = 0.3 * w.sum()
    base = stats.critical_ratio_weighted(n, w.sum(), (w * w).sum())
    for c in (1e-3, 0.5, 7.0, 1e4):
        cw = c * w
        assert stats.critical_ratio_weighted(c * n, cw.sum(), (cw * cw).sum()) == pytest.approx(base, rel=1e-12)


def test_weighted_cr_is_standard_in_noise():
    """Weighted counts n = sum_i w_i n_i with n_i ~ Bernoulli(p0) (a noise-only
    cell of Eq. ncountadap): the weighted CR has mean 0 and deviation 1.
    Weights U(0.05, 3) make sum w^2 differ from sum w, so a variance built
    from sum w (or a mean without p0) would fail."""
    rng = np.random.default_rng(8333)
    q = stats.p0(2.5)
    w = rng.uniform(0.05, 3.0, 3000)
    hits = rng.random((4000, w.size)) < q
    n = hits.astype(np.float64) @ w
    cr = stats.critical_ratio_weighted(n, w.sum(), (w * w).sum())
    assert float(np.mean(cr)) == pytest.approx(0.0, abs=0.05)
    assert float(np.std(cr)) == pytest.approx(1.0, abs=0.03)
    wrong = (n - q * w.sum()) / np.sqrt(q * (1 - q) * w.sum())
    assert abs(float(np.std(wrong)) - 1.0) > 0.2
