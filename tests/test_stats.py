"""Threshold helpers of the package against the numbers the paper prints
(Table III, Eqs. p0, houghmean, crthr, nthr_gauss; tests/golden/paper_values.txt)."""
import math
import os

import pytest

from paper_1407_8333_amd import stats


def _golden():
    g = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")):
        if line.startswith("#") or "|" not in line:
            continue
        name, value, _ = [x.strip() for x in line.split("|", 2)]
        g[name] = [float(v) for v in value.split(",")]
    return g


G = _golden()


def test_p0_and_cell_statistics():
    assert stats.p0(2.5) == pytest.approx(G["p0_theta_2.5"][0], abs=5e-5)
    mu, sd = stats.hough_mean_std(int(G["n_fft_1yr_1024s"][0]), G["p0_theta_2.5"][0])
    assert mu == pytest.approx(G["hough_mean_N61594"][0], abs=0.05)
    assert sd == pytest.approx(G["hough_std_N61594"][0], abs=0.05)


def test_table3_thresholds():
    q = G["p0_theta_2.5"][0]
    for n, pfa, nthr, cr in zip(G["table3_n_fft"], G["table3_pfa"], G["table3_nthr"], G["table3_crthr"]):
        assert stats.cr_threshold(pfa) == pytest.approx(cr, abs=0.006)
        assert stats.n_threshold(int(n), pfa, sqrt2=False, p=q) == pytest.approx(nthr, abs=0.6)
        # with the printed sqrt(2), the count threshold is the CR threshold in
        # counts (the column itself is smaller by that factor on sigma)
        mu, sd = stats.hough_mean_std(int(n), q)
        assert stats.n_threshold(int(n), pfa, sqrt2=True, p=q) == pytest.approx(
            mu + stats.cr_threshold(pfa) * sd, rel=1e-12)


def test_inverses_and_limits():
    for pfa in [1e-3, 5e-9, 0.25]:
        thr = stats.n_threshold(7699, pfa, sqrt2=True)
        assert stats.false_alarm_of_threshold(thr, 7699) == pytest.approx(pfa, rel=1e-9)
    assert stats.cr_threshold(0.5) == pytest.approx(0.0, abs=1e-12)
    assert stats.cr_threshold(0.158655253931457) == pytest.approx(1.0, abs=1e-9)  # 1-sigma tail
    assert stats.false_alarm_of_candidates(1e6, 2e17) == 5e-12
    mu, sd = stats.hough_mean_std(61594, stats.p0(2.5))
    assert stats.critical_ratio(mu + 2 * sd, 61594) == pytest.approx(2.0, rel=1e-12)
    with pytest.raises(ValueError):
        stats.cr_threshold(0.0)
    with pytest.raises(ValueError):
        stats.false_alarm_of_candidates(0, 10)
    assert math.isfinite(stats.cr_threshold(1e-300))
