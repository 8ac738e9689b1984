"""Thresholds and significance of Hough candidates (Sec. "Search
sensitivity estimation" and Table III): host-side closed forms for choosing
the peakmap and candidate thresholds of a search."""
from __future__ import annotations

import math


def p0(theta: float) -> float:
    """Probability that a bin of Exp(1) noise is a local maximum above theta
    (Eq. p0): e^-t - e^-2t + e^-3t / 3."""
    return math.exp(-theta) - math.exp(-2.0 * theta) + math.exp(-3.0 * theta) / 3.0


def hough_mean_std(n_fft: int, p: float):
    """Binomial mean and standard deviation of a noise-only map cell (Eq.
    houghmean)."""
    return n_fft * p, math.sqrt(n_fft * p * (1.0 - p))


def critical_ratio(n: float, n_fft: int, theta: float = 2.5) -> float:
    """CR = (n - N p0) / sqrt(N p0 (1 - p0)) of a number count n."""
    mu, sd = hough_mean_std(n_fft, p0(theta))
    return (n - mu) / sd


def false_alarm_of_candidates(n_cand: float, n_tot: float) -> float:
    """P_fa = N_cand / N_tot (Eq. pfa_cand): the fraction of the parameter
    space's points kept as candidates."""
    if not (0 < n_cand <= n_tot):
        raise ValueError("need 0 < n_cand <= n_tot")
    return n_cand / n_tot


def _erfcinv(y: float) -> float:
    """Inverse of math.erfc on (0, 2) by bisection on the monotone erfc
    (60 halvings of a bracket of width 20: below double resolution)."""
    if not (0.0 < y < 2.0):
        raise ValueError("erfc^-1 needs 0 < y < 2")
    lo, hi = -10.0, 10.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if math.erfc(mid) > y:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def cr_threshold(p_fa: float) -> float:
    """Critical-ratio threshold of a false-alarm probability (Eq. crthr):
    CR_thr = sqrt(2) erfc^-1(2 P_fa)."""
    return math.sqrt(2.0) * _erfcinv(2.0 * p_fa)


def n_threshold(n_fft: int, p_fa: float, theta: float = 2.5, sqrt2: bool = True, p=None) -> float:
    """Number-count threshold of a false-alarm probability, Gaussian
    approximation (Eq. nthr_gauss): N p0 + c sqrt(N p0 (1 - p0)) erfc^-1(2 P_fa)
    with c = sqrt(2) as printed.  The n_thr column of Table III follows
    c = 1 (the form consistent with Eq. crthr); pass sqrt2=False for it.
    p overrides p0(theta)."""
    q = p0(theta) if p is None else p
    c = math.sqrt(2.0) if sqrt2 else 1.0
    return n_fft * q + c * math.sqrt(n_fft * q * (1.0 - q)) * _erfcinv(2.0 * p_fa)


def false_alarm_of_threshold(n_thr: float, n_fft: int, theta: float = 2.5, p=None) -> float:
    """P_fa = erfc((n_thr - N p0) / sqrt(2 N p0 (1 - p0))) / 2 (Gaussian
    approximation of the binomial tail above n_thr)."""
    q = p0(theta) if p is None else p
    return 0.5 * math.erfc((n_thr - n_fft * q) / math.sqrt(2.0 * n_fft * q * (1.0 - q)))
