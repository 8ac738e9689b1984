"""Closed forms of the paper's statistics sections -- TEST INFRASTRUCTURE ONLY.

They pin the synthetic generator and the reading of printed tables; none of
them is on the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def p0(theta: float) -> float:
    """Eq. p0: local maximum above theta in Exp(1) noise."""
    return math.exp(-theta) - math.exp(-2 * theta) + math.exp(-3 * theta) / 3.0


def p_plain_threshold(theta: float) -> float:
    """Probability of exceeding theta without the local-maximum condition."""
    return math.exp(-theta)


def p_lambda_approx(theta: float, lam: float) -> float:
    """Eq. plambda_approx (first order in lambda)."""
    return p0(theta) + 0.5 * lam * theta * (math.exp(-theta) - 2 * math.exp(-2 * theta)
                                            + math.exp(-3 * theta))


def _pdf_signal(x, lam):
    """Eq. noncenchi2, normalised non-central chi^2 with 2 dof."""
    return np.exp(-x - lam / 2.0) * special.i0(np.sqrt(2.0 * x * lam))


def p_lambda_exact(theta: float, lam: float) -> float:
    """Probability that the signal bin is a local max above theta when its two
    neighbours are noise (Exp(1)) -- the model of the synthetic generator."""
    f = lambda x: _pdf_signal(x, lam) * (1.0 - math.exp(-x)) ** 2
    return integrate.quad(f, theta, np.inf, limit=200)[0]


def p_lambda_paper_integral(theta: float, lam: float) -> float:
    """The integral the paper expands into Eq. plambda_approx, in which the two
    neighbouring bins follow the same non-central density as the centre."""
    cdf = lambda x: integrate.quad(lambda y: _pdf_signal(y, lam), 0.0, x)[0]
    f = lambda x: _pdf_signal(x, lam) * cdf(x) ** 2
    return integrate.quad(f, theta, 60.0, limit=200)[0]


def critical_ratio(n, n_fft: int, theta: float = 2.5, q=None):
    """Eq. cr: CR = (n - N p0) / sqrt(N p0 (1 - p0)); q overrides p0(theta)."""
    q = p0(theta) if q is None else q
    return (np.asarray(n, dtype=np.float64) - n_fft * q) / np.sqrt(n_fft * q * (1.0 - q))


def critical_ratio_weighted(n, w_sum: float, w2_sum: float, theta: float = 2.5, q=None):
    """Critical ratio of a weighted count n = sum_i w_i n_i (Eq. ncountadap):
    with independent n_i ~ Bernoulli(p0) in noise, E n = p0 sum w and
    Var n = p0 (1 - p0) sum w^2, so CR = (n - p0 sum w) / sqrt(p0 (1 - p0) sum w^2).
    Unit weights give Eq. cr."""
    q = p0(theta) if q is None else q
    return (np.asarray(n, dtype=np.float64) - q * w_sum) / np.sqrt(q * (1.0 - q) * w2_sum)


def hough_mean_std(n_fft: int, eta: float):
    """Eq. houghmean: binomial mean and standard deviation of a map cell."""
    return n_fft * eta, math.sqrt(n_fft * eta * (1.0 - eta))


def n_thr(n_fft: int, p_fa: float, theta: float = 2.5, sqrt2: bool = True, q=None) -> float:
    """Eq. nthr_gauss (sqrt2=True); sqrt2=False is the reading that reproduces
    the n_thr column of Table III.  q overrides p0(theta)."""
    q = p0(theta) if q is None else q
    c = math.sqrt(2.0) if sqrt2 else 1.0
    return n_fft * q + c * math.sqrt(n_fft * q * (1 - q)) * special.erfcinv(2 * p_fa)


def cr_threshold(n_cand: float, n_tot: float) -> float:
    """Eq. crthr: CR_thr = sqrt(2) erfc^-1(2 N_cand / N_tot)."""
    return math.sqrt(2.0) * special.erfcinv(2.0 * n_cand / n_tot)


def n_fft_interlaced(t_obs: float, t_fft: float) -> int:
    """Number of half-interlaced FFTs in T_obs."""
    return int(round(t_obs / (0.5 * t_fft)))
