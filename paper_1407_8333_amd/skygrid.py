"""Sky grids in ecliptic coordinates.

* Coarse grid (Sec. "Grid in the sky", Eqs. gammalong, gammalat, ND, and the
  appendix on the construction of the coarse sky grid): the resolution along
  the ecliptic longitude is 1 / (N_D cos beta) and along the latitude
  1 / (N_D sin beta), N_D = f0 Omega_orb R_orb T_FFT / c being the number of
  frequency bins in the maximum orbital Doppler band.  Latitudes start at the
  pole and step by K / (N_D sin beta) with the largest K <= 1 that lands on
  the ecliptic equator; each latitude ring holds the fewest equally spaced
  longitudes whose spacing does not exceed 1 / (N_D cos beta).
* Refined grid around a candidate (Sec. "Refined grid in the sky"): a
  K_hat x K_hat rectangle in (lambda, beta) centred on the candidate, with
  steps of the coarse spacings divided by K_hat.

Directions are returned as equatorial unit vectors (the frame of the detector
velocity), rotating the ecliptic frame by the obliquity about the x axis.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

OBLIQUITY = math.radians(23.44)
# Earth's mean orbital speed over c: 2 pi (1 au) / (1 sidereal year) / c
V_ORB_OVER_C = 2.0 * math.pi * 1.495978707e11 / (365.25636 * 86400.0) / 299792458.0


def doppler_bins(f0: float, t_fft: float) -> float:
    """N_D of Eq. ND: frequency bins of width 1/T_FFT in the orbital Doppler
    band f0 Omega_orb R_orb / c."""
    return f0 * V_ORB_OVER_C * t_fft


def _descend(n_d: float, k: float, steps: int) -> float:
    b = 0.5 * math.pi
    for _ in range(steps):
        b = b - k / (n_d * math.sin(b))
        if b <= 0.0:
            return b
    return b


def latitudes(n_d: float) -> tuple[np.ndarray, float]:
    """Ring latitudes from the north pole to the south pole (N odd, the
    equator in the middle) and the constant K of the recurrence
    beta_i = beta_{i-1} - K / (N_D sin beta_{i-1})."""
    if not n_d > 0:
        raise ValueError("N_D must be positive")
    # steps needed at K = 1 to reach or pass the equator
    b, m = 0.5 * math.pi, 0
    while b > 0.0:
        b = b - 1.0 / (n_d * math.sin(b))
        m += 1
    # the largest K <= 1 whose m-th iterate is exactly 0 (the m-th iterate
    # decreases monotonically with K): bisection
    lo, hi = 0.0, 1.0
    if _descend(n_d, 1.0, m) == 0.0:
        lo = 1.0
    else:
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _descend(n_d, mid, m) > 0.0:
                lo = mid
            else:
                hi = mid
    k = lo
    north = [0.5 * math.pi]
    b = 0.5 * math.pi
    for _ in range(m - 1):
        b = b - k / (n_d * math.sin(b))
        north.append(b)
    north.append(0.0)
    north = np.array(north)
    return np.concatenate([north, -north[-2::-1]]), k


def ring_sizes(beta: np.ndarray, n_d: float) -> np.ndarray:
    """Longitudes per ring: the fewest n with 2 pi / n <= 1 / (N_D cos beta),
    i.e. spacing H / (N_D cos beta) with the largest H <= 1 that divides
    2 pi (one point at a pole)."""
    c = np.abs(np.cos(beta))
    n = np.ceil(2.0 * math.pi * n_d * c - 1e-9).astype(np.int64)
    n[np.abs(beta) >= 0.5 * math.pi - 1e-12] = 1
    return np.maximum(n, 1)


@dataclasses.dataclass
class SkyGrid:
    lam: np.ndarray      # ecliptic longitude [rad]
    beta: np.ndarray     # ecliptic latitude [rad]
    dlam: np.ndarray     # longitude spacing of the point's ring [rad]
    dbeta: np.ndarray    # latitude distance to the adjacent ring towards the equator [rad]
    n_d: float
    k: float             # latitude constant K

    def __len__(self) -> int:
        return len(self.lam)

    def nhat(self) -> np.ndarray:
        return ecliptic_to_equatorial(self.lam, self.beta)


def coarse_grid(f0: float, t_fft: float, k_sky: float = 1.0) -> SkyGrid:
    """Coarse sky grid for maximum frequency f0 and FFT length T_FFT; the
    over-resolution K_sky scales the point count (both spacings by
    1/sqrt(K_sky))."""
    n_d = doppler_bins(f0, t_fft) * math.sqrt(k_sky)
    beta, k = latitudes(n_d)
    n = ring_sizes(beta, n_d)
    nr = len(beta)
    mid = nr // 2
    # distance to the adjacent ring towards the equator (the equator ring
    # takes its neighbour's)
    db = np.empty(nr)
    for i in range(nr):
        j = i + 1 if i < mid else (i - 1 if i > mid else i + 1)
        db[i] = abs(beta[i] - beta[j])
    lam = np.concatenate([np.arange(m) * (2.0 * math.pi / m) for m in n])
    bet = np.repeat(beta, n)
    dlam = np.repeat(2.0 * math.pi / n, n)
    dbet = np.repeat(db, n)
    return SkyGrid(lam, bet, dlam, dbet, n_d, k)


def ecliptic_to_equatorial(lam, beta) -> np.ndarray:
    lam = np.asarray(lam, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    x = np.cos(beta) * np.cos(lam)
    ye = np.cos(beta) * np.sin(lam)
    ze = np.sin(beta)
    ce, se = math.cos(OBLIQUITY), math.sin(OBLIQUITY)
    n = np.stack([x, ye * ce - ze * se, ye * se + ze * ce], axis=-1)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def refined_points(lam_c: float, beta_c: float, dlam: float, dbeta: float, k_hat: int):
    """The K_hat x K_hat refined directions around a candidate (K_hat odd,
    N_layers = (K_hat - 1) / 2 layers on each side): longitudes
    lam_c + i dlam / K_hat and latitudes beta_c + j dbeta / K_hat,
    i, j = -N_layers .. N_layers (latitudes folded back into [-pi/2, pi/2]).
    Returns (lam, beta), row-major over (j, i)."""
    if k_hat < 1 or k_hat % 2 == 0:
        raise ValueError("K_hat must be a positive odd number")
    L = (k_hat - 1) // 2
    off = np.arange(-L, L + 1, dtype=np.float64)
    bb, ll = np.meshgrid(beta_c + off * (dbeta / k_hat), lam_c + off * (dlam / k_hat), indexing="ij")
    bb = bb.ravel()
    ll = ll.ravel()
    over = np.abs(bb) > 0.5 * math.pi
    ll = np.where(over, ll + math.pi, ll)
    bb = np.where(over, np.sign(bb) * math.pi - bb, bb)
    return np.mod(ll, 2.0 * math.pi), bb
