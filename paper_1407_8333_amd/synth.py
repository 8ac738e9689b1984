"""Seeded synthetic workloads for the frequency-Hough (FH) path.

This module only *draws inputs*: time-frequency peakmaps, detector velocities,
sky directions, weights and search grids.  It holds none of the FH arithmetic
(no Doppler correction of peaks, no stripe mapping, no histogram).  Both the
CPU oracle and the GPU library consume what it produces.

What it models, and where the paper defines it:

* Peakmap (Sec. "Peakmap", Eq. pm): per FFT, the equalised spectrum R is
  Exp(1) distributed in Gaussian noise; a peak is a bin that is above the
  threshold theta AND a strict local maximum.  Noise-peak probability is
  Eq. p0, p0 = e^-t - e^-2t + e^-3t/3 (0.0755 at theta = 2.5).
* Signal bins follow the normalised non-central chi^2 with 2 dof (Eq.
  noncenchi2): R = ((g1 + sqrt(lambda))^2 + g2^2)/2, mean 1 + lambda/2,
  variance 1 + lambda.
* SFDB (Sec. "Short FFT Data Base"): FFTs of length T_FFT interlaced by half,
  so FFT i starts at t_i = i*T_FFT/2; the peak time tag is the FFT start.
* Signal frequency at the detector: Eq. sd (first-order spin-down) times the
  Doppler factor of Eq. fdopp, f(t) = (f0 + fdot (t - t0)) (1 + v.n).
* Detector velocity (units of c): annual term 1e-4 (Eq. fv scale) in the
  ecliptic, tilted by the obliquity into equatorial axes, plus a daily term of
  1.5e-6 (the Earth-rotation Doppler quoted in the cleaning section,
  1.9e-4 Hz at 128 Hz).
* Grids (Sec. "Coarse grid in the parameter space"): delta_f = 1/T_FFT,
  K_f = 10 fine bins per natural bin (Eq. freqres), spin-down step
  delta_f / T_obs with K_fdot = 1 (Eq. sdstep), t0 at mid-observation.

All draws use numpy ``Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

YEAR_S = 365.25 * 86400.0
SIDEREAL_DAY_S = 86164.0905
OBLIQUITY = math.radians(23.44)
V_ORB = 1.0e-4  # |v_orb|/c
V_ROT = 1.5e-6  # |v_rot|/c at mid latitude


@dataclasses.dataclass
class Peakmap:
    """CSR time-frequency peakmap: FFT i owns bins[offsets[i]:offsets[i+1]]."""

    t_fft: float            # FFT length T_FFT [s]
    t: np.ndarray           # [N] float64, FFT start times [s]
    v: np.ndarray           # [N, 3] float64, detector velocity / c (equatorial)
    offsets: np.ndarray     # [N + 1] int64
    bins: np.ndarray        # [P] int32, original bin index k (f = k / T_FFT), ascending per FFT
    k_lo: int = 0           # first natural bin that was drawn
    k_hi: int = 0           # one past the last natural bin that was drawn

    @property
    def n_fft(self) -> int:
        return int(self.t.shape[0])

    @property
    def n_peaks(self) -> int:
        return int(self.bins.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset_ffts(self, idx) -> "Peakmap":
        """Peakmap restricted to the FFTs listed in ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        segs = [self.bins[self.offsets[i]:self.offsets[i + 1]] for i in idx]
        cnt = np.array([len(s) for s in segs], dtype=np.int64)
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(cnt, out=off[1:])
        bins = np.concatenate(segs).astype(np.int32) if segs else np.zeros(0, np.int32)
        return Peakmap(self.t_fft, self.t[idx].copy(), self.v[idx].copy(), off, bins,
                       self.k_lo, self.k_hi)


@dataclasses.dataclass
class Grid:
    """Search grid of one Hough map: fine frequency bins x spin-down rows.

    Fine bin b (0 <= b < nf) has label f0 = (b0 + b) / (kf * T_FFT);
    row s (0 <= s < ns) has spin-down fdot0 + s * dfdot; t0 is the reference time.
    """

    kf: int
    b0: int
    nf: int
    ns: int
    fdot0: float
    dfdot: float
    t0: float


@dataclasses.dataclass
class Selection:
    """Candidate selection: sub-bands of ``width`` fine bins, second-order
    candidates searched outside +-excl of the first and kept when at least
    ``sep`` bins away (Sec. "Selection of first level candidates")."""

    width: int
    excl: int = 4
    sep: int = 8
    theta: float = 2.5


@dataclasses.dataclass
class Injection:
    f0: float
    fdot: float
    nhat: np.ndarray
    lam: float = 0.0


# ----------------------------------------------------------------------------
# elementary draws


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def fft_times(n_fft: int, t_fft: float, t_start: float = 0.0) -> np.ndarray:
    """Start times of N FFTs interlaced by half."""
    return t_start + np.arange(n_fft, dtype=np.float64) * (0.5 * t_fft)


def detector_velocity(t: np.ndarray, rng: Optional[np.random.Generator],
                      scale_orb: float = V_ORB, scale_rot: float = V_ROT,
                      phases=None) -> np.ndarray:
    """Annual + daily sinusoidal detector velocity in units of c, equatorial axes."""
    if phases is None:
        phases = rng.uniform(0.0, 2.0 * np.pi, size=2)
    po, ps = phases
    wo = 2.0 * np.pi / YEAR_S
    ws = 2.0 * np.pi / SIDEREAL_DAY_S
    a = wo * t + po
    d = ws * t + ps
    v = np.empty((t.shape[0], 3), dtype=np.float64)
    v[:, 0] = -scale_orb * np.sin(a) - scale_rot * np.sin(d)
    v[:, 1] = scale_orb * math.cos(OBLIQUITY) * np.cos(a) + scale_rot * np.cos(d)
    v[:, 2] = scale_orb * math.sin(OBLIQUITY) * np.cos(a)
    return v


def sky_uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """n unit vectors drawn uniformly on the sphere."""
    x = rng.standard_normal((n, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def sky_fibonacci(n: int) -> np.ndarray:
    """Near-isotropic grid of n directions (Fibonacci lattice)."""
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = j * (np.pi * (3.0 - math.sqrt(5.0)))
    x = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def fft_weights(n_fft: int, rng: np.random.Generator, lo=0.5, hi=1.5) -> np.ndarray:
    """Per-FFT adaptive weights drawn U(lo, hi), stored as float32."""
    return rng.uniform(lo, hi, size=n_fft).astype(np.float32)


# ----------------------------------------------------------------------------
# peakmaps


def _local_max_peaks(R: np.ndarray, theta: float):
    """Rows of R with one guard bin on each side -> (row, col) of the peaks."""
    c = R[:, 1:-1]
    m = (c > theta) & (c > R[:, :-2]) & (c > R[:, 2:])
    return np.nonzero(m)


def signal_track_bins(t: np.ndarray, v: np.ndarray, t_fft: float, inj: Injection,
                      t0: float) -> np.ndarray:
    """Natural bin holding the signal in each FFT (Eqs. sd and fdopp)."""
    fsrc = inj.f0 + inj.fdot * (t - t0)
    fdet = fsrc * (1.0 + v @ np.asarray(inj.nhat, dtype=np.float64))
    return np.rint(fdet * t_fft).astype(np.int64), fdet * t_fft


def make_noise_peakmap(n_fft: int, t_fft: float, k_lo: int, k_hi: int, seed: int,
                       theta: float = 2.5, velocity: str = "annual+daily",
                       injections=(), t0: Optional[float] = None,
                       chunk_cells: int = 1 << 24) -> Peakmap:
    """Gaussian-noise peakmap over natural bins [k_lo, k_hi) with optional signals.

    velocity: "annual+daily" (default) or "none" (v = 0).
    Each injection replaces, in every FFT, the equalised power of the bin that
    holds the signal with a non-central chi^2 draw of parameter lambda.
    """
    rng = rng_for(seed)
    t = fft_times(n_fft, t_fft)
    if velocity == "none":
        v = np.zeros((n_fft, 3))
    else:
        v = detector_velocity(t, rng)
    if t0 is None:
        t0 = 0.5 * (t[0] + t[-1])
    nb = k_hi - k_lo
    tracks = [signal_track_bins(t, v, t_fft, inj, t0)[0] for inj in injections]
    rows_per = max(1, chunk_cells // (nb + 2))
    counts = np.zeros(n_fft, dtype=np.int64)
    chunks = []
    for i0 in range(0, n_fft, rows_per):
        i1 = min(n_fft, i0 + rows_per)
        R = rng.standard_exponential((i1 - i0, nb + 2), dtype=np.float32)
        for inj, kt in zip(injections, tracks):
            col = kt[i0:i1] - (k_lo - 1)
            ok = (col >= 0) & (col < nb + 2)
            rows = np.nonzero(ok)[0]
            g = rng.standard_normal((rows.size, 2))
            R[rows, col[ok]] = (((g[:, 0] + math.sqrt(inj.lam)) ** 2 + g[:, 1] ** 2) * 0.5
                                ).astype(np.float32)
        r, c = _local_max_peaks(R, theta)
        counts[i0:i1] = np.bincount(r, minlength=i1 - i0)
        chunks.append((c + k_lo).astype(np.int32))
    offsets = np.zeros(n_fft + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    bins = np.concatenate(chunks) if chunks else np.zeros(0, np.int32)
    return Peakmap(float(t_fft), t, v, offsets, bins, k_lo, k_hi)


def make_track_peakmap(t: np.ndarray, v: np.ndarray, t_fft: float, injections,
                       t0: float) -> Peakmap:
    """Noiseless peakmap: only the bins holding each injected signal."""
    per = [signal_track_bins(t, v, t_fft, inj, t0)[0] for inj in injections]
    n = t.shape[0]
    segs = []
    for i in range(n):
        segs.append(np.unique(np.array([p[i] for p in per], dtype=np.int64)))
    counts = np.array([s.size for s in segs], dtype=np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    bins = np.concatenate(segs).astype(np.int32)
    return Peakmap(float(t_fft), t.copy(), v.copy(), offsets, bins,
                   int(bins.min()) if bins.size else 0, int(bins.max()) + 1 if bins.size else 0)


def track_is_clean(t, v, t_fft, inj: Injection, t0: float, margin: float = 1e-3) -> bool:
    """True when, in every FFT, the signal sits at least ``margin`` natural bins
    away from a bin edge, so that rounding to the natural bin is unambiguous."""
    _, x = signal_track_bins(t, v, t_fft, inj, t0)
    frac = x - np.floor(x)
    return bool(np.all(np.abs(frac - 0.5) > margin))


def random_peakmap(n_fft: int, t_fft: float, k_lo: int, k_hi: int, density: float,
                   rng: np.random.Generator, velocity_scale: float = 1.0,
                   t_start: float = 0.0, min_gap: int = 2) -> Peakmap:
    """Small random peakmap for tests: each bin is a peak with prob ``density``,
    then peaks closer than ``min_gap`` natural bins are thinned (local maxima are
    never adjacent)."""
    t = fft_times(n_fft, t_fft, t_start)
    v = detector_velocity(t, rng) * velocity_scale
    segs = []
    for _ in range(n_fft):
        ks = np.nonzero(rng.random(k_hi - k_lo) < density)[0] + k_lo
        keep = []
        last = None
        for k in ks:
            if last is None or k - last >= min_gap:
                keep.append(k)
                last = k
        segs.append(np.array(keep, dtype=np.int64))
    counts = np.array([s.size for s in segs], dtype=np.int64)
    offsets = np.zeros(n_fft + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    bins = (np.concatenate(segs) if segs else np.zeros(0)).astype(np.int32)
    return Peakmap(float(t_fft), t, v, offsets, bins, k_lo, k_hi)


# ----------------------------------------------------------------------------
# grids


def spin_down_rows(fdot_min: float, fdot_max: float, dfdot: float):
    """Rows anchored at fdot = 0: s in [floor(min/step), ceil(max/step)]."""
    s_min = math.floor(fdot_min / dfdot)
    s_max = math.ceil(fdot_max / dfdot)
    return s_min, s_max - s_min + 1


def make_grid(pm: Peakmap, f_lo: float, f_hi: float, fdot_min: float, fdot_max: float,
              kf: int = 10, t0: Optional[float] = None) -> Grid:
    """Coarse grid for band [f_lo, f_hi): K_f fine bins per natural bin and
    K_fdot = 1 spin-down rows of step delta_f / T_obs, T_obs = N T_FFT / 2."""
    t_fft = pm.t_fft
    t_obs = pm.n_fft * t_fft * 0.5
    dfdot = (1.0 / t_fft) / t_obs
    s_min, ns = spin_down_rows(fdot_min, fdot_max, dfdot)
    b0 = int(round(f_lo * kf * t_fft))
    nf = int(round((f_hi - f_lo) * kf * t_fft))
    if t0 is None:
        t0 = 0.5 * (float(pm.t[0]) + float(pm.t[-1]))
    return Grid(kf=kf, b0=b0, nf=nf, ns=ns, fdot0=s_min * dfdot, dfdot=dfdot, t0=t0)


def band_margin_bins(f_hi: float, t_fft: float, n_fft: int, fdot_abs_max: float,
                     v_max: float = V_ORB + V_ROT) -> int:
    """Natural bins needed beyond the band so that every peak whose corrected
    stripe can land in the band is present (Doppler + spin-down drift + 1)."""
    tau_max = 0.5 * n_fft * t_fft * 0.5 + t_fft
    return int(math.ceil((f_hi * v_max * 1.02 + fdot_abs_max * tau_max) * t_fft)) + 2


# ----------------------------------------------------------------------------
# named workloads (sizes follow the SFDB tables and the 1-yr FFT counts)


@dataclasses.dataclass
class Workload:
    name: str
    pm: Peakmap
    grid: Grid
    sky: np.ndarray          # [n_sky, 3]
    weights: Optional[np.ndarray]  # [N] float32 or None
    sel: Selection
    injections: list


def _band_peakmap(n_fft, t_fft, f_lo, f_hi, fdot_min, fdot_max, seed, velocity="annual+daily",
                  injections=()):
    m = band_margin_bins(f_hi, t_fft, n_fft, max(abs(fdot_min), abs(fdot_max)),
                         v_max=0.0 if velocity == "none" else V_ORB + V_ROT)
    k_lo = int(math.floor(f_lo * t_fft)) - m
    k_hi = int(math.ceil(f_hi * t_fft)) + m
    return make_noise_peakmap(n_fft, t_fft, k_lo, k_hi, seed, velocity=velocity,
                              injections=injections)


def workload(name: str, seed: int = 1234, n_sky: Optional[int] = None,
             n_fft: Optional[int] = None) -> Workload:
    """Named synthetic workloads.

    plain-50hz   : 1 sky, v = 0, T_FFT 8192 s, 200 FFTs, 50.0-50.1 Hz, one signal.
    sky-100hz    : 1 random sky, T_FFT 8192 s, 3140 FFTs, 100-101 Hz, weights.
    batch-256hz  : Fibonacci sky grid (1024), T_FFT 4096 s, 6300 FFTs, 256-257 Hz,
                   weights, 0.1 Hz sub-bands.
    large-1024hz : Fibonacci sky grid (4096), T_FFT 1024 s, 25000 FFTs,
                   1024-1034 Hz, weights, 100 signals.
    """
    rng = rng_for(seed + 17)
    if name == "plain-50hz":
        n = n_fft or 200
        t_fft = 8192.0
        t = fft_times(n, t_fft)
        t0 = 0.5 * (t[0] + t[-1])
        inj = Injection(50.05, -5e-10, np.array([1.0, 0.0, 0.0]), lam=1.19)
        pm = _band_peakmap(n, t_fft, 50.0, 50.1, -1e-9, 1e-10, seed, velocity="none",
                           injections=[inj])
        grid = make_grid(pm, 50.0, 50.1, -1e-9, 1e-10, t0=t0)
        return Workload(name, pm, grid, np.array([[0.0, 0.0, 1.0]]), None,
                        Selection(width=int(round(0.01 * 10 * t_fft))), [inj])
    if name == "sky-100hz":
        n = n_fft or 3140
        t_fft = 8192.0
        pm = _band_peakmap(n, t_fft, 100.0, 101.0, -1e-9, 1e-10, seed)
        grid = make_grid(pm, 100.0, 101.0, -1e-9, 1e-10)
        sky = sky_uniform(n_sky or 1, rng)
        return Workload(name, pm, grid, sky, fft_weights(n, rng),
                        Selection(width=int(round(0.1 * 10 * t_fft))), [])
    if name == "batch-256hz":
        n = n_fft or 6300
        t_fft = 4096.0
        pm = _band_peakmap(n, t_fft, 256.0, 257.0, -1e-8, 1e-9, seed)
        grid = make_grid(pm, 256.0, 257.0, -1e-8, 1e-9)
        sky = sky_fibonacci(n_sky or 1024)
        return Workload(name, pm, grid, sky, fft_weights(n, rng),
                        Selection(width=int(round(0.1 * 10 * t_fft))), [])
    if name == "large-1024hz":
        n = n_fft or 25000
        t_fft = 1024.0
        ninj = 100
        t = fft_times(n, t_fft)
        t0 = 0.5 * (t[0] + t[-1])
        injs = []
        for _ in range(ninj):
            injs.append(Injection(float(rng.uniform(1024.05, 1033.95)),
                                  float(rng.uniform(-1e-8, 1e-9)),
                                  sky_uniform(1, rng)[0], lam=1.0))
        pm = _band_peakmap(n, t_fft, 1024.0, 1034.0, -1e-8, 1e-9, seed, injections=injs)
        grid = make_grid(pm, 1024.0, 1034.0, -1e-8, 1e-9, t0=t0)
        sky = sky_fibonacci(n_sky or 4096)
        return Workload(name, pm, grid, sky, fft_weights(n, rng),
                        Selection(width=int(round(0.1 * 10 * t_fft))), injs)
    raise KeyError(name)
