"""Pure-Python cell-major frequency-Hough map -- TEST INFRASTRUCTURE ONLY.

For tiny inputs only.  It evaluates, for every cell (row s, fine bin b) of the
map, which peaks' stripes contain the cell label, with the same fixed-point
definition as the C oracle but organised the other way round (cell-major
instead of peak-major) and written independently in Python floats/ints, which
are IEEE binary64 with round-half-even ``round`` and exact ``math.floor``.

Definitions (Eqs. fdopp, uno, due, ncount, ncountadap, freqres, sdstep), with
Q = 2^16 fixed-point steps per fine bin:
  S = (K_f T_FFT) Q; G_is = rint(((fdot0 + s dfdot) tau_i) S)   (row s)
  r_i = 1 / (1 + ((v_x n_x + v_y n_y) + v_z n_z))
  X = floor((K_f k r_i) Q); L_s = X - b0 Q - K_f Q/2 - G_is
  cell (s, b) counts the peak iff L_s <= b Q < L_s + K_f Q
"""
from __future__ import annotations

import math

QD = 65536.0
QI = 1 << 16


def _row_shift(t_i, t0, t_fft, kf, fdot0, dfdot, s):
    tau = t_i - t0
    S = (float(kf) * t_fft) * QD
    fs = fdot0 + float(s) * dfdot
    return round((fs * tau) * S)


def _inv_doppler(vi, n):
    d = 1.0 + ((vi[0] * n[0] + vi[1] * n[1]) + vi[2] * n[2])
    return 1.0 / d


def hough_map_cells(pm, grid, nhat, weights=None):
    """Cell-major map as a list of lists of floats."""
    n = [float(x) for x in nhat]
    kf, b0, nf, ns = int(grid.kf), int(grid.b0), int(grid.nf), int(grid.ns)
    peaks = []  # (X, FFT, w)
    for i in range(pm.t.shape[0]):
        r = _inv_doppler([float(x) for x in pm.v[i]], n)
        w = 1.0 if weights is None else float(weights[i])
        for p in range(int(pm.offsets[i]), int(pm.offsets[i + 1])):
            k = int(pm.bins[p])
            X = math.floor((float(kf * k) * r) * QD)
            peaks.append((X, i, w))
    out = []
    for s in range(ns):
        shift = [_row_shift(float(pm.t[i]), float(grid.t0), float(pm.t_fft), kf, float(grid.fdot0),
                            float(grid.dfdot), s) for i in range(pm.t.shape[0])]
        row = []
        for b in range(nf):
            lab = b * QI
            acc = 0.0
            for X, i, w in peaks:
                L = X - b0 * QI - kf * (QI // 2) - shift[i]
                if L <= lab < L + kf * QI:
                    acc += w
            row.append(acc)
        out.append(row)
    return out


def stripe_float_membership(pm, grid, nhat, s, b, i, k):
    """Signed distance (in fine bins) of cell label (s, b) from the open stripe
    of peak (i, k) in plain floating point, straight from Eq. due with the
    stripe width delta_f: positive inside, negative outside."""
    n = [float(x) for x in nhat]
    vi = [float(x) for x in pm.v[i]]
    d = 1.0 + (vi[0] * n[0] + vi[1] * n[1] + vi[2] * n[2])
    t_fft = float(pm.t_fft)
    df = 1.0 / t_fft
    dfh = df / grid.kf
    f_corr = (k * df) / d
    tau = float(pm.t[i]) - float(grid.t0)
    fdot = grid.fdot0 + s * grid.dfdot
    f0_label = (grid.b0 + b) * dfh
    lo = f_corr - fdot * tau - df / 2.0
    hi = f_corr - fdot * tau + df / 2.0
    return min(f0_label - lo, hi - f0_label) / dfh
