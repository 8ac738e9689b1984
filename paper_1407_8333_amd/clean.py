"""Peakmap cleaning on the device (Sec. "Removal of time and frequency domain
disturbances"): the wandering-line veto on the gross histogram, the
persistency veto with the robust statistic (appendix "Robust statistic"), and
the line finder that runs the Hough map without Doppler correction.  Thin
wrappers over the library; the arithmetic runs in its kernels."""
from __future__ import annotations

import ctypes
import math
import numpy as np
import torch

from . import _lib
from ._lib import check
from .api import Context, DevicePeakmap, _stream, grid_struct


def gross_geometry(t, k_lo: int, k_hi: int, dt_h: float, df_h: float, t_fft: float):
    """Gross cells (t_origin, dt_h, n_t, df_h, c0, n_f) covering FFT times t
    and natural bins [k_lo, k_hi): time cells from the first FFT, frequency
    cells floor(k / (df_h T_FFT)) from that of k_lo."""
    t = np.asarray(t, dtype=np.float64)
    t0 = float(t.min())
    n_t = int(math.floor((float(t.max()) - t0) / dt_h)) + 1
    width = df_h * t_fft
    c0 = int(math.floor(float(k_lo) / width))
    return t0, float(dt_h), n_t, float(df_h), c0, int(math.floor(float(k_hi - 1) / width)) - c0 + 1


def gross_expectation(dt_h: float, df_h: float, t_fft: float, p0: float, overlap: float = 0.5):
    """(N, E_H, sigma_H) of a gross cell for a peak probability p0 (FFTs
    interlaced by `overlap`)."""
    n = dt_h / (t_fft * (1.0 - overlap)) * (df_h * t_fft)
    return n, n * p0, math.sqrt(n * p0 * (1.0 - p0))


def _geo(geo) -> _lib.fh_gross:
    t0, dt_h, n_t, df_h, c0, n_f = geo
    return _lib.fh_gross(float(t0), float(dt_h), float(df_h), int(c0), int(n_t), int(n_f))


def gross_histogram(ctx: Context, dpm: DevicePeakmap, geo, stream=None) -> torch.Tensor:
    """int32 [n_t, n_f] peaks per gross cell (fh_gross_histogram)."""
    g = _geo(geo)
    h = torch.empty((g.n_t, g.n_f), dtype=torch.int32, device="cuda:%d" % ctx.device)
    check(_lib.fh_gross_histogram(ctx.handle, dpm.handle, ctypes.byref(g), ctypes.c_void_p(h.data_ptr()),
                                  _stream(stream)))
    return h


def clean_gross(ctx: Context, dpm: DevicePeakmap, geo, threshold: float, stream=None):
    """(peakmap without the peaks of cells over threshold, gross histogram)."""
    g = _geo(geo)
    hist = torch.empty((g.n_t, g.n_f), dtype=torch.int32, device="cuda:%d" % ctx.device)
    out = ctypes.c_void_p()
    check(_lib.fh_clean_gross(ctx.handle, dpm.handle, ctypes.byref(g), float(threshold),
                              ctypes.c_void_p(hist.data_ptr()), _stream(stream), ctypes.byref(out)))
    return DevicePeakmap.wrap(ctx, out), hist


def bin_counts(ctx: Context, dpm: DevicePeakmap, k_lo: int, k_hi: int, stream=None) -> torch.Tensor:
    """int32 [k_hi - k_lo]: FFTs holding a peak at each natural bin."""
    c = torch.empty(k_hi - k_lo, dtype=torch.int32, device="cuda:%d" % ctx.device)
    check(_lib.fh_bin_counts(ctx.handle, dpm.handle, int(k_lo), int(k_hi), ctypes.c_void_p(c.data_ptr()),
                             _stream(stream)))
    return c


def robust_stats(ctx: Context, x: torch.Tensor, x_max: int, stream=None):
    """(m1, m2): median and median absolute deviation / 0.6745 of an int32
    device tensor with values in [0, x_max]."""
    assert x.dtype == torch.int32 and x.is_cuda and x.is_contiguous()
    out = (ctypes.c_double * 2)()
    check(_lib.fh_robust_stats(ctx.handle, ctypes.c_void_p(x.data_ptr()), int(x.numel()), int(x_max), out,
                               _stream(stream)))
    return float(out[0]), float(out[1])


def line_counts(ctx: Context, dpm: DevicePeakmap, grid, stream=None) -> torch.Tensor:
    """int32 [nf]: per fine bin, the largest count over the grid's rows of the
    Hough map without Doppler correction."""
    g = grid_struct(grid)
    out = torch.empty(g.nf, dtype=torch.int32, device="cuda:%d" % ctx.device)
    check(_lib.fh_line_counts(ctx.handle, dpm.handle, ctypes.byref(g), ctypes.c_void_p(out.data_ptr()),
                              _stream(stream)))
    return out


def veto_bins(ctx: Context, dpm: DevicePeakmap, k_lo: int, k_hi: int, x: torch.Tensor, step: int,
              offset: int, threshold: float, stream=None) -> DevicePeakmap:
    """Peakmap without the peaks of natural bins k in [k_lo, k_hi) whose
    statistic x[step (k - k_lo) + offset] exceeds threshold."""
    assert x.dtype == torch.int32 and x.is_cuda and x.is_contiguous()
    out = ctypes.c_void_p()
    check(_lib.fh_veto_bins(ctx.handle, dpm.handle, int(k_lo), int(k_hi), ctypes.c_void_p(x.data_ptr()),
                            int(x.numel()), int(step), int(offset), float(threshold), _stream(stream),
                            ctypes.byref(out)))
    return DevicePeakmap.wrap(ctx, out)


def persistency_veto(ctx: Context, dpm: DevicePeakmap, k_lo: int, k_hi: int, kappa: float,
                     stream=None):
    """Constant lines by persistency: bins whose FFT count exceeds
    m1 + kappa m2 are removed.  Returns (peakmap, counts, m1, m2)."""
    c = bin_counts(ctx, dpm, k_lo, k_hi, stream)
    m1, m2 = robust_stats(ctx, c, dpm.n_fft, stream)
    return veto_bins(ctx, dpm, k_lo, k_hi, c, 1, 0, m1 + kappa * m2, stream), c, m1, m2


def line_veto(ctx: Context, dpm: DevicePeakmap, grid, k_lo: int, k_hi: int, threshold: float,
              stream=None):
    """Constant lines by the Hough map without Doppler correction: natural
    bin k is removed when the fine bin K_f k of the map (rows around zero
    spin-down) counts more than threshold.  Returns (peakmap, line counts)."""
    lc = line_counts(ctx, dpm, grid, stream)
    off = grid.kf * k_lo - grid.b0
    return veto_bins(ctx, dpm, k_lo, k_hi, lc, grid.kf, off, threshold, stream), lc

