"""Python front end of the frequency-Hough library.

Thin wrappers over the C ABI (``_lib``): they marshal numpy / torch arguments
and allocate outputs as torch tensors on the device; every computation runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check

CANDIDATE_FIELDS = ("sky", "subband", "rank", "bin", "row", "value", "cr", "valid")


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def grid_struct(g) -> _lib.fh_grid:
    return _lib.fh_grid(int(g.kf), int(g.b0), int(g.nf), int(g.ns), float(g.fdot0),
                        float(g.dfdot), float(g.t0))


def select_struct(sel) -> _lib.fh_select:
    return _lib.fh_select(int(sel.width), int(sel.excl), int(sel.sep), float(sel.theta))


class Context:
    """An fh_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        torch.cuda.set_device(self.device)
        h = ctypes.c_void_p()
        check(_lib.fh_ctx_create(self.device, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.fh_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, stream=None):
        check(_lib.fh_ctx_check(self.handle, _stream(stream)))

    def set_option(self, name: str, value: int):
        check(_lib.fh_ctx_set_option(self.handle, name.encode(), int(value)))

    def set_doppler(self, mode: str = "exact", f_ref: float = 0.0):
        """Doppler correction of later searches: "exact" per peak, or "shift"
        per FFT at f_ref Hz (0: each map's band centre) (fh_ctx_set_doppler)."""
        m = {"exact": 0, "shift": 1}[mode]
        check(_lib.fh_ctx_set_doppler(self.handle, m, float(f_ref)))

    def profile(self, enable: bool):
        check(_lib.fh_ctx_profile(self.handle, 1 if enable else 0))

    def profile_read(self) -> dict:
        p = _lib.fh_profile()
        check(_lib.fh_ctx_profile_read(self.handle, ctypes.byref(p)))
        return {f: getattr(p, f) for f, _ in p._fields_}

    def upload(self, pm, stream=None) -> "DevicePeakmap":
        return DevicePeakmap(self, pm, stream)

    def plan(self, dpm: "DevicePeakmap", grid, tile_bins: int = 0) -> dict:
        info = _lib.fh_plan_info()
        g = grid_struct(grid)
        check(_lib.fh_plan_query(self.handle, dpm.handle, ctypes.byref(g), int(tile_bins),
                                 ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in info._fields_}


class DevicePeakmap:
    """A peakmap resident in device memory (fh_peakmap)."""

    def __init__(self, ctx: Context, pm, stream=None):
        self.ctx = ctx
        self.n_fft = int(pm.t.shape[0])
        self.n_peaks = int(pm.bins.shape[0])
        off = np.ascontiguousarray(pm.offsets, dtype=np.int64)
        bins = np.ascontiguousarray(pm.bins, dtype=np.int32)
        t = np.ascontiguousarray(pm.t, dtype=np.float64)
        v = np.ascontiguousarray(pm.v, dtype=np.float64).reshape(-1, 3)
        d = _lib.fh_peakmap_desc(self.n_fft, self.n_peaks, off.ctypes.data, bins.ctypes.data,
                                 t.ctypes.data, v.ctypes.data, float(pm.t_fft))
        h = ctypes.c_void_p()
        check(_lib.fh_peakmap_upload(ctx.handle, ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_spectra(cls, ctx: Context, sp: torch.Tensor, k0: int, theta: float, t, v, t_fft: float,
                     sar: Optional[torch.Tensor] = None, stream=None) -> "DevicePeakmap":
        """Peakmap of equalised spectra R = sp / sar (Eq. pm) built on the GPU.
        sp, sar: device float32 [n_fft, n_bins]; row bin j is natural bin k0 + j."""
        assert sp.dtype == torch.float32 and sp.is_cuda and sp.dim() == 2 and sp.stride(1) == 1
        if sar is not None:
            assert sar.shape == sp.shape and sar.dtype == torch.float32 and sar.stride() == sp.stride()
        t = np.ascontiguousarray(t, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        self = cls.__new__(cls)
        self.ctx = ctx
        h = ctypes.c_void_p()
        check(_lib.fh_peakmap_from_spectra(ctx.handle, sp.shape[0], sp.shape[1], sp.stride(0),
                                           ctypes.c_void_p(sp.data_ptr()),
                                           None if sar is None else ctypes.c_void_p(sar.data_ptr()),
                                           int(k0), float(theta), t.ctypes.data, v.ctypes.data,
                                           float(t_fft), _stream(stream), ctypes.byref(h)))
        self.handle = h
        n, p = ctypes.c_int32(), ctypes.c_int64()
        check(_lib.fh_peakmap_shape(h, ctypes.byref(n), ctypes.byref(p)))
        self.n_fft, self.n_peaks = n.value, p.value
        return self

    def download(self):
        """(offsets int64 [N+1], bins int32 [P]) on the host."""
        off = np.zeros(self.n_fft + 1, np.int64)
        bins = np.zeros(max(1, self.n_peaks), np.int32)
        check(_lib.fh_peakmap_download(self.ctx.handle, self.handle, off.ctypes.data, bins.ctypes.data))
        return off, bins[: int(off[-1])]

    @classmethod
    def wrap(cls, ctx: "Context", handle) -> "DevicePeakmap":
        """Take ownership of a peakmap handle returned by the library."""
        q = cls.__new__(cls)
        q.ctx = ctx
        q.handle = handle
        n, p = ctypes.c_int32(), ctypes.c_int64()
        check(_lib.fh_peakmap_shape(handle, ctypes.byref(n), ctypes.byref(p)))
        q.n_fft, q.n_peaks = n.value, p.value
        return q

    def slice(self, k_lo: int, k_hi: int, stream=None) -> "DevicePeakmap":
        """The peaks with natural bin in [k_lo, k_hi) (fh_peakmap_slice)."""
        h = ctypes.c_void_p()
        check(_lib.fh_peakmap_slice(self.ctx.handle, self.handle, int(k_lo), int(k_hi), _stream(stream),
                                    ctypes.byref(h)))
        return DevicePeakmap.wrap(self.ctx, h)

    @property
    def nbytes(self) -> int:
        return int(_lib.fh_peakmap_bytes(self.handle))

    def release(self):
        if self.handle:
            torch.cuda.synchronize()
            _lib.fh_peakmap_release(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.release()
        except Exception:
            pass


REFINED_DTYPE = np.dtype([("cand", "<i4"), ("sky", "<i4"), ("bin", "<i4"), ("row", "<i4"),
                          ("value", "<f4"), ("cr", "<f4"), ("valid", "<i4"), ("pad", "<i4"),
                          ("f0", "<f8"), ("fdot", "<f8"), ("lambda", "<f8"), ("beta", "<f8")])


def refine(ctx: Context, dpm: DevicePeakmap, cands, kf: int, k_fdot: int, k_sky: int, dfdot: float,
           t0: float, theta: float = 2.5, weights: Optional[torch.Tensor] = None, stream=None):
    """Refined candidates (fh_refine).  cands: array [n, 6] of (f0, fdot,
    lambda, beta, dlambda, dbeta).  Returns a uint8 device tensor of n
    fh_refined records; decode with ``decode_refined``."""
    c = np.ascontiguousarray(np.asarray(cands, dtype=np.float64).reshape(-1, 6))
    n = c.shape[0]
    out = torch.empty((max(n, 1) * REFINED_DTYPE.itemsize,), dtype=torch.uint8, device="cuda:%d" % ctx.device)
    w_ptr = None
    if weights is not None:
        assert weights.dtype == torch.float32 and weights.is_cuda and weights.numel() == dpm.n_fft
        w_ptr = ctypes.c_void_p(weights.data_ptr())
    o = _lib.fh_refine_opts(int(kf), int(k_fdot), int(k_sky), 0, float(dfdot), float(t0), float(theta))
    check(_lib.fh_refine(ctx.handle, dpm.handle, n, c.ctypes.data, ctypes.byref(o), w_ptr,
                         ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out[: n * REFINED_DTYPE.itemsize]


def decode_refined(raw: torch.Tensor) -> np.ndarray:
    return raw.detach().cpu().numpy().view(REFINED_DTYPE)


def _nhat(n) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(n, dtype=np.float64).reshape(3))
    return (ctypes.c_double * 3)(*a.tolist())


def fh_hough_map_i32(ctx: Context, dpm: DevicePeakmap, nhat, grid, out=None, stream=None):
    """Unweighted Hough map [ns][nf] int32 of one sky direction."""
    if out is None:
        out = torch.empty((grid.ns, grid.nf), dtype=torch.int32, device="cuda:%d" % ctx.device)
    assert out.dtype == torch.int32 and out.is_contiguous() and tuple(out.shape) == (grid.ns, grid.nf)
    g = grid_struct(grid)
    check(_lib.fh_hough_map_i32(ctx.handle, dpm.handle, _nhat(nhat), ctypes.byref(g),
                                ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def fh_hough_map_i32_static(ctx: Context, dpm: DevicePeakmap, nhat, grid, out: torch.Tensor, stream=None):
    """fh_hough_map_i32 without any device allocation in the library: the
    workspace is the library's static per-GPU scratch; `out` is caller-owned."""
    assert out.dtype == torch.int32 and out.is_contiguous() and tuple(out.shape) == (grid.ns, grid.nf)
    g = grid_struct(grid)
    check(_lib.fh_hough_map_i32_static(ctx.handle, dpm.handle, _nhat(nhat), ctypes.byref(g),
                                       ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def fh_hough_map_f32(ctx: Context, dpm: DevicePeakmap, nhat, weights: torch.Tensor, grid,
                     out=None, stream=None):
    """Weighted Hough map [ns][nf] float32; weights: device float32 [N]."""
    assert weights.dtype == torch.float32 and weights.is_cuda and weights.is_contiguous()
    assert weights.numel() == dpm.n_fft
    if out is None:
        out = torch.empty((grid.ns, grid.nf), dtype=torch.float32, device="cuda:%d" % ctx.device)
    g = grid_struct(grid)
    check(_lib.fh_hough_map_f32(ctx.handle, dpm.handle, _nhat(nhat),
                                ctypes.c_void_p(weights.data_ptr()), ctypes.byref(g),
                                ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def n_subbands(grid, sel) -> int:
    return (int(grid.nf) + int(sel.width) - 1) // int(sel.width)


def fh_hough_candidates(ctx: Context, dpm: DevicePeakmap, sky, grid, sel,
                        weights: Optional[torch.Tensor] = None, schedule: int = 1,
                        tile_bins: int = 0, sky_chunk: int = 0, use_graph: int = 0,
                        out=None, stream=None):
    """Candidates of n_sky maps.  Returns an int32 tensor [n_sky, n_sb, 2, 8]
    holding fh_candidate records (value and cr are float32 bit patterns;
    use ``decode_candidates``)."""
    sky = np.ascontiguousarray(np.asarray(sky, dtype=np.float64).reshape(-1, 3))
    n_sky = sky.shape[0]
    n_sb = n_subbands(grid, sel)
    if out is None:
        out = torch.empty((n_sky, n_sb, 2, 8), dtype=torch.int32, device="cuda:%d" % ctx.device)
    w_ptr, w_stride = None, 0
    if weights is not None:
        assert weights.dtype == torch.float32 and weights.is_cuda and weights.is_contiguous()
        if weights.dim() == 2:
            assert tuple(weights.shape) == (n_sky, dpm.n_fft)
            w_stride = dpm.n_fft
        else:
            assert weights.numel() == dpm.n_fft
        w_ptr = ctypes.c_void_p(weights.data_ptr())
    g = grid_struct(grid)
    s = select_struct(sel)
    o = _lib.fh_options(int(schedule), int(tile_bins), int(sky_chunk), int(use_graph))
    check(_lib.fh_hough_candidates(ctx.handle, dpm.handle, n_sky, sky.ctypes.data, w_ptr, w_stride,
                                   ctypes.byref(g), ctypes.byref(s), ctypes.byref(o),
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def fh_hough_colmax(ctx: Context, dpm: DevicePeakmap, sky, grid, weights: Optional[torch.Tensor] = None,
                    schedule: int = 1, tile_bins: int = 0, sky_chunk: int = 0, stream=None):
    """Per-bin column maxima of n_sky maps: (value float32 [n_sky, nf],
    smallest row holding it int32 [n_sky, nf])."""
    sky = np.ascontiguousarray(np.asarray(sky, dtype=np.float64).reshape(-1, 3))
    n_sky = sky.shape[0]
    dev = "cuda:%d" % ctx.device
    value = torch.empty((n_sky, grid.nf), dtype=torch.float32, device=dev)
    row = torch.empty((n_sky, grid.nf), dtype=torch.int32, device=dev)
    w_ptr, w_stride = None, 0
    if weights is not None:
        assert weights.dtype == torch.float32 and weights.is_cuda and weights.is_contiguous()
        if weights.dim() == 2:
            assert tuple(weights.shape) == (n_sky, dpm.n_fft)
            w_stride = dpm.n_fft
        else:
            assert weights.numel() == dpm.n_fft
        w_ptr = ctypes.c_void_p(weights.data_ptr())
    g = grid_struct(grid)
    o = _lib.fh_options(int(schedule), int(tile_bins), int(sky_chunk), 0)
    check(_lib.fh_hough_colmax(ctx.handle, dpm.handle, n_sky, sky.ctypes.data, w_ptr, w_stride,
                               ctypes.byref(g), ctypes.byref(o), ctypes.c_void_p(value.data_ptr()),
                               ctypes.c_void_p(row.data_ptr()), _stream(stream)))
    return value, row


def decode_candidates(raw: torch.Tensor) -> dict:
    """Split a [.., 8] int32 candidate tensor into numpy fields."""
    a = raw.detach().cpu().numpy()
    out = {}
    for k, name in enumerate(CANDIDATE_FIELDS):
        col = a[..., k]
        out[name] = col.view(np.float32) if name in ("value", "cr") else col
    return out


class Server:
    """fh_server: continuous batching of candidate searches over resident peakmaps."""

    def __init__(self, ctx: Context, hbm_budget: int, lanes: int = 4, max_queue: int = 1 << 16):
        self.ctx = ctx
        h = ctypes.c_void_p()
        check(_lib.fh_server_create(ctx.handle, int(hbm_budget), int(lanes), int(max_queue),
                                    ctypes.byref(h)))
        self.handle = h
        self._keep = {}  # host and device objects a queued request still references

    def submit(self, dpm: DevicePeakmap, sky, grid, sel, out: torch.Tensor,
               weights: Optional[torch.Tensor] = None, tag: int = 0) -> int:
        sky = np.ascontiguousarray(np.asarray(sky, dtype=np.float64).reshape(-1, 3))
        w_ptr, w_stride = None, 0
        if weights is not None:
            w_ptr = weights.data_ptr()
            w_stride = dpm.n_fft if weights.dim() == 2 else 0
        r = _lib.fh_request(dpm.handle, grid_struct(grid), select_struct(sel), sky.shape[0],
                            sky.ctypes.data, w_ptr, w_stride, out.data_ptr(), int(tag))
        rid = ctypes.c_uint64()
        check(_lib.fh_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (dpm, out, weights)
        return rid.value

    def poll(self, max_n: int = 256) -> list:
        buf = (_lib.fh_completion * max_n)()
        n = ctypes.c_int32()
        check(_lib.fh_server_poll(self.handle, buf, max_n, ctypes.byref(n)))
        res = []
        for k in range(n.value):
            c = buf[k]
            d = {f: getattr(c, f) for f, _ in c._fields_}
            self._keep.pop(d["id"], None)
            res.append(d)
        return res

    def drain(self):
        """Run every queued request to completion (fh_server_drain); the
        completions are then returned by ``poll``."""
        check(_lib.fh_server_drain(self.handle))

    def cancel(self, rid: int) -> int:
        return _lib.fh_server_cancel(self.handle, ctypes.c_uint64(rid))

    def stats(self) -> dict:
        q, r, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        b = ctypes.c_int64()
        check(_lib.fh_server_stats(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f),
                                   ctypes.byref(b)))
        return {"queued": q.value, "running": r.value, "finished": f.value, "bytes_in_flight": b.value}

    def close(self):
        if self.handle:
            _lib.fh_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()
