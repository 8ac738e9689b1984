"""ctypes binding of libfh.so (include/fh.h).  Argument marshalling only.

The functions keep the C names.  Device buffers are passed as raw pointers
(``tensor.data_ptr()``); streams as ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfh.so")

FH_OK = 0
FH_E_INVALID = -1
FH_E_NOMEM = -2
FH_E_DEVICE = -3
FH_E_UNSUPPORTED = -4
FH_E_BUSY = -5
FH_E_CANCELLED = -6
FH_SCHED_PLAIN = 0
FH_SCHED_PERSISTENT = 1

_STATUS = {0: "FH_OK", -1: "FH_E_INVALID", -2: "FH_E_NOMEM", -3: "FH_E_DEVICE",
           -4: "FH_E_UNSUPPORTED", -5: "FH_E_BUSY", -6: "FH_E_CANCELLED"}


class fh_peakmap_desc(ctypes.Structure):
    _fields_ = [("n_fft", ctypes.c_int32), ("n_peaks", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("bins", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("v", ctypes.c_void_p), ("t_fft", ctypes.c_double)]


class fh_grid(ctypes.Structure):
    _fields_ = [("kf", ctypes.c_int32), ("b0", ctypes.c_int64), ("nf", ctypes.c_int32),
                ("ns", ctypes.c_int32), ("fdot0", ctypes.c_double), ("dfdot", ctypes.c_double),
                ("t0", ctypes.c_double)]


class fh_select(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("excl", ctypes.c_int32), ("sep", ctypes.c_int32),
                ("theta", ctypes.c_double)]


class fh_candidate(ctypes.Structure):
    _fields_ = [("sky", ctypes.c_int32), ("subband", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("bin", ctypes.c_int32), ("row", ctypes.c_int32), ("value", ctypes.c_float),
                ("cr", ctypes.c_float), ("valid", ctypes.c_int32)]


class fh_options(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("tile_bins", ctypes.c_int32),
                ("sky_chunk", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class fh_plan_info(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("tile_bins", ctypes.c_int32),
                ("n_row_blocks", ctypes.c_int32), ("n_bin_blocks", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("cell_updates", ctypes.c_int64)]


class fh_profile(ctypes.Structure):
    _fields_ = [("tiles_ms", ctypes.c_double), ("tiles_launches", ctypes.c_int64),
                ("front_ms", ctypes.c_double), ("front_launches", ctypes.c_int64),
                ("select_ms", ctypes.c_double), ("select_launches", ctypes.c_int64),
                ("cell_updates", ctypes.c_int64), ("graph_ms", ctypes.c_double),
                ("graph_launches", ctypes.c_int64)]


class fh_coarse_cand(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double), ("fdot", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("beta", ctypes.c_double), ("dlambda", ctypes.c_double), ("dbeta", ctypes.c_double)]


class fh_gross(ctypes.Structure):
    _fields_ = [("t_origin", ctypes.c_double), ("dt_h", ctypes.c_double), ("df_h", ctypes.c_double),
                ("c0", ctypes.c_int64), ("n_t", ctypes.c_int32), ("n_f", ctypes.c_int32)]


class fh_refine_opts(ctypes.Structure):
    _fields_ = [("kf", ctypes.c_int32), ("k_fdot", ctypes.c_int32), ("k_sky", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("dfdot", ctypes.c_double), ("t0", ctypes.c_double),
                ("theta", ctypes.c_double)]


class fh_request(ctypes.Structure):
    _fields_ = [("pm", ctypes.c_void_p), ("grid", fh_grid), ("sel", fh_select),
                ("n_sky", ctypes.c_int32), ("sky", ctypes.c_void_p), ("d_w", ctypes.c_void_p),
                ("w_stride", ctypes.c_int32), ("d_out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class fh_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("lane", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("footprint", ctypes.c_int64), ("cell_updates", ctypes.c_int64)]


P = ctypes.c_void_p
_PROTOS = {
    "fh_version": ([], ctypes.c_char_p),
    "fh_last_error": ([], ctypes.c_char_p),
    "fh_ctx_create": ([ctypes.c_int32, ctypes.POINTER(P)], ctypes.c_int),
    "fh_ctx_destroy": ([P], None),
    "fh_ctx_check": ([P, P], ctypes.c_int),
    "fh_ctx_set_option": ([P, ctypes.c_char_p, ctypes.c_int64], ctypes.c_int),
    "fh_ctx_set_doppler": ([P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "fh_peakmap_upload": ([P, ctypes.POINTER(fh_peakmap_desc), P, ctypes.POINTER(P)], ctypes.c_int),
    "fh_peakmap_release": ([P, P], None),
    "fh_peakmap_from_spectra": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_int32,
                                 ctypes.c_float, P, P, ctypes.c_double, P, ctypes.POINTER(P)], ctypes.c_int),
    "fh_peakmap_download": ([P, P, P, P], ctypes.c_int),
    "fh_peakmap_shape": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fh_peakmap_bytes": ([P], ctypes.c_int64),
    "fh_plan_query": ([P, P, ctypes.POINTER(fh_grid), ctypes.c_int32,
                       ctypes.POINTER(fh_plan_info)], ctypes.c_int),
    "fh_hough_map_i32": ([P, P, P, ctypes.POINTER(fh_grid), P, P], ctypes.c_int),
    "fh_hough_map_i32_static": ([P, P, P, ctypes.POINTER(fh_grid), P, P], ctypes.c_int),
    "fh_hough_colmax": ([P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.POINTER(fh_grid),
                         ctypes.POINTER(fh_options), P, P, P], ctypes.c_int),
    "fh_hough_map_f32": ([P, P, P, P, ctypes.POINTER(fh_grid), P, P], ctypes.c_int),
    "fh_hough_candidates": ([P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.POINTER(fh_grid),
                             ctypes.POINTER(fh_select), ctypes.POINTER(fh_options), P, P],
                            ctypes.c_int),
    "fh_peakmap_slice": ([P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.POINTER(P)], ctypes.c_int),
    "fh_refine": ([P, P, ctypes.c_int32, P, ctypes.POINTER(fh_refine_opts), P, P, P], ctypes.c_int),
    "fh_gross_histogram": ([P, P, ctypes.POINTER(fh_gross), P, P], ctypes.c_int),
    "fh_clean_gross": ([P, P, ctypes.POINTER(fh_gross), ctypes.c_double, P, P, ctypes.POINTER(P)], ctypes.c_int),
    "fh_bin_counts": ([P, P, ctypes.c_int32, ctypes.c_int32, P, P], ctypes.c_int),
    "fh_robust_stats": ([P, P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
    "fh_line_counts": ([P, P, ctypes.POINTER(fh_grid), P, P], ctypes.c_int),
    "fh_veto_bins": ([P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                      ctypes.c_double, P, ctypes.POINTER(P)], ctypes.c_int),
    "fh_server_create": ([P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)],
                         ctypes.c_int),
    "fh_server_submit": ([P, ctypes.POINTER(fh_request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "fh_server_poll": ([P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "fh_server_cancel": ([P, ctypes.c_uint64], ctypes.c_int),
    "fh_server_drain": ([P], ctypes.c_int),
    "fh_server_stats": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fh_server_destroy": ([P], None),
    "fh_ctx_profile": ([P, ctypes.c_int32], ctypes.c_int),
    "fh_ctx_profile_read": ([P, ctypes.POINTER(fh_profile)], ctypes.c_int),
}

_lib = None


class FHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


def load(path: str = LIB_PATH):
    """Load libfh.so and attach prototypes (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libfh.so is not built (%s); run `python -m paper_1407_8333_amd.build`"
                               % path)
        lib = ctypes.CDLL(path)
        for name, (args, res) in _PROTOS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def exported_names():
    return list(_PROTOS)


def check(status: int):
    if status != FH_OK:
        raise FHError(status, load().fh_last_error().decode())
    return status


def _fwd(name):
    def f(*args):
        return getattr(load(), name)(*args)
    f.__name__ = name
    return f


fh_version = _fwd("fh_version")
fh_last_error = _fwd("fh_last_error")
fh_ctx_create = _fwd("fh_ctx_create")
fh_ctx_destroy = _fwd("fh_ctx_destroy")
fh_ctx_check = _fwd("fh_ctx_check")
fh_peakmap_upload = _fwd("fh_peakmap_upload")
fh_peakmap_release = _fwd("fh_peakmap_release")
fh_peakmap_bytes = _fwd("fh_peakmap_bytes")
fh_plan_query = _fwd("fh_plan_query")
fh_hough_map_i32 = _fwd("fh_hough_map_i32")
fh_hough_map_i32_static = _fwd("fh_hough_map_i32_static")
fh_hough_colmax = _fwd("fh_hough_colmax")
fh_hough_map_f32 = _fwd("fh_hough_map_f32")
fh_hough_candidates = _fwd("fh_hough_candidates")
fh_ctx_profile = _fwd("fh_ctx_profile")
fh_ctx_profile_read = _fwd("fh_ctx_profile_read")
fh_server_create = _fwd("fh_server_create")
fh_server_submit = _fwd("fh_server_submit")
fh_server_poll = _fwd("fh_server_poll")
fh_server_cancel = _fwd("fh_server_cancel")
fh_server_stats = _fwd("fh_server_stats")
fh_server_destroy = _fwd("fh_server_destroy")
fh_ctx_set_option = _fwd("fh_ctx_set_option")
fh_peakmap_from_spectra = _fwd("fh_peakmap_from_spectra")
fh_peakmap_download = _fwd("fh_peakmap_download")
fh_peakmap_shape = _fwd("fh_peakmap_shape")
fh_peakmap_slice = _fwd("fh_peakmap_slice")
fh_refine = _fwd("fh_refine")
fh_server_drain = _fwd("fh_server_drain")
fh_ctx_set_doppler = _fwd("fh_ctx_set_doppler")
fh_gross_histogram = _fwd("fh_gross_histogram")
fh_clean_gross = _fwd("fh_clean_gross")
fh_bin_counts = _fwd("fh_bin_counts")
fh_robust_stats = _fwd("fh_robust_stats")
fh_line_counts = _fwd("fh_line_counts")
fh_veto_bins = _fwd("fh_veto_bins")
