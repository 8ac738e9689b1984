"""The C-ABI library loads on a machine without a GPU and exports every
function declared in include/fh.h (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fh_[a-z0-9_]+)\s*\(", src)))


def _lib_path():
    from paper_1407_8333_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1407_8333_amd import build
        build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fh_ctx_create", "fh_peakmap_upload", "fh_hough_map_i32", "fh_hough_map_f32",
              "fh_hough_candidates", "fh_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1407_8333_amd import _lib
    assert set(_declared()) <= set(_lib.exported_names())


def test_version_and_error_strings_without_gpu():
    from paper_1407_8333_amd import _lib
    lib = _lib.load(_lib_path())
    assert b"gfx950" in lib.fh_version()
    assert lib.fh_last_error() is not None
    # invalid arguments are rejected on the host before any device work
    assert lib.fh_ctx_create(0, None) == _lib.FH_E_INVALID
