"""The C-ABI library loads on a machine without a GPU and exports every entry
point declared in include/mvp.h (no compute calls here)."""
import ctypes
import os
import re

from paper_2103_01954_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mvp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mvp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("mvp_build_accel", "mvp_render_fwd", "mvp_render_bwd", "mvp_submit", "mvp_poll"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_version_and_error_strings_need_no_device():
    lib = _lib.load()
    assert b"gfx950" in lib.mvp_version()
    assert lib.mvp_last_error() is not None
    # argument errors are reported synchronously, without touching a device
    h = ctypes.c_void_p()
    assert lib.mvp_destroy(None) == _lib.MVP_ERR_INVALID
    assert b"NULL" in lib.mvp_last_error()
    assert lib.mvp_build_accel(None, None, None, 0, None, ctypes.byref(h), None) == _lib.MVP_ERR_INVALID


def test_timing_entry_points_reject_bad_arguments_without_a_device():
    lib = _lib.load()
    ms = (ctypes.c_float * 4)()
    n = ctypes.c_int32()
    assert lib.mvp_timing_start(None, 4) == _lib.MVP_ERR_INVALID
    assert lib.mvp_timing_read(None, 0, ms, ctypes.byref(n)) == _lib.MVP_ERR_INVALID
    assert lib.mvp_timing_stop(None) == _lib.MVP_ERR_INVALID
