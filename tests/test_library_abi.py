"""The C-ABI library loads and exports every symbol include/ebe.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ebe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebe_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for needed in ("ebe_create", "ebe_assemble", "ebe_predict", "ebe_refine", "ebe_step", "ebe_apply",
                   "ebe_get_state", "ebe_set_state", "ebe_destroy"):
        assert needed in names


def test_library_exports_every_declared_symbol():
    from paper_2409_20380_amd import ebe
    if not os.path.exists(ebe.LIB_PATH):
        pytest.skip("libebe.so not built")
    lib = ctypes.CDLL(ebe.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(ebe.EXPORTS) == declared_functions()
    lib.ebe_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ebe_version()


def test_create_rejects_bad_config_without_touching_a_device():
    from paper_2409_20380_amd import ebe
    if not os.path.exists(ebe.LIB_PATH):
        pytest.skip("libebe.so not built")
    L = ebe.lib()
    h = ctypes.c_void_p()
    cfg = ebe.Config(dt=-1.0, tol=1e-8)
    assert L.ebe_create(ctypes.byref(cfg), None, ctypes.byref(h)) == ebe.E_INVALID_ARG
    assert b"invalid configuration" in L.ebe_last_error(None)
    assert L.ebe_destroy(None) == ebe.OK
