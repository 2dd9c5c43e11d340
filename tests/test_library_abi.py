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


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No CPU fallback: with the library missing, the first call into the binding raises."""
    from paper_2409_20380_amd import ebe
    monkeypatch.setattr(ebe, "_lib", None)
    monkeypatch.setattr(ebe, "LIB_PATH", os.path.join(os.path.dirname(ebe.LIB_PATH), "missing_libebe.so"))
    with pytest.raises(ImportError):
        ebe.lib()
    with pytest.raises(ImportError):
        ebe.Solver(0.01)


def test_product_code_does_not_use_the_oracle():
    """Only the tests, smoke() and the bench's CPU-baseline leg may touch oracle/: the package imports none of it."""
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2409_20380_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(root, f), encoding="utf-8").read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.c" not in text and "liboracle" not in text, f
