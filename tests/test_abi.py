"""The C-ABI library loads and exports every entry point include/lqt.h declares.

CPU-only: loads the shared object and resolves symbols; makes no compute call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqt.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lqt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lqt_plan", "lqt_solve", "lqt_submit", "lqt_poll", "lqt_destroy", "lqt_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2104_03186_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblqt.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTED) == set(declared_functions())


def test_last_error_without_plan_is_host_only():
    from paper_2104_03186_amd import _lib

    lib = _lib.load()
    s = lib.lqt_last_error(None)
    assert isinstance(s, bytes)


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2104_03186_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()
