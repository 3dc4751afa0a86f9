"""The C-ABI library loads and exports every entry point include/dr.h
declares (no compute calls: these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_documented_calls():
    names = _declared()
    for n in ["dr_create", "dr_destroy", "dr_render", "dr_estimate_grad", "dr_step", "dr_decode_grad",
              "dr_signs", "dr_stats"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2404_09758_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdr.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_lib.SIGNATURES) == set(_declared())


def test_host_side_argument_errors_need_no_gpu():
    from paper_2404_09758_amd import _lib
    lib = _lib.load()
    assert lib.dr_create(None, None, None, None) == -1
    assert lib.dr_destroy(None) == -1
    assert lib.dr_status_str(-1) == b"invalid argument"
    assert lib.dr_last_error(None) == b""
    assert lib.dr_param_count(None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2404_09758_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _lib.load()
