"""The C ABI library loads and exports every symbol include/psi.h declares.

No compute call is made here (this runs without a GPU).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psi.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psi_[a-z_]+)\s*\(", src)))


def test_header_declares_the_paper_calls():
    names = declared_symbols()
    for n in ("psi_build", "psi_batch_insert", "psi_batch_delete", "psi_knn", "psi_range_count",
              "psi_range_report"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2601_05347_amd as psi
    if not os.path.exists(psi.LIB_PATH):
        pytest.fail("libpsi.so is not built (python -m paper_2601_05347_amd.build)")
    lib = ctypes.CDLL(psi.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_every_symbol():
    import paper_2601_05347_amd as psi
    assert set(declared_symbols()) == set(psi.SIGNATURES)
    for n in declared_symbols():
        assert callable(getattr(psi, n)), n


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2601_05347_amd as psi
    monkeypatch.setattr(psi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(psi, "_lib", None)
    with pytest.raises(RuntimeError):
        psi.lib()


def test_status_strings():
    import paper_2601_05347_amd as psi
    assert psi.psi_status_str(0) == "ok"
    assert psi.psi_status_str(2) == "coordinate out of range"


def test_kernel_objects_are_gfx950():
    import paper_2601_05347_amd as psi
    blob = open(psi.LIB_PATH, "rb").read()
    assert b"gfx950" in blob
