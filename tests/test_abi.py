"""The C ABI library loads and exports every entry point declared in mm.h
(no GPU needed: nothing is called)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b((?:mm|mmk)_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("mm_setup", "mm_decompose", "mm_step_modal",
                     "mm_step_cholesky", "mm_probe"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2407_11993_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmm.so is not built (run __graft_entry__.build())")
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_lib.SYMBOLS) == _declared()


def test_binding_refuses_a_missing_library(tmp_path):
    from paper_2407_11993_amd import _lib
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "libmm.so"))
