"""The C-ABI library loads and exports every entry point include/h2d.h
declares (no compute call: this runs without a GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "h2d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(h2d_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("h2d_build", "h2d_matvec", "h2d_solve", "h2d_destroy", "h2d_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2204_05536_amd import hodlr2d
    L = hodlr2d.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(hodlr2d.EXPORTED) == _declared()
