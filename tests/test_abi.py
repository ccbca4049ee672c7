"""The built library loads and exports every entry point include/dgj.h
declares (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgj.h")
LIB = os.path.join(ROOT, "paper_2002_04222_amd", "lib", "libdgj.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgj_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_path():
    names = declared()
    for must in ("dgj_create", "dgj_destroy", "dgj_residual", "dgj_stage_residual", "dgj_jfnk_matvec",
                 "dgj_precond_build", "dgj_precond_apply", "dgj_sdirk_step", "dgj_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_header():
    from paper_2002_04222_amd import binding
    lib = binding.load_library()
    for n in declared():
        assert getattr(lib, n).argtypes is not None, n
