"""The C-ABI library builds for gfx950, loads on the CPU host and exports every
entry point that include/jfnk.h declares (no compute calls: no GPU here)."""
import os
import re

import pytest

from paper_2007_10411_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "jfnk.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(jfnk_\w+)\s*\(", txt, re.M)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(L.EXPORTS)


@pytest.mark.skipif(not L.lib_available(), reason="libjfnk.so not built")
def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not L.lib_available(), reason="libjfnk.so not built")
def test_invalid_problem_is_rejected_without_a_gpu():
    import ctypes as C
    from paper_2007_10411_amd import inputs as I
    lib = L.load()
    h = C.c_void_p()
    bad = L.problem_struct(I.thermal_neutral_2d(4, 4))     # below the 8-point minimum
    assert lib.jfnk_create(C.byref(bad), 30, None, C.byref(h)) == L.JFNK_ERR_ARG
    assert b"8 points" in lib.jfnk_last_error()
    assert lib.jfnk_create(None, 30, None, C.byref(h)) == L.JFNK_ERR_ARG
    # the derivative order parameter is 2 or 3
    bad3 = L.problem_struct(I.thermal_neutral_3d(16, 16, 16).replace(dd_p=4))
    assert lib.jfnk_create(C.byref(bad3), 30, None, C.byref(h)) == L.JFNK_ERR_ARG
    assert b"dd_p" in lib.jfnk_last_error()
