"""The C-ABI library loads and exports every symbol include/esmp2.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2003_12923_amd", "libesmp2.so")


def declared():
    txt = open(os.path.join(ROOT, "include", "esmp2.h")).read()
    return sorted(set(re.findall(r"^\s*(?:esmp2_status|const char\*)\s+(esmp2_\w+)\s*\(", txt, re.M)))


def test_header_declares_calls():
    names = declared()
    for n in ["esmp2_create", "esmp2_destroy", "esmp2_set_problem", "esmp2_rotate_top", "esmp2_space",
              "esmp2_build_rhs", "esmp2_sigma", "esmp2_solve", "esmp2_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libesmp2.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libesmp2.so not built")
def test_null_handle_and_bad_args_fail_cleanly():
    lib = ctypes.CDLL(LIB)
    lib.esmp2_last_error.restype = ctypes.c_char_p
    assert lib.esmp2_destroy(None) == 0
    assert lib.esmp2_rotate_top(None, None) == 1          # ESMP2_INVALID_ARG
    assert lib.esmp2_create(None, 0, None) == 1
    assert lib.esmp2_last_error(None) == b"null handle"
