"""The C-ABI library loads on the CPU and exports every entry point of include/fraclap.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1802_03770_amd", "libfraclap.so")


def declared():
    src = open(os.path.join(ROOT, "include", "fraclap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["fl_make_weights", "fl_apply", "fl_precond", "fl_solve", "fl_step", "fl_solve_batched",
              "fl_step_batched", "fl_op_destroy", "fl_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    import paper_1802_03770_amd as fl
    assert sorted(fl.EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_rejected_without_gpu():
    # argument validation happens before any device call
    lib = ctypes.CDLL(LIB)
    lib.fl_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(8, 8, 1)
    lib.fl_make_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    for d, a, hh in [(4, 1.0, 0.1), (2, 0.0, 0.1), (2, 2.0, 0.1), (2, 1.0, -1.0)]:
        st = lib.fl_make_weights(d, a, hh, n, None, None, ctypes.byref(h))
        assert st == -1, (d, a, hh)
        assert lib.fl_last_error()
