"""The C-ABI library loads on the CPU host and exports every symbol the header declares.
No compute call is made (there is no GPU here); only argument checks that return before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "endgame.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1811_03852_amd as eg
    if not os.path.exists(eg.LIB_PATH):
        pytest.fail("libendgame.so is not built (run __graft_entry__.build())")
    return eg.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "eg_solve" in names and "eg_create_operator" in names
    for name in names:
        assert hasattr(lib, name), name
    import paper_1811_03852_amd as eg
    assert sorted(eg.EXPORTED) == sorted(n for n in names if n in eg.EXPORTED)
    assert set(names) <= set(eg.EXPORTED) | {n for n in names if n.startswith("eg_")}


def test_argument_errors_without_device_work(lib):
    h = ctypes.c_void_p()
    assert lib.eg_create_operator(None, 10, 10, 10, ctypes.byref(h)) == -1
    assert b"NULL" in lib.eg_last_error()
    assert lib.eg_create_operator(ctypes.c_void_p(8), 2, 10, 10, ctypes.byref(h)) == -1
    assert b"nlon" in lib.eg_last_error()
    assert lib.eg_create_operator(ctypes.c_void_p(8), 10, 0, 10, ctypes.byref(h)) == -1
    assert lib.eg_solve(None, None, None, 1e-8, 10, 0) == -1
    assert lib.eg_set_option(None, b"eta", 1e-4) == -1
    assert lib.eg_harvest_krylov(None, None, 5, None, None) == -1
    assert lib.eg_harvest(None, None, 5, None, None) == -1
    lib.eg_destroy_operator(None)


def test_modes_and_status_codes_match_header():
    import paper_1811_03852_amd as eg
    src = open(HEADER).read()
    for name, val in [("EG_FP64", eg.FP64), ("EG_FP32_IR", eg.FP32_IR), ("EG_FP32_IR_BF16", eg.FP32_IR_BF16),
                      ("EG_FP32_IR_FP16", eg.FP32_IR_FP16), ("EG_LEARNED_FP64", eg.LEARNED_FP64),
                      ("EG_LEARNED_FP32_IR", eg.LEARNED_FP32_IR), ("EG_CONVERGED", eg.CONVERGED),
                      ("EG_MAXIT", eg.MAXIT), ("EG_STALLED", eg.STALLED), ("EG_EINVAL", eg.EINVAL),
                      ("EG_ENONFINITE", eg.ENONFINITE), ("EG_ENOPC", eg.ENOPC)]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == val, name
