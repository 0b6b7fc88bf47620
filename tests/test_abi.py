"""The C-ABI library loads on the CPU host and exports every symbol the header declares.
No compute call is made (there is no GPU here); only argument checks that return before any
device work."""
import ctypes
import os
import re
import shutil
import subprocess

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
    assert lib.eg_train_learned_pc(None, b"rhs=2", 1, 1e-3, 0) == -1
    assert lib.eg_save_learned_pc(None, None, 0) == -1
    assert lib.eg_load_learned_pc(None, None, 0) == -1
    assert lib.eg_get_learned_pc(None, None) == -1
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


def _fake_operator(n_shape=(8, 6, 5)):
    """An Operator object with its shape fields set and no library handle: enough to reach the
    binding's argument checks, which must raise before any library call."""
    import torch
    import paper_1811_03852_amd as eg
    op = eg.Operator.__new__(eg.Operator)
    op.nlon, op.nlat, op.nlev = n_shape
    op.n = n_shape[0] * n_shape[1] * n_shape[2]
    op.device = torch.device("cuda", 0)
    op._h = None
    return op


def test_binding_rejects_wrong_dtype_size_and_host_tensors():
    """A float32 or short vector handed to a call that reads n doubles would make the library
    read past the buffer: the binding checks dtype, length and placement first."""
    import torch
    import paper_1811_03852_amd as eg
    op = _fake_operator()
    n = op.n
    good = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="float64"):
        op.solve(torch.zeros(n, dtype=torch.float32), good)
    with pytest.raises(ValueError, match="elements"):
        op.solve(good, torch.zeros(n - 1, dtype=torch.float64))
    with pytest.raises(TypeError, match="CUDA"):
        op.solve(good, good.clone())
    with pytest.raises(ValueError, match="float32"):
        op.apply(good, prec=eg.PREC_FP32)
    with pytest.raises(ValueError, match="elements"):
        op.precond(torch.zeros(2 * n, dtype=torch.float64))
    with pytest.raises(ValueError, match="precision"):
        op.apply(good, prec=7)
    with pytest.raises(ValueError, match="contiguous"):
        op.residual(torch.zeros(2 * n, dtype=torch.float64)[::2], good)
    with pytest.raises(ValueError):
        op.dot(torch.zeros(n, dtype=torch.float64), torch.zeros(n, dtype=torch.float32))
    with pytest.raises(ValueError, match="nvec"):
        op.harvest_krylov(good, 65)


def test_binding_rejects_bad_training_sets():
    """Training pairs must be float32 of shape (len(pair_op), n), every pair_op index must name
    an operator, and all operators must share a grid."""
    import torch
    import paper_1811_03852_amd as eg
    ops = [_fake_operator(), _fake_operator()]
    n = ops[0].n
    net = eg.Net.__new__(eg.Net)
    net._h = None
    r = torch.zeros((3, n), dtype=torch.float32)
    with pytest.raises(ValueError, match="shape"):
        net.train(ops, r, torch.zeros((2, n), dtype=torch.float32), [0, 1, 1], epochs=1)
    with pytest.raises(ValueError, match="pair_op"):
        net.train(ops, r, r, [0, 1, 2], epochs=1)
    with pytest.raises(ValueError, match="float32"):
        net.eval(ops, r.double(), r, [0, 0, 1])
    with pytest.raises(ValueError, match="same grid"):
        net.eval([ops[0], _fake_operator((8, 6, 4))], r, r, [0, 0, 1])
    with pytest.raises(ValueError, match="elements"):
        net.loss_grad(ops[0], torch.zeros(n + 1, dtype=torch.float32), torch.zeros(n, dtype=torch.float32))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_compiles_as_c_and_every_entry_point_links(lib, tmp_path):
    """A plain C99 caller: the header compiles warning-free under -pedantic, a program that takes
    the address of every declared entry point links against libendgame.so, and it runs on the
    host as far as an argument check (no device work)."""
    import paper_1811_03852_amd as eg
    names = _declared()
    refs = ",\n".join(f"        (void (*)(void)){n}" for n in names)
    prog = tmp_path / "caller.c"
    prog.write_text('#include "endgame.h"\n#include <stdio.h>\nint main(void)\n{\n'
                    f"    void (*fns[])(void) = {{\n{refs}\n    }};\n"
                    "    int i, k = 0;\n"
                    "    for (i = 0; i < (int)(sizeof fns / sizeof fns[0]); ++i) k += fns[i] != 0;\n"
                    '    printf("%d\\n", k);\n'
                    "    return eg_create_operator(0, 10, 10, 10, 0) == EG_EINVAL ? 0 : 1;\n}\n")
    libdir = os.path.dirname(eg.LIB_PATH)
    exe = tmp_path / "caller"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.dirname(HEADER),
                        str(prog), "-L", libdir, "-lendgame", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert int(r.stdout.strip()) == len(names)
