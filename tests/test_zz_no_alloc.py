"""The allocation-free inner product (eg_dot_noalloc, static per-GPU scratch) against eg_dot,
through the C ABI: two calls in a row, the second on a smaller input, so that a result built
from the first call's partial sums left in the static array would show."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_dot_noalloc_matches_eg_dot():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = eg.load_library()
    p = synth.Problem(24, 12, 9, seed=0)
    coef = torch.from_numpy(synth.make_coeffs(p)).cuda()
    rng = np.random.default_rng(21)
    with eg.Operator(coef) as op:
        for dtype in (torch.float64, torch.float32):
            for n in (3_000_001, 5_001):          # 2930 partial rows, then 5
                a = torch.from_numpy(rng.standard_normal(n)).to(dtype).cuda()
                b = torch.from_numpy(rng.standard_normal(n)).to(dtype).cuda()
                ref = op.dot(a, b)
                got = eg.dot_noalloc(a, b)
                print(f"{dtype} n={n}: eg_dot {ref!r}, eg_dot_noalloc {got!r}")
                assert got == ref                  # the same kernels and partition: bitwise
            # integer-valued vectors: the FP64 sum is exact
            ia = rng.integers(-1000, 1000, 1_000_003)
            ib = rng.integers(-1000, 1000, 1_000_003)
            exact = float(np.dot(ia, ib))
            assert eg.dot_noalloc(torch.from_numpy(ia).to(dtype).cuda(), torch.from_numpy(ib).to(dtype).cuda()) == exact
    # empty input, and sizes beyond the documented maximum are refused
    out = ctypes.c_double(7.0)
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert lib.eg_dot_noalloc(x.data_ptr(), x.data_ptr(), 0, eg.PREC_FP64, None, ctypes.byref(out)) == 0
    assert out.value == 0.0
    assert lib.eg_dot_noalloc(x.data_ptr(), x.data_ptr(), (1 << 40) + 1, eg.PREC_FP64, None, ctypes.byref(out)) == eg.EINVAL
    assert b"2^40" in lib.eg_last_error()
    assert lib.eg_dot_noalloc(x.data_ptr(), x.data_ptr(), -1, eg.PREC_FP64, None, ctypes.byref(out)) == eg.EINVAL
    assert lib.eg_dot_noalloc(None, x.data_ptr(), 4, eg.PREC_FP64, None, ctypes.byref(out)) == eg.EINVAL
