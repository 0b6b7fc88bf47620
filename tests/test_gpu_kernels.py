"""Parity of the HIP building blocks with the CPU oracle (SpMV, tridiagonal preconditioner, dot
products, FP64 residual), element by element, across tile edges and ragged tails."""
import numpy as np
import pytest

import synth
from oracle.quant import quantized_coeffs
from tests.helpers import EPS32, EPS64, abs_bound, dev, host

pytestmark = pytest.mark.gpu

SHAPES = [
    synth.Problem(96, 72, 20, seed=0),              # the small benchmark grid
    synth.Problem(67, 13, 9, seed=1),               # ragged in every direction
    synth.Problem(130, 37, 5, seed=2),              # more than two lon tiles, ragged
    synth.Problem(3, 1, 1, seed=3),                 # smallest legal grid
    synth.Problem(64, 16, 70, seed=4),              # exact tiles, 70 levels
    synth.Problem(40, 30, 24, seed=5, shift=1e-6, bands=True, ratio=synth._stress_ratio()),
    synth.Problem(8, 1, 33, seed=6),                # one latitude row
    # 140 levels with whole waves of columns: the register-resident tridiagonal solves (FP64
    # at one wave per SIMD)
    synth.Problem(128, 8, 140, seed=7, shift=1e-6, bands=True, ratio=synth._stress_ratio()),
]


@pytest.fixture(scope="module")
def eg():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    return eg


def _op(eg, p):
    coef = synth.make_coeffs(p)
    return coef, eg.Operator(dev(coef))


@pytest.mark.parametrize("p", SHAPES, ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_spmv_fp64_matches_oracle(eg, oracle_mod, p):
    coef, op = _op(eg, p)
    x = np.random.default_rng(p.seed + 100).standard_normal(p.n)
    y = host(op.apply(dev(x)))
    ref = oracle_mod.apply(coef, x)
    # |fl(y) - y| <= gamma_8 (C|x| + sum a|x_d|) for either summation form; margin from FP64 C - sum a
    bound = 4 * 8 * EPS64 * abs_bound(oracle_mod, coef, x)
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    op.close()


@pytest.mark.parametrize("p", SHAPES[:3], ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_spmv_fp32_matches_oracle(eg, oracle_mod, p):
    import torch
    coef, op = _op(eg, p)
    x32 = np.random.default_rng(p.seed + 200).standard_normal(p.n).astype(np.float32)
    y = host(op.apply(dev(x32), prec=eg.PREC_FP32)).astype(np.float64)
    ref = oracle_mod.apply(coef, x32.astype(np.float64))
    # coefficient rounding (<= eps32/2 relative each) plus FP32 arithmetic
    bound = 16 * EPS32 * abs_bound(oracle_mod, coef, x32.astype(np.float64))
    assert np.all(np.abs(y - ref) <= bound)
    op.close()


@pytest.mark.parametrize("kind,prec_name", [("bf16", "PREC_BF16"), ("fp16", "PREC_FP16")])
@pytest.mark.parametrize("p", [SHAPES[0], SHAPES[1], SHAPES[5]], ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_spmv_16bit_matches_oracle_on_quantized_operator(eg, oracle_mod, p, kind, prec_name):
    coef, op = _op(eg, p)
    cq = quantized_coeffs(coef, kind)
    x32 = np.random.default_rng(p.seed + 300).standard_normal(p.n).astype(np.float32)
    y = host(op.apply(dev(x32), prec=getattr(eg, prec_name))).astype(np.float64)
    ref = oracle_mod.apply(cq, x32.astype(np.float64))
    bound = 16 * EPS32 * abs_bound(oracle_mod, cq, x32.astype(np.float64))
    assert np.all(np.abs(y - ref) <= bound)
    # and the quantized operator is within the format's rounding of the FP64 one
    rel = 2.0 ** -8 if kind == "bf16" else 2.0 ** -11
    full = oracle_mod.apply(coef, x32.astype(np.float64))
    assert np.all(np.abs(y - full) <= (rel + 16 * EPS32) * abs_bound(oracle_mod, coef, x32.astype(np.float64)))
    op.close()


def _tridiag_backward_bound(oracle_mod, coef, z, q, eps):
    """|T z - q| <= c nlev eps (|T| |z|): componentwise backward error of a stable tridiagonal solve."""
    dec = coef.copy()
    dec[:4] = 0.0
    res = oracle_mod.apply(dec, z) - q
    neg = dec.copy()
    neg[4:6] = -neg[4:6]
    scale = oracle_mod.apply(neg, np.abs(z))
    return np.abs(res), scale


@pytest.mark.parametrize("p", SHAPES, ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_thomas_fp64_matches_oracle(eg, oracle_mod, p):
    coef, op = _op(eg, p)
    q = np.random.default_rng(p.seed + 400).standard_normal(p.n)
    z = host(op.precond(dev(q)))
    ref = oracle_mod.thomas(coef, q)
    res, scale = _tridiag_backward_bound(oracle_mod, coef, z, q, EPS64)
    assert np.all(res <= 16 * p.nlev * EPS64 * scale)
    # forward agreement per column: ||T^{-1}||_inf <= 1 / min(C - D - U) (diagonal dominance,
    # Varah) and ||T||_inf <= 2 max C bound the column's condition number
    zc = ref.reshape(p.nlev, -1)
    tmin = (coef[6] - coef[4] - coef[5]).reshape(p.nlev, -1).min(axis=0)
    tmax = coef[6].reshape(p.nlev, -1).max(axis=0) * 2
    kappa = tmax / tmin
    err = np.abs(z - ref).reshape(p.nlev, -1).max(axis=0)
    assert np.all(err <= 32 * p.nlev * EPS64 * kappa * np.abs(zc).max(axis=0) + 1e-300)
    op.close()


@pytest.mark.parametrize("prec_name", ["PREC_FP32", "PREC_BF16", "PREC_FP16"])
@pytest.mark.parametrize("p", [SHAPES[0], SHAPES[1], SHAPES[4], SHAPES[5], SHAPES[7]],
                         ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_thomas_low_precision_backward_error(eg, oracle_mod, p, prec_name):
    """Every FP32-vector precision applies the FP64 T's LU factors rounded to FP32: a
    componentwise backward error of order nlev eps32 against the FP64 T (for an M-matrix
    tridiagonal |L||U| = |T|, so factor rounding stays within the same bound)."""
    coef, op = _op(eg, p)
    q32 = np.random.default_rng(p.seed + 500).standard_normal(p.n).astype(np.float32)
    z = host(op.precond(dev(q32), prec=getattr(eg, prec_name))).astype(np.float64)
    res, scale = _tridiag_backward_bound(oracle_mod, coef, z, q32.astype(np.float64), EPS32)
    assert np.all(res <= 16 * p.nlev * EPS32 * scale)
    op.close()


def test_dot_exact_and_deterministic(eg, oracle_mod):
    p = synth.Problem(100, 50, 7)
    coef, op = _op(eg, p)
    rng = np.random.default_rng(9)
    for n in (1, 255, 256, 257, 10_000, 1_000_003):
        a = rng.integers(-1000, 1000, n).astype(np.float64)
        b = rng.integers(-1000, 1000, n).astype(np.float64)
        exact = float(np.dot(a.astype(np.int64), b.astype(np.int64)))
        assert op.dot(dev(a), dev(b)) == exact
        assert op.dot(dev(a.astype(np.float32)), dev(b.astype(np.float32))) == exact
    x = rng.standard_normal(3_000_001)
    d1 = op.dot(dev(x), dev(x))
    d2 = op.dot(dev(x), dev(x))
    assert d1 == d2
    assert abs(d1 - oracle_mod.dot(x, x)) <= 1e-12 * d1
    op.close()


@pytest.mark.parametrize("p", SHAPES[:3], ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_residual_fp64_matches_oracle(eg, oracle_mod, p):
    import torch
    coef, op = _op(eg, p)
    rng = np.random.default_rng(p.seed + 600)
    b = rng.standard_normal(p.n)
    x = rng.standard_normal(p.n)
    r = torch.empty(p.n, dtype=torch.float64, device="cuda")
    rel = op.residual(dev(b), dev(x), r)
    ref = b - oracle_mod.apply(coef, x)
    bound = 4 * 8 * EPS64 * (abs_bound(oracle_mod, coef, x) + np.abs(b))
    assert np.all(np.abs(host(r) - ref) <= bound)
    assert abs(rel - np.linalg.norm(ref) / np.linalg.norm(b)) <= 1e-12 * rel
    op.close()


def test_operator_validation(eg):
    p = synth.Problem(10, 6, 4)
    coef = synth.make_coeffs(p)
    for mutate, word in [(lambda c: c.__setitem__((2, 0, 0, 3), 0.1), "boundary"),
                         (lambda c: c.__setitem__((0, 1, 2, 3), -0.1), "negative"),
                         (lambda c: c.__setitem__((6, 1, 2, 3), 0.5), "margin"),
                         (lambda c: c.__setitem__((4, 2, 2, 2), np.nan), "non-finite")]:
        c = coef.copy()
        mutate(c)
        with pytest.raises(eg.EndgameError) as ei:
            eg.Operator(dev(c))
        assert ei.value.code == eg.EINVAL and word in str(ei.value)
