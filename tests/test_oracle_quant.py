"""Pins for the 16-bit coefficient reference (oracle/quant.py): its rounding against torch's
and numpy's correctly rounded conversions and against hand-made ties, its scales, and the
row sums of the operator it rebuilds."""
import numpy as np
import pytest

import synth
from oracle import net as onet
from oracle import quant


def _float32_values(rng, count):
    """Positive float32 values over BF16's whole range, subnormals included."""
    mant = rng.integers(1 << 23, 1 << 24, count).astype(np.float64)
    exp = rng.integers(-149 - 23, 128 - 23, count)
    v = np.ldexp(mant, exp)
    v = v[(v > 0) & (v < 3.0e38)]
    return v.astype(np.float32).astype(np.float64)


def test_bf16_rounding_matches_torch():
    """round_sig(., 8, -126) is torch's float32 -> bfloat16 conversion (round to nearest even)
    on float32 inputs, over the normal and the subnormal range."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    v = _float32_values(rng, 200000)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    ours = quant.round_sig(v, 8, -126)
    finite = np.isfinite(ref)
    assert np.array_equal(ours[finite], ref[finite])
    # the network oracle's own BF16 rounding (pinned against torch elsewhere) agrees
    assert np.array_equal(ours, onet.bf16(v))


def test_fp16_rounding_matches_numpy():
    """round_sig(., 11, -14) is numpy's correctly rounded float64 -> float16 conversion,
    subnormals (down to 2^-24) included."""
    rng = np.random.default_rng(1)
    v = np.ldexp(rng.uniform(1.0, 2.0, 200000), rng.integers(-26, 15, 200000))   # below FP16's overflow
    ref = v.astype(np.float16).astype(np.float64)
    assert np.array_equal(quant.round_sig(v, 11, -14), ref)


def test_rounding_ties_go_to_even():
    """Exact halfway cases: 1 + k/2^8 + 1/2^9 lies halfway between two BF16 values and goes to
    the one with an even last bit; below the normal range the spacing stays 2^-133."""
    k = np.arange(0, 128)
    u = 1.0 + k / 256.0 + 1.0 / 512.0
    r = quant.round_sig(u, 8, -126)
    lo, hi = 1.0 + k / 256.0, 1.0 + (k + 1) / 256.0
    expect = np.where(k % 2 == 0, lo, hi)
    assert np.array_equal(r, expect)
    sub = np.ldexp(np.array([1.5, 2.5, 3.5, 0.5, 0.49]), -133)
    assert np.array_equal(quant.round_sig(sub, 8, -126), np.ldexp(np.array([2.0, 2.0, 4.0, 0.0, 0.0]), -133))


@pytest.mark.parametrize("kind,rel", [("bf16", 2.0 ** -8), ("fp16", 2.0 ** -11)])
def test_quantized_operator(kind, rel):
    """Offsets: 0 on rows holding a zero coupling or spread over more than a factor 2, else an
    FP32 value no farther than half the row's spread (plus its own rounding) from every
    coupling of the row; scales are powers of
    two with the row's largest |a - offset| in (1/2, 1] after scaling; each coupling is within
    half a unit in the last place of its remainder a - offset (the unit roundoff 2^-8 for BF16
    and 2^-11 for FP16, relative; these magnitudes are far from underflow) plus the FP32
    rounding of offset + remainder; zero couplings stay zero; the rebuilt operator's row sums
    are the FP32 margin, and its diagonal differs from C by no more than the FP32 rounding of
    the true margin plus the couplings' roundings."""
    p = synth.Problem(40, 30, 12, seed=3)
    coef = synth.make_coeffs(p)
    a = coef[:6]
    lo, hi = a.min(axis=3, keepdims=True), a.max(axis=3, keepdims=True)
    o = quant.offsets(coef)
    narrow = (lo > 0) & (hi <= 2 * lo)
    assert np.all(o[~narrow] == 0) and np.all(o[narrow] > 0)
    assert np.array_equal(o, o.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(a - o) <= 0.5 * (hi - lo) + 2.0 ** -24 * o)
    s = quant.scales(coef)
    assert np.array_equal(s, np.ldexp(1.0, np.frexp(s)[1] - 1))
    mx = np.abs(a - o).max(axis=3, keepdims=True)
    ratio = mx[mx > 0] / np.broadcast_to(s, mx.shape)[mx > 0]
    assert np.all((ratio > 0.5) & (ratio <= 1.0))
    cq = quant.quantized_coeffs(coef, kind)
    aq = cq[:6]
    assert np.array_equal(aq == 0, a == 0) and np.all(aq >= 0)
    assert np.array_equal(aq, aq.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(aq - a) <= rel * np.abs(a - o) + 2.0 ** -24 * aq)
    assert np.all(np.abs(aq - a) <= rel * a + 2.0 ** -24 * aq)      # never worse than the plain format
    # the offsets pay: on these operators the coupling error is far below the plain format's
    assert np.max(np.abs(aq - a) / np.where(a > 0, a, 1.0)) < 0.25 * rel
    # a zero among positive couplings: its row keeps offset 0, so the zero stays zero
    c2 = coef.copy()
    c2[0, 3, 5, 7] = 0.0
    assert quant.offsets(c2)[0, 3, 5, 0] == 0 and quant.quantized_coeffs(c2, kind)[0, 3, 5, 7] == 0
    # a row spread over more than a factor 2 keeps offset 0: its smallest coupling keeps the
    # format's relative precision
    c3 = coef.copy()
    c3[1, 4, 6, 9] *= 100.0
    aq3 = quant.quantized_coeffs(c3, kind)[1, 4, 6]
    assert quant.offsets(c3)[1, 4, 6, 0] == 0
    assert np.all(np.abs(aq3 - c3[1, 4, 6]) <= rel * c3[1, 4, 6] + 2.0 ** -24 * aq3)
    m32 = quant.margin(coef).astype(np.float32).astype(np.float64)
    rows = cq[6] - aq.sum(axis=0)
    assert np.allclose(rows, m32, rtol=0, atol=1e-15 * np.abs(cq[6]).max())
    m_true = coef[6] - coef[:6].sum(axis=0)
    bound = 2.0 ** -24 * np.abs(m_true) + np.abs(aq - a).sum(axis=0) + 1e-14 * np.abs(coef[6])
    assert np.all(np.abs(cq[6] - coef[6]) <= bound)
