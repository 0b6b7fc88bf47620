"""FP64 reference of the operator the 16-bit coefficient modes solve with (TEST
INFRASTRUCTURE ONLY).

The paper keeps the matrix in 64 or 32 bits (Sec. 3-4); the BF16/FP16 coefficient store is this
project's extension of its mixed-precision idea.  Its definition, written out plainly:

* each of the six off-diagonal coupling planes (W, E, S, N, D, U) is stored per level and
  latitude row as an offset o plus a scaled remainder: o is the FP32 rounding of the midpoint
  of the row's smallest and largest coupling when all of them are positive and the largest is
  at most twice the smallest, else 0 (zero couplings stay zero, and no coupling's relative
  error exceeds the plain format's), and the remainder a - o is divided by the power of two
  s = 2^ceil(log2 max |a - o|) of the row, so that every scaled value lies in [-1, 1] and the
  scaling itself is exact;
* the scaled value is rounded to nearest, ties to even, to 8 significant bits with the
  exponent range of BF16 (normal exponents down to -126, gradual underflow below) or to 11
  significant bits with that of FP16 (down to -14), its sign kept;
* the coupling the operator uses is o + q s rounded once to FP32 (q s is exact);
* the margin m = C - (((((W + E) + S) + N) + D) + U) is rounded to FP32, and the diagonal of
  the 16-bit operator is rebuilt as m32 plus the sum of the dequantised couplings, so that
  the operator's row sums stay exactly its FP32 margin (the tiny shift is not swamped by the
  coupling rounding).
"""
from __future__ import annotations

import numpy as np

KINDS = {"bf16": (8, -126), "fp16": (11, -14)}


def round_sig(u: np.ndarray, p: int, emin: int) -> np.ndarray:
    """Round non-negative doubles to p significant bits, ties to even, with gradual underflow
    below 2^emin (the spacing stays 2^(emin - p + 1) there), as IEEE binary formats do."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    nz = u > 0
    _, e = np.frexp(u[nz])
    lead = np.maximum(e - 1, emin)
    ulp = np.ldexp(1.0, lead - (p - 1))
    out[nz] = np.rint(u[nz] / ulp) * ulp   # np.rint rounds halves to even
    return out


def margin(coef: np.ndarray) -> np.ndarray:
    """m = C - (((((W + E) + S) + N) + D) + U), summed in this order."""
    hs = ((coef[0] + coef[1]) + coef[2]) + coef[3]
    return coef[6] - ((hs + coef[4]) + coef[5])


def offsets(coef: np.ndarray) -> np.ndarray:
    """Offset per (direction, level, latitude row): shape (6, nlev, nlat, 1)."""
    lo = coef[:6].min(axis=3, keepdims=True)
    hi = coef[:6].max(axis=3, keepdims=True)
    mid = (0.5 * (lo + hi)).astype(np.float32).astype(np.float64)
    return np.where((lo > 0) & (hi <= 2.0 * lo), mid, 0.0)


def scales(coef: np.ndarray) -> np.ndarray:
    """Power-of-two scale per (direction, level, latitude row) of the remainders a - offset:
    shape (6, nlev, nlat, 1)."""
    mx = np.abs(coef[:6] - offsets(coef)).max(axis=3, keepdims=True)
    f, e = np.frexp(mx)
    e = np.where(f == 0.5, e - 1, e)   # an exact power of two is its own scale
    return np.where(mx > 0, np.ldexp(1.0, e), 1.0)


def quantized_coeffs(coef: np.ndarray, kind: str) -> np.ndarray:
    """The 16-bit operator as coefficient planes (W, E, S, N, D, U, C) in FP64: dequantised
    couplings and the rebuilt diagonal."""
    p, emin = KINDS[kind]
    out = np.empty_like(coef)
    o, s = offsets(coef), scales(coef)
    u = (coef[:6] - o) / s
    q = np.sign(u) * round_sig(np.abs(u), p, emin)
    out[:6] = (o + q * s).astype(np.float32).astype(np.float64)
    m32 = margin(coef).astype(np.float32).astype(np.float64)
    out[6] = m32 + out[:6].sum(axis=0)
    return out
