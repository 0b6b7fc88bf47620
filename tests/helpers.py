"""Shared helpers of the GPU tests: device transfer, error bounds, 16-bit coefficient emulation.

Nothing here calls the GPU library's arithmetic; expected values always come from ``oracle``.
"""
from __future__ import annotations

import numpy as np

EPS64 = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def abs_bound(oracle, coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """S = C|x| + sum_d a_d |x_d| per row: the scale of the rounding error of y = A x."""
    neg = coef.copy()
    neg[:6] = -neg[:6]
    return oracle.apply(neg, np.abs(x))


def margin_split(coef: np.ndarray):
    """m = C - (((((W+E)+S)+N)+D)+U) and g = m + (((W+E)+S)+N), in the library's summation order."""
    hs = ((coef[0] + coef[1]) + coef[2]) + coef[3]
    m = coef[6] - ((hs + coef[4]) + coef[5])
    return m, m + hs


def round_sig(u: np.ndarray, p: int, emin: int) -> np.ndarray:
    """Round non-negative doubles to p significant bits, ties to even (textbook definition)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    nz = u > 0
    _, e = np.frexp(u[nz])
    lead = np.maximum(e - 1, emin)
    ulp = np.ldexp(1.0, lead - (p - 1))
    out[nz] = np.rint(u[nz] / ulp) * ulp
    return out


def quantized_coeffs(coef: np.ndarray, kind: str) -> np.ndarray:
    """The 16-bit operator the library builds: couplings rounded (RNE) after division by a
    power-of-two scale per (direction, level, latitude row); C rebuilt as m + sum of the
    dequantized couplings with m = float32(C - sum a)."""
    out = np.empty_like(coef)
    m, _ = margin_split(coef)
    for d in range(6):
        a = coef[d]
        mx = a.max(axis=2, keepdims=True)
        f, e = np.frexp(mx)
        e = np.where(f == 0.5, e - 1, e)
        s = np.where(mx > 0, np.ldexp(1.0, e), 1.0)
        u = a / s
        if kind == "bf16":
            q = round_sig(u, 8, -126)
        else:
            q = u.astype(np.float16).astype(np.float64)   # numpy's correctly rounded conversion
        out[d] = q * s
    m32 = m.astype(np.float32).astype(np.float64)
    out[6] = m32 + out[:6].sum(axis=0)
    return out
