"""Shared helpers of the GPU tests: device transfer and error bounds.

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
