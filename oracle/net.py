"""FP64 reference of the learned right preconditioner (TEST INFRASTRUCTURE ONLY).

The paper's preconditioner is the tridiagonal-based SOR of Sec. 2 (Eq. 6-7); the learned form
below keeps the exact tridiagonal solve T^{-1} of that section and lets a small network add a
correction in residual space:

    M(q) = T^{-1} (q + rho * delta(q)),   rho = rms(q)

delta is a per-point scalar produced from four input channels per grid point

    x0 = [ q / rho,  T^{-1} q / rms(T^{-1} q),  D + U,  W + E + S + N ]

by  conv1d over levels (4 -> 32, 5 taps) -> ReLU -> 3x3 horizontal mixing on each level
(32 -> 32) -> ReLU -> conv1d (32 -> 32, 5 taps) -> ReLU -> conv1d (32 -> 1, 5 taps).
Levels and latitudes are zero-padded, longitude is periodic.  With the last layer zero the
preconditioner is exactly T^{-1}.

Parameter vector theta (15,233 floats), in this order:
    W1[5][32][4], b1[32], W2[9][32][32], b2[32], W3[5][32][32], b3[32], W4[5][32], b4[1]
vertical tap t couples level k + t - 2; horizontal tap t couples (i + t % 3 - 1, j + t // 3 - 1).

With ``bf16=True`` the weights, the input channels, the hidden activations and the hidden
gradients are rounded to BF16 (round to nearest even) at the points where the GPU kernels
store them in BF16; all arithmetic is FP64.  With ``bf16=False`` the function is plain FP64
and is pinned by central finite differences in the tests.

``adam_step`` is the optimiser the training uses (Kingma & Ba 2015, Algorithm 1) in FP64, pinned
by a hand-worked two-step example and by its closed form under a constant gradient.
"""
from __future__ import annotations

import numpy as np

import oracle

C_IN, C_HID, TAPS_V, TAPS_H = 4, 32, 5, 9
SHAPES = [("W1", (TAPS_V, C_HID, C_IN)), ("b1", (C_HID,)), ("W2", (TAPS_H, C_HID, C_HID)), ("b2", (C_HID,)),
          ("W3", (TAPS_V, C_HID, C_HID)), ("b3", (C_HID,)), ("W4", (TAPS_V, C_HID)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    assert o == theta.size == N_PARAMS
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value, ties to even (8 significant bits)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    ax = np.abs(x[nz])
    _, e = np.frexp(ax)
    ulp = np.ldexp(1.0, np.maximum(e - 1, -126) - 7)
    out[nz] = np.sign(x[nz]) * np.rint(ax / ulp) * ulp
    return out


def thomas_transpose(coef: np.ndarray, y: np.ndarray) -> np.ndarray:
    """T^{-T} y: T^T is the tridiagonal with sub-diagonal -U(k-1) and super-diagonal -D(k+1)."""
    ct = np.zeros_like(coef)
    ct[6] = coef[6]
    ct[4, 1:] = coef[5, :-1]
    ct[5, :-1] = coef[4, 1:]
    return oracle.thomas(ct, y)


def _shift_v(h, dk):
    """out[k] = h[k + dk] with zeros outside (h: nlev, nlat, nlon, C)."""
    out = np.zeros_like(h)
    nlev = h.shape[0]
    if dk >= 0:
        out[:nlev - dk] = h[dk:]
    else:
        out[-dk:] = h[:nlev + dk]
    return out


def _shift_h(h, di, dj):
    """out[:, j, i] = h[:, j + dj, i + di], periodic in i, zeros outside in j."""
    out = np.zeros_like(h)
    nlat = h.shape[1]
    rolled = np.roll(h, -di, axis=2)
    if dj >= 0:
        out[:, :nlat - dj] = rolled[:, dj:]
    else:
        out[:, -dj:] = rolled[:, :nlat + dj]
    return out


def _vtap(t):
    return t - 2


def _htap(t):
    return t % 3 - 1, t // 3 - 1


def features(coef: np.ndarray, q: np.ndarray, scales=None):
    """The four input channels; ``scales`` = (rms of q, rms of T^{-1} q) over the whole grid
    when q is a window cut out of it (default: taken from q itself)."""
    nlev, nlat, nlon = coef.shape[1:]
    q = np.asarray(q, dtype=np.float64).ravel()
    z0 = oracle.thomas(coef, q)
    if scales is None:
        rho = np.sqrt(np.mean(q * q))
        rhoz = np.sqrt(np.mean(z0 * z0))
    else:
        rho, rhoz = scales
    x0 = np.stack([q / rho, z0 / rhoz, (coef[4] + coef[5]).ravel(), (coef[0] + coef[1] + coef[2] + coef[3]).ravel()],
                  axis=1)
    return x0.reshape(nlev, nlat, nlon, C_IN), rho


def forward(theta: np.ndarray, coef: np.ndarray, q: np.ndarray, bf16_round: bool = True, scales=None):
    """delta(q) (flat) and the cache needed by ``backward``."""
    P = unpack(theta)
    rnd = bf16 if bf16_round else (lambda a: a)
    W1, W2, W3, W4 = (rnd(P[k]) for k in ("W1", "W2", "W3", "W4"))
    x0, rho = features(coef, q, scales)
    x0 = rnd(x0)
    z1 = sum(_shift_v(x0, _vtap(t)) @ W1[t].T for t in range(TAPS_V)) + P["b1"]
    a1 = rnd(np.maximum(z1, 0.0))
    z2 = sum(_shift_h(a1, *_htap(t)) @ W2[t].T for t in range(TAPS_H)) + P["b2"]
    a2 = rnd(np.maximum(z2, 0.0))
    z3 = sum(_shift_v(a2, _vtap(t)) @ W3[t].T for t in range(TAPS_V)) + P["b3"]
    a3 = rnd(np.maximum(z3, 0.0))
    delta = sum(_shift_v(a3, _vtap(t)) @ W4[t] for t in range(TAPS_V)) + P["b4"][0]
    cache = dict(x0=x0, a1=a1, a2=a2, a3=a3, rho=rho, W=(W1, W2, W3, W4), rnd=rnd)
    return delta.ravel(), cache


def apply(theta: np.ndarray, coef: np.ndarray, q: np.ndarray, bf16_round: bool = True) -> np.ndarray:
    """M(q) = T^{-1}(q + rho delta(q))."""
    delta, c = forward(theta, coef, q, bf16_round)
    return oracle.thomas(coef, np.asarray(q, dtype=np.float64).ravel() + c["rho"] * delta)


def transpose_coeffs(coef: np.ndarray) -> np.ndarray:
    """Coefficients of A^T as a 7-point operator: row c of A^T holds the couplings of the
    neighbours' rows to c (W'(i) = E(i-1), E'(i) = W(i+1), S'(j) = N(j-1), N'(j) = S(j+1),
    D'(k) = U(k-1), U'(k) = D(k+1)); the diagonal is unchanged."""
    ct = np.zeros_like(coef)
    ct[0] = np.roll(coef[1], 1, axis=2)
    ct[1] = np.roll(coef[0], -1, axis=2)
    ct[2, :, 1:] = coef[3, :, :-1]
    ct[3, :, :-1] = coef[2, :, 1:]
    ct[4, 1:] = coef[5, :-1]
    ct[5, :-1] = coef[4, 1:]
    ct[6] = coef[6]
    return ct


LOSS_ERROR, LOSS_RESIDUAL = 0, 1


def loss(theta, coef, r, e, bf16_round=True, kind=LOSS_ERROR) -> float:
    """kind 0: ||M(r) - e||^2 / ||e||^2;  kind 1: ||A M(r) - r||^2 / ||r||^2 (A e = r)."""
    m = apply(theta, coef, r, bf16_round)
    if kind == LOSS_RESIDUAL:
        r = np.asarray(r, dtype=np.float64).ravel()
        return float(np.sum((oracle.apply(coef, m) - r) ** 2) / np.sum(r * r))
    e = np.asarray(e, dtype=np.float64).ravel()
    return float(np.sum((m - e) ** 2) / np.sum(e * e))


def loss_and_grad(theta, coef, r, e, bf16_round: bool = True, kind: int = LOSS_ERROR):
    """Loss (see ``loss``) and its gradient with respect to theta (chain rule by hand: through
    A by A^T, through T^{-1} by T^{-T}, through each layer by the transposed convolution)."""
    r = np.asarray(r, dtype=np.float64).ravel()
    e = np.asarray(e, dtype=np.float64).ravel()
    delta, c = forward(theta, coef, r, bf16_round)
    rho, rnd = c["rho"], c["rnd"]
    W1, W2, W3, W4 = c["W"]
    m = oracle.thomas(coef, r + rho * delta)
    if kind == LOSS_RESIDUAL:
        d = oracle.apply(coef, m) - r
        rr = np.sum(r * r)
        L = float(np.sum(d * d) / rr)
        g_m = oracle.apply(transpose_coeffs(coef), 2.0 * d / rr)
    else:
        ee = np.sum(e * e)
        L = float(np.sum((m - e) ** 2) / ee)
        g_m = 2.0 * (m - e) / ee
    g_delta = (rho * thomas_transpose(coef, g_m)).reshape(c["a3"].shape[:3])
    G = {}
    # layer 4: delta = sum_t shift_v(a3, t) . W4[t] + b4
    G["b4"] = np.array([g_delta.sum()])
    G["W4"] = np.stack([np.einsum("kji,kjic->c", g_delta, _shift_v(c["a3"], _vtap(t))) for t in range(TAPS_V)])
    g_a3 = sum(_shift_v(g_delta[..., None] * W4[t], -_vtap(t)) for t in range(TAPS_V))
    g_z3 = rnd(g_a3 * (c["a3"] > 0))
    # layer 3
    G["b3"] = g_z3.sum(axis=(0, 1, 2))
    G["W3"] = np.stack([np.einsum("kjio,kjic->oc", g_z3, _shift_v(c["a2"], _vtap(t))) for t in range(TAPS_V)])
    g_a2 = sum(_shift_v(g_z3 @ W3[t], -_vtap(t)) for t in range(TAPS_V))
    g_z2 = rnd(g_a2 * (c["a2"] > 0))
    # layer 2
    G["b2"] = g_z2.sum(axis=(0, 1, 2))
    G["W2"] = np.stack([np.einsum("kjio,kjic->oc", g_z2, _shift_h(c["a1"], *_htap(t))) for t in range(TAPS_H)])
    g_a1 = sum(_shift_h(g_z2 @ W2[t], *(-d for d in _htap(t))) for t in range(TAPS_H))
    g_z1 = rnd(g_a1 * (c["a1"] > 0))
    # layer 1
    G["b1"] = g_z1.sum(axis=(0, 1, 2))
    G["W1"] = np.stack([np.einsum("kjio,kjic->oc", g_z1, _shift_v(c["x0"], _vtap(t))) for t in range(TAPS_V)])
    return L, pack(G)


class AdamState:
    """Optimiser state of ``adam_step``: first and second moment estimates and the step count."""

    def __init__(self, size: int):
        self.m = np.zeros(size)
        self.v = np.zeros(size)
        self.t = 0


def adam_step(theta: np.ndarray, grad: np.ndarray, state: AdamState, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8) -> np.ndarray:
    """One Adam update in FP64 (Kingma & Ba, ICLR 2015, Algorithm 1): exponential moving
    averages of the gradient and of its square, each divided by one minus its decay rate to
    the power t (the bias correction of the zero start), then a step of lr along the ratio of
    the corrected first moment to the square root of the corrected second moment plus eps.
    Updates ``state`` in place and returns the new parameters."""
    g = np.asarray(grad, dtype=np.float64)
    state.t += 1
    state.m = beta1 * state.m + (1.0 - beta1) * g
    state.v = beta2 * state.v + (1.0 - beta2) * (g * g)
    m_hat = state.m / (1.0 - beta1 ** state.t)
    v_hat = state.v / (1.0 - beta2 ** state.t)
    return np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)


def init_theta(seed: int) -> np.ndarray:
    """He-style random weights, zero biases, zero last layer (so M = T^{-1} at start)."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = rng.standard_normal((TAPS_V, C_HID, C_IN)) * np.sqrt(2.0 / (TAPS_V * C_IN))
    d["b1"] = np.zeros(C_HID)
    d["W2"] = rng.standard_normal((TAPS_H, C_HID, C_HID)) * np.sqrt(2.0 / (TAPS_H * C_HID))
    d["b2"] = np.zeros(C_HID)
    d["W3"] = rng.standard_normal((TAPS_V, C_HID, C_HID)) * np.sqrt(2.0 / (TAPS_V * C_HID))
    d["b3"] = np.zeros(C_HID)
    d["W4"] = np.zeros((TAPS_V, C_HID))
    d["b4"] = np.zeros(1)
    return pack(d)
