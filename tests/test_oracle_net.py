"""Pins for the FP64 reference of the learned preconditioner (oracle/net.py)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import net


def _small():
    p = synth.Problem(8, 6, 7, seed=3)
    coef = synth.make_coeffs(p)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(p.n)
    e = rng.standard_normal(p.n)
    th = net.init_theta(5)
    d = net.unpack(th)
    d["W4"] = rng.standard_normal(d["W4"].shape) * 0.3
    d["b1"] = rng.standard_normal(32) * 0.1
    d["b3"] = rng.standard_normal(32) * 0.1
    d["b4"] = np.array([0.05])
    return p, coef, r, e, net.pack(d)


def test_parameter_count():
    assert net.N_PARAMS == 15233


@pytest.mark.parametrize("kind", [net.LOSS_ERROR, net.LOSS_RESIDUAL])
def test_gradient_matches_central_differences(kind):
    """Plain FP64 network: the hand-written backward pass agrees with central differences."""
    p, coef, r, e, th = _small()
    L, g = net.loss_and_grad(th, coef, r, e, bf16_round=False, kind=kind)
    rng = np.random.default_rng(7)
    # a sample of parameters from every tensor
    offs, o = [], 0
    for _, shape in net.SHAPES:
        size = int(np.prod(shape))
        offs.extend(o + rng.choice(size, size=min(size, 12), replace=False))
        o += size
    h = 1e-6
    fd = []
    for i in offs:
        tp = th.copy()
        tp[i] += h
        tm = th.copy()
        tm[i] -= h
        fd.append((net.loss(tp, coef, r, e, False, kind) - net.loss(tm, coef, r, e, False, kind)) / (2 * h))
    fd = np.array(fd)
    ga = g[offs]
    assert np.linalg.norm(fd - ga) <= 1e-6 * np.linalg.norm(ga), (np.linalg.norm(fd - ga), np.linalg.norm(ga))


def test_transposed_thomas_is_the_adjoint():
    p = synth.Problem(9, 5, 11, seed=2, shift=1e-6, bands=True)
    coef = synth.make_coeffs(p)
    rng = np.random.default_rng(3)
    a = rng.standard_normal(p.n)
    b = rng.standard_normal(p.n)
    lhs = np.dot(oracle.thomas(coef, a), b)
    rhs = np.dot(a, net.thomas_transpose(coef, b))
    assert abs(lhs - rhs) <= 1e-9 * (abs(lhs) + 1.0) * np.linalg.norm(a) * np.linalg.norm(b)


def test_zero_last_layer_is_plain_tridiagonal():
    p, coef, r, _, _ = _small()
    th = net.init_theta(11)
    assert np.array_equal(net.apply(th, coef, r), oracle.thomas(coef, r))


def test_lon_translation_equivariance():
    """Rolling the right-hand side and the operator in longitude rolls the correction."""
    p, coef, r, _, th = _small()
    d1, _ = net.forward(th, coef, r, bf16_round=False)
    s = 3
    coef_r = np.roll(coef, s, axis=3)
    r_r = np.roll(r.reshape(p.shape), s, axis=2).ravel()
    d2, _ = net.forward(th, coef_r, r_r, bf16_round=False)
    assert np.allclose(np.roll(d1.reshape(p.shape), s, axis=2).ravel(), d2, rtol=1e-12, atol=1e-12)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, 3.0e-3, -2.5, 0.0, 1.0 + 2 ** -8])
    y = net.bf16(x)
    assert y[0] == 1.0 and y[1] == 1.0   # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even
    assert y[2] == 1.0078125               # above the tie: rounds up
    assert y[5] == 0.0 and y[4] == -2.5
    # agrees with torch's float32 -> bfloat16 conversion on float32-exact inputs
    import torch
    v = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    t = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(v.astype(np.float64)), t)


def test_transpose_coefficients_give_the_adjoint():
    """<A x, y> = <x, A^T y> with A^T applied as a 7-point operator (non-symmetric operator,
    periodic longitude, pole and top/bottom rows)."""
    p = synth.Problem(9, 6, 5, seed=12)
    coef = synth.make_coeffs(p)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(p.n)
    y = rng.standard_normal(p.n)
    lhs = np.dot(oracle.apply(coef, x), y)
    rhs = np.dot(x, oracle.apply(net.transpose_coeffs(coef), y))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * 10
    A = oracle.dense_matrix(coef)
    assert np.allclose(oracle.dense_matrix(net.transpose_coeffs(coef)), A.T, rtol=0, atol=1e-15)


def _golden_adam():
    path = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "adam_two_steps.txt")
    rows = [list(map(float, ln.split())) for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return np.array(rows)


def test_adam_two_steps_match_hand_worked_example():
    """Two Adam steps on three parameters (one of them with a zero first gradient) against the
    values worked out by hand in decimal arithmetic (tests/golden/adam_two_steps.txt)."""
    g = _golden_adam()
    st = net.AdamState(3)
    th1 = net.adam_step(g[:, 0], g[:, 1], st, lr=0.1)
    assert np.allclose(st.m, g[:, 3], rtol=1e-14, atol=1e-18) and np.allclose(st.v, g[:, 4], rtol=1e-14, atol=1e-22)
    assert np.allclose(th1, g[:, 5], rtol=1e-15, atol=0)
    th2 = net.adam_step(th1, g[:, 2], st, lr=0.1)
    assert np.allclose(st.m, g[:, 6], rtol=1e-14, atol=0) and np.allclose(st.v, g[:, 7], rtol=1e-14, atol=0)
    # 1 - b2^2 = 0.001999 cancels three digits: a few units in the last place
    assert np.allclose(th2, g[:, 8], rtol=5e-15, atol=0)
    assert st.t == 2


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g the bias-corrected moments are exactly g and g^2 at every
    step, so each step moves every parameter by lr g / (|g| + eps): a step of lr against the
    gradient's sign whatever its scale (a missing correction or swapped decay rates would give
    steps that grow or shrink with t)."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50) * np.logspace(-6, 3, 50)
    th0 = rng.standard_normal(50)
    st = net.AdamState(50)
    th = th0
    for t in range(1, 6):
        th = net.adam_step(th, g, st, lr=1e-2)
        assert np.allclose(th, th0 - t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
