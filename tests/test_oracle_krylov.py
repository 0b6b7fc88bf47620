"""Pins for the FP64 restarted flexible GMRES reference (oracle/krylov.py)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import krylov


def _tiny(seed=4, **kw):
    p = synth.Problem(6, 4, 3, seed=seed, **kw)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    return p, coef, b


def test_full_cycle_is_a_direct_solve():
    """m = n: one cycle reaches the exact solution (the Krylov space spans everything)."""
    p, coef, b = _tiny()
    x, info = krylov.fgmres(coef, b, tol=1e-12, m=p.n)
    assert info.status == 0 and info.cycles == 1
    xd = oracle.dense_solve(coef, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_residual_is_the_krylov_minimum(k):
    """After k steps with a fixed M the residual is min over y of ||r0 - A M K_k y||, K_k the
    Krylov space of A M on r0 (least squares over an explicitly built basis)."""
    p, coef, b = _tiny(seed=7)
    A = oracle.dense_matrix(coef)
    M = np.stack([oracle.thomas(coef, e) for e in np.eye(p.n)], axis=1)
    AM = A @ M
    K = [b]
    for _ in range(k - 1):
        K.append(AM @ K[-1])
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    y = np.linalg.lstsq(AM @ Q, b, rcond=None)[0]
    rmin = np.linalg.norm(b - AM @ Q @ y) / np.linalg.norm(b)
    _, info = krylov.fgmres(coef, b, tol=0.0, m=k, maxit=k)
    assert info.iterations == k
    assert info.history[-1] == pytest.approx(rmin, rel=1e-8, abs=1e-14)
    assert info.true_rel_residual == pytest.approx(rmin, rel=1e-8, abs=1e-12)


def test_restarted_history_is_monotone_and_true():
    p, coef, b = _tiny(seed=9)
    x, info = krylov.fgmres(coef, b, tol=1e-12, m=3, maxit=2000)
    assert info.status == 0 and info.cycles > 1
    h = info.history
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-9))
    rel = np.linalg.norm(b - oracle.apply(coef, x)) / np.linalg.norm(b)
    assert rel <= 1e-12 and rel == pytest.approx(info.true_rel_residual)


def test_flexible_preconditioner():
    """A preconditioner that changes every step (T^{-1} on even steps, a scaled identity on odd
    ones): the iteration still minimises over the stored z_j, so its estimate equals the true
    residual at the end of the cycle and the solve converges."""
    p, coef, b = _tiny(seed=11)
    pc = lambda j, v: oracle.thomas(coef, v) if j % 2 == 0 else v / coef[6].ravel()   # noqa: E731
    x, info = krylov.fgmres(coef, b, tol=1e-11, m=8, maxit=3000, precond=pc)
    assert info.status == 0
    rel = np.linalg.norm(b - oracle.apply(coef, x)) / np.linalg.norm(b)
    assert rel <= 1e-11


def test_identity_preconditioner_on_diagonal_system():
    """A diagonal operator (all couplings zero) with M = I: the Krylov space of a diagonal
    matrix on b has dimension = number of distinct diagonal values, so GMRES ends after that
    many steps."""
    p = synth.Problem(4, 3, 2, seed=1)
    coef = np.zeros((7,) + p.shape)
    diag = np.array([1.0, 2.0, 3.0])
    coef[6] = diag[np.arange(p.n) % 3].reshape(p.shape)
    b = np.random.default_rng(0).standard_normal(p.n)
    x, info = krylov.fgmres(coef, b, tol=1e-13, m=10, precond=lambda j, v: v)
    assert info.status == 0 and info.iterations == 3
    assert np.allclose(x, b / coef[6].ravel(), rtol=1e-12)
