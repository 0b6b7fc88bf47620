"""Pins for the FP64 Krylov references with a changing preconditioner (oracle/krylov.py):
restarted flexible GMRES and flexible BiCGStab with the stall fallback."""
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


@pytest.mark.parametrize("eps_bd", [2.0 ** -52, 1e-2])
@pytest.mark.parametrize("code", [1, 0], ids=["tri", "identity"])
def test_flexible_bicgstab_with_fixed_m_is_the_c_oracle(code, eps_bd):
    """With the same M at every call the flexible BiCGStab is, bit for bit, the C oracle's
    BiCGStab (same iterations, restarts, residual history and x), breakdown restarts included."""
    p = synth.Problem(48, 24, 10, seed=7)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    M = (lambda q: oracle.thomas(coef, q)) if code == 1 else (lambda q: q.copy())
    x_ref, ref = oracle.bicgstab(coef, b, tol=1e-10, precond=code, eps_bd=eps_bd)
    x, info = krylov.bicgstab_flex(coef, b, M, tol=1e-10, eps_bd=eps_bd)
    assert info.status == ref.status == 0 and info.iterations == ref.iterations
    assert info.restarts == ref.restarts and info.fallbacks == 0
    assert np.array_equal(info.history, ref.history) and np.array_equal(x, x_ref)
    if eps_bd > 1e-10 and code == 1:
        assert ref.sigma_restarts >= 1 and ref.rho_restarts >= 1


def test_flexible_bicgstab_with_changing_m():
    """M alternates between the tridiagonal solve and two line-SOR sweeps from call to call:
    the iteration converges to the dense LU solution and, because x moves along exactly the
    preconditioned vectors that entered A, its recursive residual is the true one."""
    p = synth.Problem(16, 12, 8, seed=4)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    calls = [0]

    def M(q):
        calls[0] += 1
        return oracle.thomas(coef, q) if calls[0] % 2 else oracle.rbsor(coef, q, sweeps=2)

    x, info = krylov.bicgstab_flex(coef, b, M, tol=1e-12)
    x_ref = oracle.dense_solve(coef, b)
    assert info.status == 0 and calls[0] >= 2 * info.iterations - 1
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-10
    assert abs(info.true_rel_residual - info.history[-1]) <= 1e-13


def test_flexible_bicgstab_stall_falls_back():
    """A preconditioner that cannot carry the solve (T^{-1} of the wrong columns: the input
    rolled by one longitude) stalls; after stall_window iterations without halving the residual
    M becomes the tridiagonal solve, the iteration restarts from the true residual and converges
    to the dense LU solution."""
    p = synth.Problem(16, 12, 8, seed=4)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    nlev, nlat, nlon = coef.shape[1:]

    def bad(q):
        return np.roll(oracle.thomas(coef, q).reshape(nlev, nlat, nlon), 5, axis=2).ravel()

    tri = lambda q: oracle.thomas(coef, q)   # noqa: E731
    x, info = krylov.bicgstab_flex(coef, b, bad, tol=1e-12, fallback=tri, stall_window=20)
    assert info.fallbacks == 1 and info.status == 0
    x_ref = oracle.dense_solve(coef, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-10
    # without the fallback the same preconditioner does not reach the tolerance in that many steps
    _, stuck = krylov.bicgstab_flex(coef, b, bad, tol=1e-12, maxit=info.iterations)
    assert stuck.status != 0
