"""Pins for the red-black vertical-line SOR preconditioner of the oracle (the paper's tri_sor,
Sec. 2, Eq. 6-7, with red-black column order)."""
import numpy as np
import pytest

import oracle
import synth


def _problem(nlon=8, nlat=6, nlev=5, seed=3, shift=1e-3):
    p = synth.Problem(nlon, nlat, nlev, seed=seed, shift=shift)
    coef = synth.make_coeffs(p)
    q = np.random.default_rng(seed).standard_normal(p.n)
    return p, coef, q


def test_decoupled_columns_one_sweep_is_the_tridiagonal_solve():
    """No horizontal couplings: one sweep with omega = 1 solves every column exactly once."""
    p, coef, q = _problem()
    coef = coef.copy()
    coef[6] -= coef[:4].sum(axis=0)
    coef[:4] = 0.0
    z = oracle.rbsor(coef, q, sweeps=1, omega=1.0)
    assert np.array_equal(z, oracle.thomas(coef, q))


@pytest.mark.parametrize("half", [1, 2, 3, 4])
def test_updated_colour_satisfies_its_equations(half):
    """With omega = 1 a half-sweep solves the equations of the colour it updates exactly,
    given the other colour: (q - A x) vanishes on that colour's columns."""
    p, coef, q = _problem()
    z = oracle.rbsor(coef, q, omega=1.0, half_sweeps=half)
    res = (q - oracle.apply(coef, z)).reshape(p.shape)
    k, j, i = np.meshgrid(np.arange(p.nlev), np.arange(p.nlat), np.arange(p.nlon), indexing="ij")
    colour = (half - 1) % 2
    on = ((i + j) % 2 == colour)
    assert np.max(np.abs(res[on])) <= 1e-12 * np.max(np.abs(q))
    assert np.max(np.abs(res[~on])) > 1e-6        # the other colour is not yet consistent


def test_matches_block_sor_on_the_dense_matrix():
    """The same iteration written with the dense matrix split into its red and black blocks:
    x_R <- (1-w) x_R + w A_RR^{-1} (q_R - A_RB x_B), then the same for black."""
    p, coef, q = _problem(nlon=6, nlat=4, nlev=3)
    A = oracle.dense_matrix(coef)
    k, j, i = np.meshgrid(np.arange(p.nlev), np.arange(p.nlat), np.arange(p.nlon), indexing="ij")
    red = ((i + j) % 2 == 0).ravel()
    R, B = np.nonzero(red)[0], np.nonzero(~red)[0]
    for sweeps, w in ((1, 1.0), (3, 1.5), (2, 0.7)):
        x = np.zeros(p.n)
        for _ in range(sweeps):
            for S, O in ((R, B), (B, R)):
                x[S] = (1 - w) * x[S] + w * np.linalg.solve(A[np.ix_(S, S)], q[S] - A[np.ix_(S, O)] @ x[O])
        z = oracle.rbsor(coef, q, sweeps=sweeps, omega=w)
        assert np.allclose(z, x, rtol=1e-11, atol=1e-13 * np.max(np.abs(x)))


def test_linear_in_q():
    p, coef, q = _problem(seed=5)
    q2 = np.random.default_rng(9).standard_normal(p.n)
    lhs = oracle.rbsor(coef, 2.0 * q - 0.5 * q2)
    rhs = 2.0 * oracle.rbsor(coef, q) - 0.5 * oracle.rbsor(coef, q2)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.max(np.abs(rhs)))


@pytest.mark.parametrize("omega", [1.0, 1.5])
def test_many_sweeps_converge_to_the_solution(omega):
    p, coef, q = _problem(shift=1e-1)
    xd = oracle.dense_solve(coef, q)
    z = oracle.rbsor(coef, q, sweeps=400, omega=omega)
    assert np.linalg.norm(z - xd) <= 1e-9 * np.linalg.norm(xd)


def test_bicgstab_with_sor_matches_dense_solve():
    p, coef, q = _problem(nlon=10, nlat=8, nlev=6, seed=7)
    x, info = oracle.bicgstab(coef, q, tol=1e-12, precond=2)
    xd = oracle.dense_solve(coef, q)
    assert info.status == 0 and np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    _, info_t = oracle.bicgstab(coef, q, tol=1e-12, precond=1)
    assert info.iterations <= info_t.iterations    # three SOR sweeps precondition at least as well


def test_lexicographic_sor_matches_the_dense_gauss_seidel_splitting():
    """The paper's splitting in the natural column order: (T + omega L) x_n = (1 - omega) T x_{n-1} + omega (q - U x_{n-1}),
    with L / U the horizontal couplings to columns before / after in lexicographic order (Eq. 7),
    solved with the dense matrix."""
    p, coef, q = _problem(nlon=6, nlat=4, nlev=3)
    A = oracle.dense_matrix(coef)
    k, j, i = np.meshgrid(np.arange(p.nlev), np.arange(p.nlat), np.arange(p.nlon), indexing="ij")
    colidx = (i + p.nlon * j).ravel()                    # lexicographic position of each row's column
    same = colidx[:, None] == colidx[None, :]
    T = np.where(same, A, 0.0)
    L = np.where(colidx[None, :] < colidx[:, None], A, 0.0)
    U = np.where(colidx[None, :] > colidx[:, None], A, 0.0)
    for sweeps, w in ((1, 1.0), (3, 1.5)):
        x = np.zeros(p.n)
        for _ in range(sweeps):
            x = np.linalg.solve(T + w * L, (1 - w) * T @ x + w * (q - U @ x))
        z = oracle.lexsor(coef, q, sweeps=sweeps, omega=w)
        assert np.allclose(z, x, rtol=1e-11, atol=1e-13 * np.max(np.abs(x)))


def test_red_black_and_lexicographic_orders_precondition_alike():
    """BiCGStab iteration counts with the two column orders (3 sweeps, omega 1.5) on the
    96x72x20 operator: the red-black order the GPU uses is as strong as the natural one."""
    p = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    _, i_rb = oracle.bicgstab(coef, b, tol=1e-8, precond=2)
    _, i_lex = oracle.bicgstab(coef, b, tol=1e-8, precond=3)
    _, i_t = oracle.bicgstab(coef, b, tol=1e-8, precond=1)
    print(f"BiCGStab iterations: T^-1 {i_t.iterations}, red-black SOR {i_rb.iterations}, "
          f"lexicographic SOR {i_lex.iterations}")
    assert i_rb.status == i_lex.status == 0
    assert i_rb.iterations <= 1.5 * i_lex.iterations and i_lex.iterations < i_t.iterations
