"""Pins for the CPU oracle: each test checks it against something other than itself
(closed forms, symmetry of the finite-volume operator, LAPACK solves, special cases)."""
import math

import numpy as np
import pytest
import scipy.linalg

import synth

EPS = np.finfo(np.float64).eps


def _eig_mode(nlon, nlat, nlev, mx, my, mz):
    i = np.arange(nlon)
    j = np.arange(nlat)
    k = np.arange(nlev)
    vx = np.cos(2 * math.pi * mx * i / nlon)
    vy = np.cos(math.pi * my * (j + 0.5) / nlat)
    vz = np.cos(math.pi * mz * (k + 0.5) / nlev)
    return vz[:, None, None] * vy[None, :, None] * vx[None, None, :]


@pytest.mark.parametrize("shape,modes", [((6, 5, 4), [(0, 0, 0), (1, 2, 3), (3, 4, 1), (5, 1, 2)]),
                                         ((16, 9, 7), [(2, 3, 5), (8, 8, 6), (1, 0, 1)])])
def test_apply_closed_form_eigenpairs(oracle_mod, shape, modes):
    """Constant-coefficient operator (periodic lon, zero-flux lat and vertical): Fourier/cosine
    eigenpairs  lambda = s + 2ax(1-cos 2 pi mx/nlon) + 2ay(1-cos pi my/nlat) + 2az(1-cos pi mz/nlev)."""
    nlon, nlat, nlev = shape
    ax, ay, az, s = 0.7, 0.3, 1.9, 1e-3
    coef = synth.constant_operator(nlon, nlat, nlev, ax, ay, az, s)
    for mx, my, mz in modes:
        v = _eig_mode(nlon, nlat, nlev, mx, my, mz).ravel()
        lam = (s + 2 * ax * (1 - math.cos(2 * math.pi * mx / nlon)) + 2 * ay * (1 - math.cos(math.pi * my / nlat))
               + 2 * az * (1 - math.cos(math.pi * mz / nlev)))
        y = oracle_mod.apply(coef, v)
        assert np.max(np.abs(y - lam * v)) <= 32 * EPS * (ax + ay + az + s) * 4 * np.max(np.abs(v))


def test_apply_lon_asymmetric_complex_eigenpair(oracle_mod):
    """aW != aE: e^{i theta i} is an eigenvector with eigenvalue
    (aW+aE)(1-cos theta) + i (aW-aE) sin theta (+ shift); swapping W and E flips the sign of
    the imaginary part, so this pins which neighbour each coupling belongs to."""
    nlon, nlat, nlev = 12, 3, 2
    aw, ae, s = 0.9, 0.2, 0.05
    coef = synth.constant_operator(nlon, nlat, nlev, aw, 0.0, 0.0, s, ax_e=ae)
    for m in (1, 2, 5):
        th = 2 * math.pi * m / nlon
        lam = complex(s + (aw + ae) * (1 - math.cos(th)), (aw - ae) * math.sin(th))
        ph = np.broadcast_to(np.exp(1j * th * np.arange(nlon)), (nlev, nlat, nlon)).ravel()
        y = oracle_mod.apply(coef, ph.real) + 1j * oracle_mod.apply(coef, ph.imag)
        assert np.max(np.abs(y - lam * ph)) < 1e-14


def test_apply_symmetric_finite_volume_operator(oracle_mod):
    """Before row scaling and perturbation the finite-volume operator is symmetric
    (aE(i) = aW(i+1), aN(j) = aS(j+1), aU(k) = aD(k+1)); <u, A v> = <A u, v> fails if the
    oracle pairs a coupling with the wrong neighbour in lat or height."""
    p = synth.Problem(10, 8, 6, perturb=0.0)
    coef = synth.make_raw_coeffs(p)
    coef = coef / coef[6].max()
    rng = np.random.default_rng(3)
    u = rng.standard_normal(p.n)
    v = rng.standard_normal(p.n)
    lhs = np.dot(u, oracle_mod.apply(coef, v))
    rhs = np.dot(oracle_mod.apply(coef, u), v)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(u) * np.linalg.norm(v))
    # and the perturbed, row-scaled operator is genuinely non-symmetric
    c2 = synth.make_coeffs(synth.Problem(10, 8, 6))
    l2 = np.dot(u, oracle_mod.apply(c2, v))
    r2 = np.dot(oracle_mod.apply(c2, u), v)
    assert abs(l2 - r2) > 1e-6


def test_apply_row_sums_equal_margin(oracle_mod):
    """A 1 = C - sum(a) = shift for the generator's operator (every neighbour term present)."""
    for p in (synth.Problem(9, 7, 5, shift=1e-3), synth.Problem(5, 1, 3, shift=0.25),
              synth.Problem(7, 4, 1, shift=2e-2), synth.Problem(8, 6, 9, shift=1e-6, bands=True)):
        coef = synth.make_coeffs(p)
        y = oracle_mod.apply(coef, np.ones(p.n))
        assert np.max(np.abs(y - p.shift)) <= 16 * EPS * coef[6].max()


def test_apply_matches_dense_assembly_and_points(oracle_mod):
    p = synth.Problem(7, 5, 4, seed=11)
    coef = synth.make_coeffs(p)
    A = oracle_mod.dense_matrix(coef)
    x = np.random.default_rng(0).standard_normal(p.n)
    y = oracle_mod.apply(coef, x)
    assert np.max(np.abs(y - A @ x)) < 1e-14 * np.abs(A).sum(axis=1).max() * np.abs(x).max() * 10
    idx = np.array([0, 1, 6, 7, 34, p.n - 1, p.n - 7, 5 * 7 + 3])
    assert np.array_equal(oracle_mod.apply_points(coef, x, idx), y[idx])


def test_thomas_closed_form_vertical_mode(oracle_mod):
    """For the constant operator, h(i,j) cos(pi m (k+1/2)/nlev) is an eigenvector of T with
    eigenvalue s + 2ax + c_j ay + 2az(1 - cos(pi m/nlev)), c_j = 1 on pole rows, else 2."""
    nlon, nlat, nlev = 5, 6, 9
    ax, ay, az, s = 0.4, 0.25, 3.0, 1e-2
    coef = synth.constant_operator(nlon, nlat, nlev, ax, ay, az, s)
    h = np.random.default_rng(1).standard_normal((nlat, nlon))
    cj = np.full(nlat, 2.0)
    cj[0] = cj[-1] = 1.0
    for m in range(nlev):
        vz = np.cos(math.pi * m * (np.arange(nlev) + 0.5) / nlev)
        v = vz[:, None, None] * h[None]
        lam = s + 2 * ax + cj * ay + 2 * az * (1 - math.cos(math.pi * m / nlev))
        z = oracle_mod.thomas(coef, v.ravel()).reshape(v.shape)
        ref = v / lam[None, :, None]
        assert np.max(np.abs(z - ref)) < 1e-12 * np.abs(ref).max() + 1e-15


def test_thomas_matches_lapack_banded(oracle_mod):
    """Per column the oracle equals LAPACK's banded solve of tridiag(-aD, C, -aU)."""
    p = synth.Problem(6, 5, 11, seed=4, shift=1e-6, bands=True)
    coef = synth.make_coeffs(p)
    q = np.random.default_rng(2).standard_normal(p.n)
    z = oracle_mod.thomas(coef, q).reshape(p.shape)
    q3 = q.reshape(p.shape)
    for j in range(p.nlat):
        for i in range(p.nlon):
            ab = np.zeros((3, p.nlev))
            ab[0, 1:] = -coef[5, :-1, j, i]
            ab[1] = coef[6, :, j, i]
            ab[2, :-1] = -coef[4, 1:, j, i]
            ref = scipy.linalg.solve_banded((1, 1), ab, q3[:, j, i])
            T = np.diag(ab[1]) + np.diag(ab[0, 1:], 1) + np.diag(ab[2, :-1], -1)
            # both are backward stable; forward errors scale with cond(T)
            tol = 8 * p.nlev * EPS * np.linalg.cond(T, np.inf) * np.abs(ref).max()
            assert np.max(np.abs(z[:, j, i] - ref)) <= tol


def test_thomas_inverts_decoupled_operator(oracle_mod):
    """With the horizontal couplings removed (C kept), A is exactly T: A (T^{-1} q) = q."""
    p = synth.Problem(8, 6, 13, seed=7)
    coef = synth.make_coeffs(p)
    coef[:4] = 0.0
    q = np.random.default_rng(5).standard_normal(p.n)
    z = oracle_mod.thomas(coef, q)
    assert np.max(np.abs(oracle_mod.apply(coef, z) - q)) < 1e-12 * np.abs(q).max()


@pytest.mark.parametrize("prob,tol", [(synth.Problem(8, 6, 5, seed=1), 1e-13), (synth.Problem(12, 8, 6, seed=2), 1e-13),
                                      (synth.Problem(8, 6, 12, seed=3, shift=1e-6, bands=True), 1e-10),
                                      (synth.Problem(5, 1, 7, seed=4), 1e-13), (synth.Problem(9, 4, 1, seed=5), 1e-13)])
def test_bicgstab_matches_dense_lu(oracle_mod, prob, tol):
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    A = oracle_mod.dense_matrix(coef)
    x_ref = np.linalg.solve(A, b)
    x, info = oracle_mod.bicgstab(coef, b, tol=tol)
    assert info.status == 0
    assert info.true_rel_residual <= tol
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    # classical forward-error bound (plus the rounding of the LU reference itself)
    assert err <= kappa * (info.true_rel_residual * 1.01 + 16 * EPS)
    if prob.shift >= 1e-3:
        assert err <= 1e-10


def test_bicgstab_reports_stall_below_attainable_accuracy(oracle_mod):
    """Near-singular operator (shift 1e-6): a tolerance below the FP64 attainable accuracy
    (about eps * cond(A)) cannot be met by the true residual; the oracle says so (status 3)."""
    prob = synth.Problem(8, 6, 12, seed=3, shift=1e-6, bands=True)
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-15)
    assert info.status == 3
    assert info.true_rel_residual > 1e-15


def test_bicgstab_unpreconditioned_matches_dense_lu(oracle_mod):
    prob = synth.Problem(8, 6, 5, seed=9)
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    x_ref = oracle_mod.dense_solve(coef, b)
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-13, precond=0)
    assert info.status == 0
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-10


def test_bicgstab_manufactured_solution_forward_error(oracle_mod):
    """b = A x* (dense product); the forward error obeys ||x - x*|| / ||x*|| <= cond(A) R_true."""
    prob = synth.Problem(16, 12, 8, seed=6)
    coef = synth.make_coeffs(prob)
    xs = synth.make_xstar(prob).ravel()
    A = oracle_mod.dense_matrix(coef)
    b = A @ xs
    kappa = np.linalg.cond(A)
    for tol in (1e-6, 1e-8, 1e-10):
        x, info = oracle_mod.bicgstab(coef, b, tol=tol)
        assert info.status == 0 and info.true_rel_residual <= tol
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        assert err <= kappa * info.true_rel_residual * 1.01 + 1e-14


def test_bicgstab_decoupled_columns_one_half_step(oracle_mod):
    """a^{W,E,S,N} = 0: M = T^{-1} = A^{-1}, so the first half step is exact."""
    prob = synth.Problem(7, 5, 9, seed=8)
    coef = synth.make_coeffs(prob)
    coef[:4] = 0.0
    b = synth.make_rhs(prob).ravel()
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-12)
    assert info.iterations == 1 and info.half_step_exit == 1 and info.status == 0
    x_ref = oracle_mod.dense_solve(coef, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-13


def test_bicgstab_eigenmode_identity_preconditioner(oracle_mod):
    """b an eigenvector of the constant operator, M = I: alpha = 1/lambda and x = b/lambda."""
    nlon, nlat, nlev = 8, 6, 5
    ax, ay, az, s = 0.5, 0.2, 1.5, 1e-3
    coef = synth.constant_operator(nlon, nlat, nlev, ax, ay, az, s)
    v = _eig_mode(nlon, nlat, nlev, 3, 2, 1).ravel()
    lam = (s + 2 * ax * (1 - math.cos(2 * math.pi * 3 / nlon)) + 2 * ay * (1 - math.cos(math.pi * 2 / nlat))
           + 2 * az * (1 - math.cos(math.pi * 1 / nlev)))
    x, info = oracle_mod.bicgstab(coef, v, tol=1e-12, precond=0)
    assert info.iterations == 1 and info.half_step_exit == 1
    assert np.max(np.abs(x - v / lam)) < 1e-13 * np.abs(v / lam).max()


def test_bicgstab_history_and_special_cases(oracle_mod):
    prob = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-8)
    h = info.history
    assert info.status == 0 and len(h) == info.iterations
    assert h[-1] <= 1e-8 and info.true_rel_residual <= 1e-8
    assert np.all(np.minimum.accumulate(h)[-1] == h.min())
    # BiCGStab is not monotone (Sec. 4 shows non-monotone R), but it must make progress
    assert np.sum(np.diff(h) > 0) > 0
    # zero right-hand side -> zero solution, no iterations
    x0, i0 = oracle_mod.bicgstab(coef, np.zeros(prob.n), tol=1e-8)
    assert i0.iterations == 0 and not np.any(x0)
    # starting from the solution -> no iterations
    x1, i1 = oracle_mod.bicgstab(coef, b, x0=x, tol=1e-8)
    assert i1.iterations == 0 and np.array_equal(x1, x)
    # iteration limit
    _, i2 = oracle_mod.bicgstab(coef, b, tol=1e-8, maxit=5)
    assert i2.status == 1 and i2.iterations == 5


def test_bicgstab_periodic_restart(oracle_mod):
    """A mandatory restart every 20 iterations (Sec. 4 uses 150 operationally) still converges."""
    prob = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    x_ref, _ = oracle_mod.bicgstab(coef, b, tol=1e-11)
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-9, restart_every=20)
    assert info.status == 0 and info.true_rel_residual <= 1e-9
    assert info.restarts >= (info.iterations - 1) // 20
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-6


def test_dot_exact_on_integers(oracle_mod):
    rng = np.random.default_rng(0)
    a = rng.integers(-1000, 1000, 100000).astype(np.float64)
    b = rng.integers(-1000, 1000, 100000).astype(np.float64)
    assert oracle_mod.dot(a, b) == float(np.dot(a.astype(np.int64), b.astype(np.int64)))


def test_bicgstab_breakdown_restarts_reach_dense_solution(oracle_mod):
    """Breakdown guards of Sec. 4 forced with a threshold of 1e-2 on the relative cosines: the
    iteration restarts once after <rhat, v> and once after <rhat, r> fell below it, and still
    converges to the dense LU solution; up to the first restart it is bitwise the run with the
    default threshold (the guard changes nothing until it fires)."""
    prob = synth.Problem(24, 16, 10, seed=1)
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    x_ref = oracle_mod.dense_solve(coef, b)
    x, info = oracle_mod.bicgstab(coef, b, tol=1e-12, eps_bd=1e-2)
    assert info.status == 0 and info.sigma_restarts == 1 and info.rho_restarts == 1
    assert info.restarts == 2
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-10
    _, plain = oracle_mod.bicgstab(coef, b, tol=1e-12)
    assert plain.restarts == 0
    h, hp = info.history, plain.history
    m = min(h.size, hp.size)
    first = int(np.argmax(h[:m] != hp[:m]))
    assert first >= 1 and np.array_equal(h[:first], hp[:first])


def test_openmp_build_agrees_with_single_thread(oracle_mod):
    """The OpenMP build of the same source: SpMV and tridiagonal solve bitwise equal to the
    single-threaded build, inner products equal up to summation order, and the whole solve at
    tol 1e-12 within 1e-11 of the single-threaded oracle."""
    prob = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(prob)
    b = synth.make_rhs(prob).ravel()
    assert np.array_equal(oracle_mod.apply(coef, b), oracle_mod.apply(coef, b, parallel=True))
    assert np.array_equal(oracle_mod.thomas(coef, b), oracle_mod.thomas(coef, b, parallel=True))
    d1, d2 = oracle_mod.dot(b, b), oracle_mod.dot(b, b, parallel=True)
    assert abs(d1 - d2) <= 1e-14 * d1
    rng = np.random.default_rng(1)
    ia = rng.integers(-1000, 1000, 100003).astype(np.float64)
    assert oracle_mod.dot(ia, ia, parallel=True) == float(np.dot(ia.astype(np.int64), ia.astype(np.int64)))
    x1, i1 = oracle_mod.bicgstab(coef, b, tol=1e-12)
    x2, i2 = oracle_mod.bicgstab(coef, b, tol=1e-12, parallel=True)
    assert i1.status == i2.status == 0 and abs(i1.iterations - i2.iterations) <= 2
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) <= 1e-11
