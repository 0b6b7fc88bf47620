"""Pins for the emulation of the paper's mixed-precision BiCGStab (oracle/mp.py, Sec. 4)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mp


def _problem(**kw):
    p = synth.Problem(48, 36, 12, seed=kw.pop("seed", 3), **kw)
    return p, synth.make_coeffs(p), synth.make_rhs(p).ravel()


@pytest.mark.parametrize("precond,code", [("tri", 1), ("sor", 2)])
@pytest.mark.parametrize("restart_every", [0, 7])
def test_without_rounding_it_is_the_fp64_bicgstab(precond, code, restart_every):
    """vec_dtype float64: step for step the FP64 BiCGStab of the C oracle (the same operations
    in the same order: identical iteration count, status, residual history and x), periodic
    restarts included."""
    p, coef, b = _problem()
    x, info = mp.bicgstab_mp(coef, b, tol=1e-9, restart_every=restart_every, precond=precond, vec_dtype=np.float64)
    x_ref, ref = oracle.bicgstab(coef, b, tol=1e-9, restart_every=restart_every, precond=code)
    assert info.status == ref.status == 0
    assert info.iterations == ref.iterations
    k = len(info.history)
    assert np.array_equal(info.history, ref.history[:k])
    assert np.array_equal(x, x_ref)
    if restart_every:
        assert info.restarts >= info.iterations // restart_every


def test_fp32_vectors_round_and_still_converge():
    """With float32 vectors the history leaves the FP64 one by about the FP32 rounding, and the
    solve still reaches the paper's tolerances (1e-3, 1e-4) in about the FP64 iteration count."""
    p, coef, b = _problem()
    _, ref = oracle.bicgstab(coef, b, tol=1e-4, precond=1)
    x, info = mp.bicgstab_mp(coef, b, tol=1e-4)
    assert info.status == 0 and info.true_rel_residual <= 1e-4
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 5)
    d = np.abs(info.history[:3] - ref.history[:3]) / ref.history[:3]
    assert np.all(d < 1e-4) and np.any(d > 1e-9)      # rounded, but only at FP32 level
    rel = np.linalg.norm(b - oracle.apply(coef, x)) / np.linalg.norm(b)
    assert rel == pytest.approx(info.true_rel_residual, rel=1e-12)


def test_restarts_every_150_from_the_true_residual():
    """Shift 1e-6 needs a few hundred iterations: a restart every 150 iterations."""
    p, coef, b = _problem(shift=1e-6, seed=5)
    x, info = mp.bicgstab_mp(coef, b, tol=1e-5, maxit=3000)
    assert info.status == 0 and info.iterations > 150
    assert info.restarts >= info.iterations // 150
    assert np.linalg.norm(b - oracle.apply(coef, x)) / np.linalg.norm(b) <= 1e-5


def test_32_bit_solution_stalls_at_its_representation_floor():
    """x_dtype float32 (the all-32-bit solver of the paper's toy model, Sec. 4 / Fig. 1): the
    solution is held in 32 bits, so its true residual cannot fall below that of the exact
    solution rounded to float32 (from a dense LU solve, independent of the iteration); the same
    iteration with a 64-bit solution goes well below that floor."""
    p = synth.Problem(12, 8, 6, seed=4)
    coef, b = synth.make_coeffs(p), synth.make_rhs(p).ravel()
    x_star = oracle.dense_solve(coef, b)
    nb = np.linalg.norm(b)
    floor = np.linalg.norm(b - oracle.apply(coef, x_star.astype(np.float32).astype(np.float64))) / nb
    assert floor > 1e-9   # float32 rounding of x is visible in the residual at this conditioning
    x32, i32 = mp.bicgstab_mp(coef, b, tol=1e-14, maxit=300, restart_every=0, x_dtype=np.float32)
    x64, i64 = mp.bicgstab_mp(coef, b, tol=1e-14, maxit=300, restart_every=0)
    assert np.array_equal(x32, x32.astype(np.float32).astype(np.float64))
    r32 = np.linalg.norm(b - oracle.apply(coef, x32)) / nb
    r64 = np.linalg.norm(b - oracle.apply(coef, x64)) / nb
    print(f"floor {floor:.2e}, 32-bit x {r32:.2e}, 64-bit x {r64:.2e}")
    assert 0.3 * floor <= r32 <= 30 * floor
    assert r64 <= 0.1 * floor


def test_32_bit_solution_follows_the_64_bit_one_early():
    """Fig. 1's first observation: the two solvers' residual histories agree at first (here to
    FP32 level over the first iterations) and part later."""
    p, coef, b = _problem()
    _, i32 = mp.bicgstab_mp(coef, b, tol=1e-10, maxit=400, restart_every=0, x_dtype=np.float32)
    _, i64 = mp.bicgstab_mp(coef, b, tol=1e-10, maxit=400, restart_every=0)
    k = min(len(i32.history), len(i64.history), 4)
    d = np.abs(i32.history[:k] - i64.history[:k]) / i64.history[:k]
    assert np.all(d < 1e-4)


@pytest.mark.parametrize("precond", ["tri", "sor"])
def test_every_32_bit_vector_is_rounded_and_x_is_not(precond):
    """Sec. 4's split, checked on the emulation's state after every iteration: each of r, r^, p,
    p^ = M p, v = A p^, s, s^ = M s and t = A s^ holds float32 values only (a rounding dropped
    anywhere leaves float64 values in that vector), while the 64-bit solution x does not."""
    p, coef, b = _problem(seed=7)
    names = ("r", "rh", "p", "ph", "v", "s", "sh", "t")
    seen = []

    def check(it, st):
        for name in names:
            v = np.asarray(st[name], dtype=np.float64)
            assert np.array_equal(v, v.astype(np.float32).astype(np.float64)), (it, name)
        x = np.asarray(st["x"], dtype=np.float64)
        seen.append(not np.array_equal(x, x.astype(np.float32).astype(np.float64)))

    _, info = mp.bicgstab_mp(coef, b, tol=1e-6, precond=precond, trace=check)
    assert info.status == 0 and len(seen) >= 5
    assert all(seen)
