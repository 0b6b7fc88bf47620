"""Solver parity: the HIP BiCGStab against the CPU oracle, in every precision mode, plus special
cases, failure paths and determinism."""
import numpy as np
import pytest

import synth
from tests.helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eg():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    return eg


@pytest.fixture(scope="module")
def small(oracle_mod):
    """The small configuration and its oracle solution at tol 1e-12."""
    p = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    x_ref, info = oracle_mod.bicgstab(coef, b, tol=1e-12)
    assert info.status == 0
    return p, coef, b, x_ref, info


def _true_rel(oracle_mod, coef, b, x):
    return np.linalg.norm(b - oracle_mod.apply(coef, x)) / np.linalg.norm(b)


def test_fp64_parity_tight_tolerance(eg, oracle_mod, small):
    """Both solvers at tol 1e-12: the GPU x matches the oracle x to 1e-10 relative L2."""
    import torch
    p, coef, b, x_ref, info_ref = small
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol=1e-12, maxit=5000, mode=eg.FP64)
        xh = host(x)
        assert info.status == eg.CONVERGED
        assert _true_rel(oracle_mod, coef, b, xh) <= 1e-12
        err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
        assert err <= 1e-10, err
        # the two iterations follow the same recurrences: counts agree closely
        assert abs(info.iterations - info_ref.iterations) <= max(3, info_ref.iterations // 10)
        hist = op.history()
        assert len(hist) == info.iterations and hist[-1] <= 1e-12


@pytest.mark.parametrize("p", [synth.Problem(67, 13, 9, seed=1), synth.Problem(130, 37, 5, seed=2),
                               synth.Problem(40, 30, 24, seed=5, shift=1e-6, bands=True, ratio=synth._stress_ratio()),
                               synth.Problem(64, 16, 70, seed=4),
                               # 140 levels, whole waves of columns: the FP64 tridiagonal kernels
                               # at one wave per SIMD
                               synth.Problem(128, 8, 140, seed=8, shift=1e-6, bands=True, ratio=synth._stress_ratio())],
                         ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_fp64_parity_shapes(eg, oracle_mod, p):
    import torch
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    tol = 1e-12 if p.shift >= 1e-3 else 1e-10
    x_ref, info_ref = oracle_mod.bicgstab(coef, b, tol=tol)
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol=tol, maxit=20000, mode=eg.FP64)
        assert info.status == eg.CONVERGED
        xh = host(x)
        assert _true_rel(oracle_mod, coef, b, xh) <= tol
        err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
        assert err <= (1e-10 if p.shift >= 1e-3 else 1e-7), err


@pytest.mark.parametrize("p", [synth.Problem(48, 24, 10, seed=7), synth.Problem(64, 32, 16, seed=3)],
                         ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_breakdown_restarts_follow_oracle(eg, oracle_mod, p):
    """A breakdown threshold of 1e-2 (option eps_bd; the cosine guards of Sec. 4) forces both
    kinds of restart: after <rhat, r> and after <rhat, v> fall below it.  The GPU takes the same
    restarts at the same iterations as the oracle, its residual history follows the oracle's and
    x agrees (the restart after a <rhat, v> breakdown restarts the recurrence from ||r||^2)."""
    import torch
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    x_ref, info_ref = oracle_mod.bicgstab(coef, b, tol=1e-10, eps_bd=1e-2)
    assert info_ref.status == 0 and info_ref.sigma_restarts >= 1 and info_ref.rho_restarts >= 1
    with eg.Operator(dev(coef)) as op:
        op.set_option("eps_bd", 1e-2)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol=1e-10, maxit=2000, mode=eg.FP64)
        hist = op.history()
    print(f"{p.nlon}x{p.nlat}x{p.nlev}: GPU {info.iterations} its {info.restarts} restarts, oracle "
          f"{info_ref.iterations} its {info_ref.restarts} restarts ({info_ref.sigma_restarts} after <rhat, v>)")
    assert info.status == eg.CONVERGED
    assert info.iterations == info_ref.iterations and info.restarts == info_ref.restarts
    dh = np.max(np.abs(hist - info_ref.history) / info_ref.history)
    assert dh <= 1e-6, dh
    err = np.linalg.norm(host(x) - x_ref) / np.linalg.norm(x_ref)
    assert err <= 1e-8, err


@pytest.mark.parametrize("mode_name", ["FP64", "FP32_IR", "FP32_IR_BF16", "FP32_IR_FP16"])
def test_modes_reach_1e8_true_residual(eg, oracle_mod, small, mode_name):
    """Every precision mode reaches ||b - A x|| / ||b|| <= 1e-8, checked by the oracle's FP64
    product on the returned x; the error against the FP64 oracle solution is reported."""
    import torch
    p, coef, b, x_ref, _ = small
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol=1e-8, maxit=20000, mode=getattr(eg, mode_name))
        xh = host(x)
        assert info.status == eg.CONVERGED, info
        rel = _true_rel(oracle_mod, coef, b, xh)
        assert rel <= 1e-8 and abs(rel - info.true_rel_residual) <= 1e-10
        err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
        print(f"{mode_name}: iterations {info.iterations} outer {info.outer_steps} true R {rel:.3e} "
              f"error vs oracle {err:.3e}")
        assert err <= 1e-5
        if mode_name != "FP64":
            assert info.outer_steps >= 1


def test_refinement_outer_residuals_fall_by_eta(eg, oracle_mod, small):
    """Each FP64 refinement step reduces the true residual by at least 10x."""
    import torch
    p, coef, b, _, _ = small
    with eg.Operator(dev(coef)) as op:
        op.set_option("eta", 1e-3)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        rels = []
        for k in range(1, 4):
            op.set_option("max_outer", k)
            x.zero_()
            info = op.solve(dev(b), x, tol=1e-14, maxit=20000, mode=eg.FP32_IR)
            rels.append(_true_rel(oracle_mod, coef, b, host(x)))
        assert rels[1] <= 0.1 * rels[0] and rels[2] <= 0.1 * rels[1], rels


@pytest.mark.parametrize("method", [0, 1], ids=["bicgstab", "fgmres"])
def test_capped_inner_solves_still_refine(eg, oracle_mod, small, method):
    """Option inner_maxit: every inner FP32 solve stops after 10 iterations, far from eta; the
    refinement keeps each correction that lowers the FP64 true residual and still reaches 1e-8,
    in more outer steps."""
    import torch
    p, coef, b, _, _ = small
    with eg.Operator(dev(coef)) as op:
        op.set_option("method", method)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        free = op.solve(dev(b), x, 1e-8, 20000, eg.FP32_IR)
        op.set_option("inner_maxit", 10)
        x.zero_()
        info = op.solve(dev(b), x, 1e-8, 20000, eg.FP32_IR)
        for bad in (0, 2.5):
            with pytest.raises(eg.EndgameError):
                op.set_option("inner_maxit", bad)
    rel = _true_rel(oracle_mod, coef, b, host(x))
    print(f"inner_maxit 10: {info.outer_steps} outer steps, {info.iterations} its (uncapped: {free.outer_steps} "
          f"outer, {free.iterations} its), {info.fallbacks} fallbacks, true R {rel:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-8 and info.fallbacks == 0
    assert info.outer_steps > free.outer_steps and info.iterations <= 10 * info.outer_steps


def test_special_cases(eg, oracle_mod, small):
    import torch
    p, coef, b, x_ref, _ = small
    with eg.Operator(dev(coef)) as op:
        # b = 0 -> x = 0
        x = torch.randn(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(torch.zeros(p.n, dtype=torch.float64, device="cuda"), x, 1e-8, 100, eg.FP64)
        assert info.status == eg.CONVERGED and not torch.any(x)
        # start at the solution -> no iteration
        x = dev(x_ref)
        info = op.solve(dev(b), x, 1e-8, 100, eg.FP64)
        assert info.status == eg.CONVERGED and info.iterations == 0
        # iteration limit
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-8, 5, eg.FP64)
        assert info.status == eg.MAXIT and info.iterations == 5
        # non-finite input
        bad = dev(b)
        bad[17] = float("nan")
        with pytest.raises(eg.EndgameError) as ei:
            op.solve(bad, torch.zeros_like(bad), 1e-8, 100, eg.FP64)
        assert ei.value.code == eg.ENONFINITE
        with pytest.raises(eg.EndgameError) as ei:
            op.solve(dev(b), torch.zeros_like(bad), 1e-8, 100, eg.LEARNED_FP64)
        assert ei.value.code == eg.ENOPC
        with pytest.raises(eg.EndgameError):
            op.solve(dev(b), torch.zeros_like(bad), -1.0, 100, eg.FP64)


def test_decoupled_columns_converge_in_one_half_step(eg, oracle_mod):
    import torch
    p = synth.Problem(70, 20, 11, seed=8)
    coef = synth.make_coeffs(p)
    coef[:4] = 0.0
    b = synth.make_rhs(p).ravel()
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-12, 100, eg.FP64)
        assert info.status == eg.CONVERGED and info.iterations == 1
        ref = oracle_mod.thomas(coef, b)
        assert np.max(np.abs(host(x) - ref)) <= 1e-13 * np.abs(ref).max()


def test_periodic_restart(eg, oracle_mod, small):
    import torch
    p, coef, b, x_ref, _ = small
    with eg.Operator(dev(coef)) as op:
        op.set_option("restart_every", 20)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-9, 20000, eg.FP64)
        assert info.status == eg.CONVERGED and info.restarts >= (info.iterations - 1) // 20
        assert _true_rel(oracle_mod, coef, b, host(x)) <= 1e-9
        _, oi = oracle_mod.bicgstab(coef, b, tol=1e-9, restart_every=20)
        assert abs(oi.iterations - info.iterations) <= max(3, oi.iterations // 10)


def test_bitwise_deterministic(eg, small):
    import torch
    p, coef, b, _, _ = small
    with eg.Operator(dev(coef)) as op:
        outs = []
        for _ in range(2):
            for mode in (eg.FP64, eg.FP32_IR_BF16):
                x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
                op.solve(dev(b), x, 1e-8, 20000, mode)
                outs.append((host(x), op.history()))
        for a, b2 in zip(outs[:2], outs[2:]):
            assert np.array_equal(a[0], b2[0]) and np.array_equal(a[1], b2[1])


def test_fgmres_fp64_matches_oracle(eg, oracle_mod, small):
    """Restarted FGMRES(30) with T^{-1}: the same residual history as the FP64 oracle FGMRES
    (the same method; the GPU orthogonalises by classical Gram-Schmidt applied twice, the oracle
    by modified Gram-Schmidt, equal in exact arithmetic) and the same solution."""
    import torch
    from oracle import krylov
    p, coef, b, x_ref, _ = small
    x_o, info_o = krylov.fgmres(coef, b, tol=1e-10, m=30, maxit=3000)
    assert info_o.status == 0
    with eg.Operator(dev(coef)) as op:
        op.set_option("method", 1)
        op.set_option("gmres_m", 30)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-10, 3000, eg.FP64)
        h = op.history()
    xh = host(x)
    rel = _true_rel(oracle_mod, coef, b, xh)
    k = min(len(h), len(info_o.history), 60)
    hdiff = np.max(np.abs(h[:k] - info_o.history[:k]) / info_o.history[:k])
    print(f"FGMRES: GPU {info.iterations} its, oracle {info_o.iterations}; history rel diff (first {k}) "
          f"{hdiff:.1e}; true R {rel:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-10
    assert abs(info.iterations - info_o.iterations) <= 2 and len(h) == info.iterations
    assert hdiff <= 1e-6
    assert np.linalg.norm(xh - x_o) <= 1e-7 * np.linalg.norm(x_o)


@pytest.mark.parametrize("mode_name", ["FP32_IR", "FP32_IR_BF16"])
def test_fgmres_refinement_modes_reach_1e8(eg, oracle_mod, small, mode_name):
    import torch
    p, coef, b, x_ref, _ = small
    with eg.Operator(dev(coef)) as op:
        op.set_option("method", 1)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-8, 5000, getattr(eg, mode_name))
    xh = host(x)
    rel = _true_rel(oracle_mod, coef, b, xh)
    print(f"FGMRES {mode_name}: {info.iterations} its, {info.outer_steps} outer, true R {rel:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-8 and info.outer_steps >= 2
    assert np.linalg.norm(xh - x_ref) <= 1e-5 * np.linalg.norm(x_ref)


def test_fgmres_options_are_checked(eg, small):
    p, coef, b, _, _ = small
    with eg.Operator(dev(coef)) as op:
        for key, bad in (("method", 2), ("learned_method", -1), ("gmres_m", 0), ("gmres_m", 65)):
            with pytest.raises(eg.EndgameError):
                op.set_option(key, bad)


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_paper_mixed_precision_mode(eg, oracle_mod, small, tol):
    """The paper's MP BiCGStab (FP32 vectors, FP64 solution and sums, no refinement) at the
    tolerances the paper uses: converges with about the FP64 iteration count."""
    import torch
    p, coef, b, x_ref, _ = small
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol, 5000, eg.FP32_MP)
        i64 = op.solve(dev(b), torch.zeros_like(x), tol, 5000, eg.FP64)
    xh = host(x)
    rel = _true_rel(oracle_mod, coef, b, xh)
    err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
    print(f"MP tol {tol:g}: {info.iterations} its (FP64 {i64.iterations}), true R {rel:.2e}, error {err:.2e}")
    assert info.status == eg.CONVERGED and rel <= tol and info.outer_steps == 0
    assert abs(info.iterations - i64.iterations) <= max(3, i64.iterations // 5)
    assert err <= 1e4 * tol


@pytest.mark.parametrize("precond", [0, 1], ids=["tri", "line_sor"])
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_paper_mixed_precision_matches_the_mp_oracle(eg, oracle_mod, small, precond, tol):
    """EG_FP32_MP against the CPU emulation of the paper's mixed-precision BiCGStab (FP32
    vectors, FP64 x and sums, restart every 150; oracle/mp.py): the first residual-history
    entries agree to FP32 rounding (eight with T^-1 within 2e-5, measured 5e-6; four with the
    line SOR within 5e-5, measured 9e-6; later entries part as BiCGStab amplifies the two
    sides' different rounding orders), the iteration counts within 10 %, and both true
    residuals are below tol."""
    import torch
    from oracle import mp
    p, coef, b, x_ref, _ = small
    xo, ref = mp.bicgstab_mp(coef, b, tol=tol, precond="sor" if precond else "tri")
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", precond)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, tol, 5000, eg.FP32_MP)
        h = op.history()
    xh = host(x)
    print(f"MP {'line SOR' if precond else 'T^-1'} tol {tol:g}: GPU {info.iterations} its, oracle {ref.iterations}; "
          f"history[:4] GPU {np.array2string(h[:4], precision=6)} oracle {np.array2string(ref.history[:4], precision=6)}")
    assert info.status == eg.CONVERGED and ref.status == 0
    assert _true_rel(oracle_mod, coef, b, xh) <= tol and ref.true_rel_residual <= tol
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 10)
    k = min(4 if precond else 8, len(h), len(ref.history))
    assert np.allclose(h[:k], ref.history[:k], rtol=5e-5 if precond else 2e-5, atol=0)
    assert np.linalg.norm(xh - xo) <= 1e4 * tol * np.linalg.norm(xo)


def test_paper_mixed_precision_restarts_every_150(eg, oracle_mod):
    """Shift 1e-6 needs a few hundred iterations: the mode restarts from the true residual
    every 150 iterations and still converges."""
    import torch
    p = synth.Problem(96, 72, 20, seed=5, shift=1e-6)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    with eg.Operator(dev(coef)) as op:
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-5, 5000, eg.FP32_MP)
    rel = _true_rel(oracle_mod, coef, b, host(x))
    print(f"MP shift 1e-6: {info.iterations} its, {info.restarts} restarts, true R {rel:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-5
    assert info.iterations > 150 and info.restarts >= info.iterations // 150


def test_all_32_bit_solver_matches_the_oracle(eg, oracle_mod, small):
    """Option mp_x32: EG_FP32_MP with the solution held in 32 bits too, the all-32-bit solver of
    the paper's toy-model comparison (Sec. 4, Fig. 1), without periodic restarts.  Against the
    oracle's emulation (oracle/mp.py, x_dtype float32): every entry of x is a float32, the first
    residual-history entries agree to FP32 rounding and the iteration counts within 10 %; run
    to 1e-12 its true residual stalls at the floor a float32 solution implies (the exact
    solution rounded to float32), while the 64-bit-solution mode goes below that floor."""
    import torch
    from oracle import mp
    p, coef, b, x_ref, _ = small
    xo, ref = mp.bicgstab_mp(coef, b, tol=1e-4, restart_every=0, x_dtype=np.float32)
    nb = np.linalg.norm(b)
    floor = np.linalg.norm(b - oracle_mod.apply(coef, x_ref.astype(np.float32).astype(np.float64))) / nb
    with eg.Operator(dev(coef)) as op:
        op.set_option("restart_every", 10 ** 9)
        op.set_option("mp_x32", 1)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-4, 5000, eg.FP32_MP)
        h = op.history()
        xt = torch.zeros_like(x)
        it = op.solve(dev(b), xt, 1e-12, 3000, eg.FP32_MP)
        op.set_option("mp_x32", 0)
        x64 = torch.zeros_like(x)
        i64 = op.solve(dev(b), x64, 1e-12, 3000, eg.FP32_MP)
    xh, xth = host(x), host(xt)
    r_tight = _true_rel(oracle_mod, coef, b, xth)
    r64 = _true_rel(oracle_mod, coef, b, host(x64))
    print(f"all-32-bit: {info.iterations} its (oracle {ref.iterations}); to 1e-12: status {it.status}, true R "
          f"{r_tight:.2e} (float32 floor {floor:.2e}); 64-bit x: status {i64.status}, true R {r64:.2e}")
    assert info.status == eg.CONVERGED and ref.status == 0
    assert np.array_equal(xh, xh.astype(np.float32).astype(np.float64))
    assert np.array_equal(xth, xth.astype(np.float32).astype(np.float64))
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 10)
    k = min(4, len(h), len(ref.history))
    assert np.allclose(h[:k], ref.history[:k], rtol=1e-4, atol=0)
    assert _true_rel(oracle_mod, coef, b, xh) <= 1e-4
    assert 0.3 * floor <= r_tight <= 30 * floor and it.status != eg.CONVERGED
    assert r64 <= 0.1 * floor
