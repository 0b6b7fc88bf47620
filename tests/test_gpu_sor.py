"""The red-black vertical-line SOR preconditioner (the paper's tri_sor, Sec. 2, Eq. 7) on the
GPU against the oracle: the preconditioner itself in every precision, BiCGStab and FGMRES
with it, and option checks."""
import numpy as np
import pytest

import synth
from oracle.quant import quantized_coeffs
from tests.helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eg():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    return eg


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# the last two take the register-resident kernel (70 levels, nlon/2 a multiple of 64; the
# second leaves its last workgroup partly empty), the others the generic one
SHAPES = [synth.Problem(96, 72, 20, seed=0), synth.Problem(40, 30, 24, seed=1), synth.Problem(130, 37, 5, seed=2),
          synth.Problem(64, 16, 70, seed=3), synth.Problem(8, 6, 1, seed=4), synth.Problem(128, 24, 70, seed=5),
          synth.Problem(256, 25, 70, seed=6),
          # 140 levels, nlon / 2 a multiple of 64: the register-resident half-sweeps at 140 levels
          synth.Problem(128, 6, 140, seed=7, ratio=synth._stress_ratio())]


@pytest.mark.parametrize("sweeps,omega", [(1, 1.0), (2, 1.5), (3, 1.5)])
@pytest.mark.parametrize("p", SHAPES, ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_sor_fp64_matches_oracle(eg, oracle_mod, p, sweeps, omega):
    coef = synth.make_coeffs(p)
    q = np.random.default_rng(p.seed + 11).standard_normal(p.n)
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        op.set_option("sor_sweeps", sweeps)
        op.set_option("sor_omega", omega)
        z = host(op.precond(dev(q)))
    ref = oracle_mod.rbsor(coef, q, sweeps=sweeps, omega=omega)
    assert _rel(z, ref) <= 1e-11


@pytest.mark.parametrize("shape", [0, 6, 7])
@pytest.mark.parametrize("prec_name", ["PREC_FP32", "PREC_BF16", "PREC_FP16"])
def test_sor_low_precision(eg, oracle_mod, prec_name, shape):
    """FP32 vectors, the FP32 rounding of the FP64 tridiagonal factors, and that precision's
    horizontal couplings: against the oracle on the same couplings."""
    p = SHAPES[shape]
    coef = synth.make_coeffs(p)
    ref_coef = coef.copy()
    if prec_name != "PREC_FP32":
        ref_coef[:4] = quantized_coeffs(coef, "bf16" if prec_name == "PREC_BF16" else "fp16")[:4]
    q32 = np.random.default_rng(12).standard_normal(p.n).astype(np.float32)
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        z = host(op.precond(dev(q32), prec=getattr(eg, prec_name))).astype(np.float64)
    ref = oracle_mod.rbsor(ref_coef, q32.astype(np.float64))
    err = _rel(z, ref)
    print(f"{prec_name}: max rel diff {err:.2e}")
    assert err <= 2e-5


def test_bicgstab_with_sor_matches_oracle(eg, oracle_mod):
    """Both at tol 1e-12: x agrees to 1e-10 and the iteration counts agree."""
    import torch
    p = SHAPES[0]
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    x_ref, info_ref = oracle_mod.bicgstab(coef, b, tol=1e-12, precond=2)
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-12, 5000, eg.FP64)
        h = op.history()
    xh = host(x)
    err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
    print(f"SOR BiCGStab: GPU {info.iterations} its, oracle {info_ref.iterations}; x rel L2 {err:.2e}")
    assert info.status == eg.CONVERGED and err <= 1e-10
    assert abs(info.iterations - info_ref.iterations) <= 2
    k = min(len(h), len(info_ref.history), 8)
    assert np.allclose(h[:k], info_ref.history[:k], rtol=1e-6)


@pytest.mark.parametrize("mode_name", ["FP32_IR", "FP32_IR_BF16", "FP32_IR_FP16"])
def test_refinement_modes_with_sor_reach_1e8(eg, oracle_mod, mode_name):
    import torch
    p = SHAPES[0]
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-8, 5000, getattr(eg, mode_name))
    rel = np.linalg.norm(b - oracle_mod.apply(coef, host(x))) / np.linalg.norm(b)
    print(f"{mode_name} + SOR: {info.iterations} its, {info.outer_steps} outer, true R {rel:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-8


def test_fgmres_with_sor_matches_oracle(eg, oracle_mod):
    import torch
    from oracle import krylov
    p = SHAPES[0]
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    pc = lambda j, v: oracle_mod.rbsor(coef, v)   # noqa: E731
    x_o, info_o = krylov.fgmres(coef, b, tol=1e-10, m=30, maxit=2000, precond=pc)
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        op.set_option("method", 1)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-10, 2000, eg.FP64)
        h = op.history()
    k = min(len(h), len(info_o.history), 30)
    hdiff = np.max(np.abs(h[:k] - info_o.history[:k]) / info_o.history[:k])
    print(f"FGMRES + SOR: GPU {info.iterations} its, oracle {info_o.iterations}, history rel diff {hdiff:.1e}")
    assert info.status == eg.CONVERGED and abs(info.iterations - info_o.iterations) <= 2 and hdiff <= 1e-6
    assert np.linalg.norm(host(x) - x_o) <= 1e-7 * np.linalg.norm(x_o)


def test_sor_options_are_checked(eg):
    p = synth.Problem(9, 6, 5, seed=1)   # odd nlon
    with eg.Operator(dev(synth.make_coeffs(p))) as op:
        with pytest.raises(eg.EndgameError):
            op.set_option("precond", 1)
        for key, bad in (("sor_sweeps", 0), ("sor_sweeps", 17), ("sor_omega", 2.0), ("sor_omega", 0.0),
                         ("precond", 2)):
            with pytest.raises(eg.EndgameError):
                op.set_option(key, bad)


def test_learned_modes_keep_the_tridiagonal_base(eg):
    """The precond option applies to the plain modes: with a zero-output network the learned
    FP64 mode still reproduces the plain tridiagonal trajectory bit for bit."""
    import torch
    p = SHAPES[0]
    coef = synth.make_coeffs(p)
    b = dev(synth.make_rhs(p).ravel())
    net = eg.Net(3)
    with eg.Operator(dev(coef)) as op:
        op.attach(net)
        op.set_option("learned_method", 0)
        x1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        op.solve(b, x1, 1e-8, 5000, eg.FP64)
        op.set_option("precond", 1)
        x2 = torch.zeros_like(x1)
        i2 = op.solve(b, x2, 1e-8, 5000, eg.LEARNED_FP64)
        x3 = torch.zeros_like(x1)
        i3 = op.solve(b, x3, 1e-8, 5000, eg.FP64)
    assert torch.equal(x1, x2) and i3.iterations < i2.iterations
    net.close()
