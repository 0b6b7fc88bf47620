"""Planted mistakes in the oracle, on the CPU: the pins have teeth.

Each mutant is a copy of ``oracle/oracle.c`` with one plausible mistake (a dropped coupling, a
wrong sign, swapped neighbours, a coefficient of the wrong direction, a wrong step of the
tridiagonal recurrences, of BiCGStab's coefficients or of the red-black line SOR, an inner
product that skips an element), compiled into a library of its own in a temporary folder.
The oracle's own pins (closed-form eigenpairs, the dense assembly, LAPACK's banded solver,
dense LU, the independent flexible BiCGStab, the dense block-SOR splitting, exact integer sums)
are then run against it: every mutant must fail at least one of them, and the unmutated copy
built the same way must pass all of them.  The Python parts of the oracle (the network and its
Adam step, the 16-bit coefficient operator, FGMRES, the mixed-precision emulation) get the same
treatment with source-level mutants run through all of their pin modules' tests.  Nothing here
touches the GPU library.
"""
from __future__ import annotations

import contextlib
import os
import subprocess

import pytest

import oracle
import synth
from tests import test_oracle as pins_main
from tests import test_oracle_krylov as pins_krylov
from tests import test_oracle_sor as pins_sor

_REAL_SRC = oracle._SRC

MUTANTS = [
    ("apply: north coupling dropped",
     [("                if (j < nlat - 1) acc = acc - aN[c] * x[c + nlon];\n", "")]),
    ("apply: west coupling with the wrong sign",
     [("acc = acc - aW[c] * x[iw + (long)nlon * (j + (long)nlat * k)];",
       "acc = acc + aW[c] * x[iw + (long)nlon * (j + (long)nlat * k)];")]),
    ("apply: west and east neighbours swapped",
     [("aW[c] * x[iw + (long)nlon", "aW[c] * x[ie + (long)nlon"),
      ("aE[c] * x[ie + (long)nlon", "aE[c] * x[iw + (long)nlon")]),
    ("apply: the upper coupling used for the level below",
     [("if (k > 0) acc = acc - aD[c] * x[c - P];", "if (k > 0) acc = acc - aU[c] * x[c - P];")]),
    ("thomas: forward elimination with the wrong sign",
     [("yy[k] = (q[c] - (-aD[c]) * yy[k - 1]) / den;", "yy[k] = (q[c] + (-aD[c]) * yy[k - 1]) / den;")]),
    ("thomas: back substitution with the wrong sign",
     [("z[col + k * P] = yy[k] - cp[k] * z[col + (k + 1) * P];",
       "z[col + k * P] = yy[k] + cp[k] * z[col + (k + 1) * P];")]),
    ("bicgstab: beta with alpha / omega inverted",
     [("double beta = (rho / rho_prev) * (alpha / omega);", "double beta = (rho / rho_prev) * (omega / alpha);")]),
    ("bicgstab: s = r + alpha v",
     [("s[i] = r[i] - alpha * v[i];", "s[i] = r[i] + alpha * v[i];")]),
    ("bicgstab: the omega term dropped from the update of x",
     [("x[i] = x[i] + alpha * ph[i] + omega * sh[i];", "x[i] = x[i] + alpha * ph[i];")]),
    ("dot: the last element skipped",
     [("for (long i = 0; i < n; ++i) s = s + a[i] * b[i];", "for (long i = 0; i < n - 1; ++i) s = s + a[i] * b[i];")]),
    ("red-black SOR: relaxation without omega",
     [("z[c] = (1.0 - omega) * old[c] + omega * col[k];", "z[c] = (1.0 - omega) * old[c] + col[k];")]),
    ("red-black SOR: north coupling dropped",
     [("                    if (j < nlat - 1) acc = acc + aN[c] * old[c + nlon];\n", "")]),
]


def _pins():
    p1 = synth.Problem(8, 6, 5, seed=1)
    return [
        ("apply eigenpairs", lambda: pins_main.test_apply_closed_form_eigenpairs(
            oracle, (6, 5, 4), [(0, 0, 0), (1, 2, 3), (3, 4, 1), (5, 1, 2)])),
        ("apply complex eigenpair", lambda: pins_main.test_apply_lon_asymmetric_complex_eigenpair(oracle)),
        ("apply dense assembly", lambda: pins_main.test_apply_matches_dense_assembly_and_points(oracle)),
        ("thomas vertical mode", lambda: pins_main.test_thomas_closed_form_vertical_mode(oracle)),
        ("thomas LAPACK banded", lambda: pins_main.test_thomas_matches_lapack_banded(oracle)),
        ("bicgstab dense LU", lambda: pins_main.test_bicgstab_matches_dense_lu(oracle, p1, 1e-13)),
        ("dot exact", lambda: pins_main.test_dot_exact_on_integers(oracle)),
        ("flexible BiCGStab = C BiCGStab", lambda: pins_krylov.test_flexible_bicgstab_with_fixed_m_is_the_c_oracle(
            1, 2.0 ** -52)),
        ("SOR dense block splitting", pins_sor.test_matches_block_sor_on_the_dense_matrix),
        ("SOR colour equations", lambda: pins_sor.test_updated_colour_satisfies_its_equations(2)),
    ]


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


def _build(workdir, tag: str, subs) -> tuple[str, str]:
    with open(_REAL_SRC) as f:
        text = f.read()
    for old, new in subs:
        assert text.count(old) == 1, (tag, old)
        text = text.replace(old, new)
    src = os.path.join(workdir, f"{tag}.c")
    lib = os.path.join(workdir, f"lib{tag}.so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", lib, src,
                           "-lm"])
    return lib, src


@contextlib.contextmanager
def _use_library(workdir, lib: str, src: str):
    """Point the oracle package at another build (and any rebuild at the temporary folder)."""
    saved = (oracle.LIB_PATH, oracle.LIB_OMP_PATH, oracle._SRC, oracle._lib)
    oracle.LIB_PATH, oracle.LIB_OMP_PATH, oracle._SRC, oracle._lib = lib, os.path.join(workdir, "omp.so"), src, None
    try:
        yield
    finally:
        oracle.LIB_PATH, oracle.LIB_OMP_PATH, oracle._SRC, oracle._lib = saved


def _failing(workdir, lib, src):
    failed = []
    with _use_library(workdir, lib, src):
        for name, pin in _pins():
            try:
                pin()
            except Exception:    # an assertion of the pin, or a failure the mistake provoked
                failed.append(name)
    return failed


def test_unmutated_copy_passes_every_pin(workdir):
    lib, src = _build(workdir, "unmutated", [])
    assert _failing(workdir, lib, src) == []


@pytest.mark.parametrize("tag", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(workdir, tag):
    name, subs = MUTANTS[tag]
    lib, src = _build(workdir, f"mutant{tag}", subs)
    failed = _failing(workdir, lib, src)
    print(f"{name}: caught by {failed}")
    assert failed, name


# ---- the Python parts of the oracle ---------------------------------------------------------
# Each mutant is the module's source with one substitution, executed as a fresh module and put
# in place of the original in the pin module's namespace; all of that pin module's tests run
# against it (every parametrisation), and at least one must fail.
import importlib            # noqa: E402
import itertools            # noqa: E402
import types                # noqa: E402

PY_MUTANTS = [
    # (oracle module, pin module, attribute the pin module binds it to, label, substitutions)
    ("oracle.net", "tests.test_oracle_net", "net", "network: ReLU of layer 2 dropped",
     [("a2 = rnd(np.maximum(z2, 0.0))", "a2 = rnd(z2)")]),
    ("oracle.net", "tests.test_oracle_net", "net", "network: layer-3 adjoint shifted the wrong way",
     [("g_a2 = sum(_shift_v(g_z3 @ W3[t], -_vtap(t)) for t in range(TAPS_V))",
       "g_a2 = sum(_shift_v(g_z3 @ W3[t], _vtap(t)) for t in range(TAPS_V))")]),
    ("oracle.net", "tests.test_oracle_net", "net", "network: T^-T built as T^-1",
     [("    ct[4, 1:] = coef[5, :-1]\n    ct[5, :-1] = coef[4, 1:]\n    return oracle.thomas(ct, y)",
       "    ct[4] = coef[4]\n    ct[5] = coef[5]\n    return oracle.thomas(ct, y)")]),
    ("oracle.net", "tests.test_oracle_net", "net", "network: A^T with the west coupling rolled the wrong way",
     [("ct[0] = np.roll(coef[1], 1, axis=2)", "ct[0] = np.roll(coef[1], -1, axis=2)")]),
    ("oracle.net", "tests.test_oracle_net", "net", "network: BF16 rounding truncates",
     [("out[nz] = np.sign(x[nz]) * np.rint(ax / ulp) * ulp", "out[nz] = np.sign(x[nz]) * np.floor(ax / ulp) * ulp")]),
    ("oracle.net", "tests.test_oracle_net", "net", "Adam: second-moment bias correction dropped",
     [("v_hat = state.v / (1.0 - beta2 ** state.t)", "v_hat = state.v")]),
    ("oracle.net", "tests.test_oracle_net", "net", "Adam: first moment decays with beta2",
     [("state.m = beta1 * state.m + (1.0 - beta1) * g", "state.m = beta2 * state.m + (1.0 - beta2) * g")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: no gradual underflow",
     [("lead = np.maximum(e - 1, emin)", "lead = e - 1")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: margin without the upper coupling",
     [("return coef[6] - ((hs + coef[4]) + coef[5])", "return coef[6] - (hs + coef[4])")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: the row's minimum as offset",
     [("mid = (0.5 * (lo + hi)).astype(np.float32).astype(np.float64)", "mid = lo")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: offsets also on rows holding a zero",
     [("return np.where((lo > 0) & (hi <= 2.0 * lo), mid, 0.0)", "return np.where(hi > 0, mid, 0.0)")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: offsets also on widely spread rows",
     [("return np.where((lo > 0) & (hi <= 2.0 * lo), mid, 0.0)", "return np.where(lo > 0, mid, 0.0)")]),
    ("oracle.quant", "tests.test_oracle_quant", "quant", "16-bit: rounding truncates",
     [("out[nz] = np.rint(u[nz] / ulp) * ulp", "out[nz] = np.floor(u[nz] / ulp) * ulp")]),
    ("oracle.krylov", "tests.test_oracle_krylov", "krylov", "FGMRES: Givens rotation with the wrong sign",
     [("H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c",
       "H[i, j], H[i + 1, j] = cs[i] * a - sn[i] * c, sn[i] * a + cs[i] * c")]),
    ("oracle.krylov", "tests.test_oracle_krylov", "krylov", "FGMRES: one Gram-Schmidt projection skipped",
     [("w = w - H[i, j] * V[i]", "w = w - (H[i, j] * V[i] if i > 0 else 0.0)")]),
    ("oracle.mp", "tests.test_oracle_mp", "mp", "mixed precision: v = A p^ left in 64 bits",
     [("v = op_lo(ph)", "v = oracle.apply(coef_lo, hi(ph))")]),
    ("oracle.mp", "tests.test_oracle_mp", "mp", "mixed precision: s left in 64 bits",
     [("s = lo(hi(r) - alpha * hi(v))", "s = hi(r) - alpha * hi(v)")]),
]


def _mutant_module(modname: str, subs):
    real = importlib.import_module(modname)
    with open(real.__file__) as f:
        text = f.read()
    for old, new in subs:
        assert text.count(old) == 1, (modname, old)
        text = text.replace(old, new)
    mod = types.ModuleType(modname)
    mod.__file__ = real.__file__
    exec(compile(text, real.__file__ + " (mutant)", "exec"), mod.__dict__)
    return mod


def _cases(fn):
    """Every parametrisation of a test function: a list of keyword dicts."""
    marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
    groups = []
    for m in marks:
        names = [s.strip() for s in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
        vals = [v if len(names) > 1 else (v,) for v in m.args[1]]
        groups.append([dict(zip(names, v)) for v in vals])
    out = []
    for combo in itertools.product(*groups):
        kw = {}
        for d in combo:
            kw.update(d)
        out.append(kw)
    return out or [{}]


def _failing_tests(pin_module) -> tuple[list[str], int]:
    failed, total = [], 0
    for name in sorted(dir(pin_module)):
        fn = getattr(pin_module, name)
        if not name.startswith("test_") or not callable(fn):
            continue
        for kw in _cases(fn):
            total += 1
            try:
                fn(**kw)
            except Exception:
                failed.append(f"{name}{kw or ''}")
    return failed, total


@pytest.mark.parametrize("tag", sorted({m[1] for m in PY_MUTANTS}))
def test_python_pins_pass_on_the_real_modules(tag):
    failed, total = _failing_tests(importlib.import_module(tag))
    assert total > 0 and failed == []


@pytest.mark.filterwarnings("ignore::RuntimeWarning")   # a mutant may produce NaN on purpose
@pytest.mark.parametrize("idx", range(len(PY_MUTANTS)), ids=[m[3] for m in PY_MUTANTS])
def test_python_planted_mistake_fails_a_pin(idx):
    modname, pinname, attr, label, subs = PY_MUTANTS[idx]
    pins = importlib.import_module(pinname)
    mutant = _mutant_module(modname, subs)
    saved = getattr(pins, attr)
    setattr(pins, attr, mutant)
    try:
        failed, total = _failing_tests(pins)
    finally:
        setattr(pins, attr, saved)
    print(f"{label}: {len(failed)} of {total} pins fail: {failed[:4]}")
    assert failed, label
