"""Planted mistakes in the oracle, on the CPU: the pins have teeth.

Each mutant is a copy of ``oracle/oracle.c`` with one plausible mistake (a dropped coupling, a
wrong sign, swapped neighbours, a coefficient of the wrong direction, a wrong step of the
tridiagonal recurrences, of BiCGStab's coefficients or of the red-black line SOR, an inner
product that skips an element), compiled into a library of its own in a temporary folder.
The oracle's own pins (closed-form eigenpairs, the dense assembly, LAPACK's banded solver,
dense LU, the independent flexible BiCGStab, the dense block-SOR splitting, exact integer sums)
are then run against it: every mutant must fail at least one of them, and the unmutated copy
built the same way must pass all of them.  Nothing here touches the GPU library.
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
