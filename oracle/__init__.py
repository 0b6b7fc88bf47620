"""Plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg import this package.
The GPU library never imports it and shares no code with it.

* ``apply``, ``apply_points``, ``thomas``, ``rbsor``, ``lexsor``, ``bicgstab`` wrap ``oracle.c`` (see its
  header for the passages of the paper each follows).
* ``dense_matrix`` / ``dense_solve`` assemble A as a dense matrix and solve it with LAPACK's
  partial-pivot LU (the exact solution the Krylov iteration approaches; tiny grids only).
* ``net`` holds the FP64 reference of the learned preconditioner's network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None
_lib_omp = None
EPS_BD = 2.0 ** -52   # default breakdown threshold of BiCGStab (relative cosine)


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, no FMA contraction, one thread) and
    into ``liboracle_omp.so`` (the same source with OpenMP: grid loops shared among threads,
    inner products over a fixed partition, see the source's header)."""
    for path, extra in ((LIB_PATH, []), (LIB_OMP_PATH, ["-fopenmp", "-DORC_OPENMP"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                                   "-Wall", *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return LIB_PATH


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("status", ctypes.c_int),
                ("half_step_exit", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("sigma_restarts", ctypes.c_int),
                ("rho_restarts", ctypes.c_int)]


@dataclass
class SolveInfo:
    iterations: int
    restarts: int
    status: int
    half_step_exit: int
    rel_residual: float
    true_rel_residual: float
    history: np.ndarray
    sigma_restarts: int = 0
    rho_restarts: int = 0


def _load(parallel: bool = False):
    """The single-threaded oracle library, or (``parallel``) its OpenMP build."""
    global _lib, _lib_omp
    if (_lib_omp if parallel else _lib) is None:
        path = LIB_OMP_PATH if parallel else LIB_PATH
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_apply.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp]
        lib.orc_apply_points.argtypes = [ctypes.c_int] * 3 + [dp, dp, ctypes.POINTER(ctypes.c_long), ctypes.c_long, dp]
        lib.orc_thomas.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp]
        lib.orc_dot.argtypes = [ctypes.c_long, dp, dp]
        lib.orc_dot.restype = ctypes.c_double
        lib.orc_bicgstab.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                          ctypes.c_int, dp, ctypes.c_int, ctypes.POINTER(_Info)]
        lib.orc_bicgstab.restype = ctypes.c_int
        lib.orc_rbsor.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.orc_lexsor.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.orc_bicgstab_sor.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                             ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                                             ctypes.c_int, ctypes.POINTER(_Info)]
        lib.orc_bicgstab_sor.restype = ctypes.c_int
        lib.orc_set_eps_bd.argtypes = [ctypes.c_double]
        if parallel:
            _lib_omp = lib
        else:
            _lib = lib
    return _lib_omp if parallel else _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(coef: np.ndarray):
    assert coef.dtype == np.float64 and coef.flags.c_contiguous and coef.ndim == 4 and coef.shape[0] == 7
    return coef.shape[3], coef.shape[2], coef.shape[1]


def _vec(v: np.ndarray, n: int) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == n
    return v


def apply(coef: np.ndarray, x: np.ndarray, parallel: bool = False) -> np.ndarray:
    """y = A x (plain row definition); ``parallel``: the OpenMP build (bitwise the same)."""
    nlon, nlat, nlev = _check(coef)
    x = _vec(x, nlon * nlat * nlev)
    y = np.empty_like(x)
    _load(parallel).orc_apply(nlon, nlat, nlev, _dp(coef), _dp(x), _dp(y))
    return y


def apply_points(coef: np.ndarray, x: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """(A x)[idx] computed one row at a time."""
    nlon, nlat, nlev = _check(coef)
    x = _vec(x, nlon * nlat * nlev)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    y = np.empty(idx.size)
    _load().orc_apply_points(nlon, nlat, nlev, _dp(coef), _dp(x),
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), idx.size, _dp(y))
    return y


def thomas(coef: np.ndarray, q: np.ndarray, parallel: bool = False) -> np.ndarray:
    """z = T^{-1} q, T = tridiag(-aD, C, -aU) per column; ``parallel``: the OpenMP build
    (bitwise the same)."""
    nlon, nlat, nlev = _check(coef)
    q = _vec(q, nlon * nlat * nlev)
    z = np.empty_like(q)
    _load(parallel).orc_thomas(nlon, nlat, nlev, _dp(coef), _dp(q), _dp(z))
    return z


def dot(a: np.ndarray, b: np.ndarray, parallel: bool = False) -> float:
    """<a, b>, summed left to right (``parallel``: over the fixed partition of the OpenMP build)."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    return _load(parallel).orc_dot(a.size, _dp(a), _dp(b))


def rbsor(coef: np.ndarray, q: np.ndarray, sweeps: int = 3, omega: float = 1.5, half_sweeps: int | None = None):
    """Red-black vertical-line SOR applied to q from x0 = 0 (the tri_sor preconditioner of
    Sec. 2, Eq. 7, with red-black column order); ``half_sweeps`` overrides 2 * sweeps."""
    nlon, nlat, nlev = _check(coef)
    q = _vec(q, nlon * nlat * nlev)
    z = np.empty_like(q)
    nh = 2 * sweeps if half_sweeps is None else half_sweeps
    _load().orc_rbsor(nlon, nlat, nlev, _dp(coef), _dp(q), _dp(z), int(nh), float(omega))
    return z


def lexsor(coef: np.ndarray, q: np.ndarray, sweeps: int = 3, omega: float = 1.5):
    """The same line SOR in the natural (lexicographic) column order of Eq. 7's L and U."""
    nlon, nlat, nlev = _check(coef)
    q = _vec(q, nlon * nlat * nlev)
    z = np.empty_like(q)
    _load().orc_lexsor(nlon, nlat, nlev, _dp(coef), _dp(q), _dp(z), int(sweeps), float(omega))
    return z


def bicgstab(coef: np.ndarray, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8,
             maxit: int = 20000, restart_every: int = 0, precond: int = 1,
             hist_cap: int | None = None, sor_sweeps: int = 3, sor_omega: float = 1.5,
             eps_bd: float = EPS_BD, parallel: bool = False) -> tuple[np.ndarray, SolveInfo]:
    """Right-preconditioned BiCGStab; precond 1 = vertical tridiagonal, 0 = identity,
    2 = red-black line SOR, 3 = lexicographic line SOR, with ``sor_sweeps`` sweeps and
    relaxation ``sor_omega``; ``eps_bd`` is the breakdown threshold (relative cosine).
    ``parallel`` runs the OpenMP build (all host threads; fixed-partition inner products)."""
    lib = _load(parallel)
    nlon, nlat, nlev = _check(coef)
    n = nlon * nlat * nlev
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    cap = maxit if hist_cap is None else hist_cap
    hist = np.full(max(cap, 1), np.nan)
    info = _Info()
    lib.orc_set_eps_bd(float(eps_bd))
    if precond in (2, 3):
        lib.orc_bicgstab_sor(nlon, nlat, nlev, _dp(coef), _dp(b), _dp(x), tol, maxit, restart_every, precond,
                             int(sor_sweeps), float(sor_omega), _dp(hist), cap, ctypes.byref(info))
    else:
        lib.orc_bicgstab(nlon, nlat, nlev, _dp(coef), _dp(b), _dp(x), tol, maxit, restart_every, precond,
                         _dp(hist), cap, ctypes.byref(info))
    lib.orc_set_eps_bd(EPS_BD)
    h = hist[:min(info.iterations, cap)].copy()
    return x, SolveInfo(info.iterations, info.restarts, info.status, info.half_step_exit, info.rel_residual,
                        info.true_rel_residual, h, info.sigma_restarts, info.rho_restarts)


def dense_matrix(coef: np.ndarray) -> np.ndarray:
    """Dense A assembled entry by entry from the coefficient arrays (tiny grids only).

    Row c has C[c] on the diagonal and -a_d[c] in the column of neighbour d; couplings whose
    neighbour lies across a pole, the bottom or the top are left out (they must be zero).
    """
    nlon, nlat, nlev = _check(coef)
    n = nlon * nlat * nlev
    assert n <= 4000, "dense assembly is for tiny grids"
    A = np.zeros((n, n))
    for k in range(nlev):
        for j in range(nlat):
            for i in range(nlon):
                c = i + nlon * (j + nlat * k)
                A[c, c] += coef[6, k, j, i]
                nbrs = [(0, (i - 1) % nlon, j, k), (1, (i + 1) % nlon, j, k), (2, i, j - 1, k), (3, i, j + 1, k),
                        (4, i, j, k - 1), (5, i, j, k + 1)]
                for d, ii, jj, kk in nbrs:
                    if 0 <= jj < nlat and 0 <= kk < nlev:
                        A[c, ii + nlon * (jj + nlat * kk)] -= coef[d, k, j, i]
    return A


def dense_solve(coef: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact solution of A x = b by LAPACK partial-pivot LU (numpy.linalg.solve)."""
    return np.linalg.solve(dense_matrix(coef), np.asarray(b, dtype=np.float64).ravel())
