"""Seeded synthetic problem instances for the Helmholtz pressure-correction solve.

This module only *builds inputs*: the seven coefficient arrays of the 7-point operator,
right-hand sides and manufactured solutions.  It holds none of the solver's arithmetic
(no matrix-vector product, no preconditioner, no Krylov step), so both the CPU oracle and
the GPU library can consume its output without sharing code with each other.

The operator family stands in for the ENDGame Helmholtz matrix of Section 2 of the paper
(Eq. 4 and the description after it): a 7-band, non-symmetric, variable-coefficient matrix
on a lon-lat-height grid whose vertical length scales are much shorter than the horizontal
ones.  The UM's own matrices are not available, so the recipe below defines one:

* Grid: ``nlon`` x ``nlat`` cell centres, ``dlam = 2 pi / nlon``, ``dphi = pi / nlat``,
  ``phi_j = -pi/2 + (j + 1/2) dphi``; lon is periodic, the two pole faces have
  ``cos phi = 0`` exactly (zero flux), the top and bottom are zero flux.
* Levels: ``dz_k = dz_0 r^k`` with ``sum dz_k = 80 km``; ``d_{k+1/2} = (dz_k + dz_{k+1})/2``.
* Finite-volume couplings (face area over centre distance, earth radius 6.371e6 m):
  ``aE = aW = dphi dz_k / (cos phi_j dlam)``, ``aN = cos phi_{j+1/2} dlam dz_k / dphi``,
  ``aS = cos phi_{j-1/2} dlam dz_k / dphi``, ``aU = K R^2 cos phi_j dlam dphi / d_{k+1/2}``
  (0 on the top level), ``aD`` likewise with ``d_{k-1/2}`` (0 on the bottom level).
* Row scaling: each row's six couplings are divided by their sum.  This plays the role of
  the diagonal scaling that the paper applies outside the solver (Eq. 5).
* Non-symmetry: each of the six scaled couplings is multiplied by ``1 + 0.1 u``,
  ``u ~ U[-1, 1]`` drawn independently per (direction, point).
* Diagonal: ``C = sum of the six couplings + shift``.  Off-diagonal *entries* of A are the
  negated couplings, so A is a row-diagonally-dominant M-matrix with margin ``shift``.
* Stress variant: ``K`` takes one of 8 values per contiguous band of levels, drawn
  log-uniform in [1e-2, 1e2] with the extreme draws pinned to 1e-2 and 1e2.

Array layout everywhere: ``coeffs[d, k, j, i]`` with direction order W, E, S, N, D, U, C and
lon fastest (``idx = i + nlon (j + nlat k)``).

Random streams: every draw comes from its own ``numpy`` PCG64 stream keyed by
``SeedSequence(seed, spawn_key=(stream, level))``, so any level can be produced on its own
(large grids are generated level by level and never held whole on the host).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

EARTH_RADIUS = 6.371e6
Z_TOP = 80_000.0
DIRS = ("W", "E", "S", "N", "D", "U", "C")

# stream identifiers for SeedSequence spawn keys
_S_PERTURB = 0
_S_RHS = 1
_S_XSTAR_NOISE = 2
_S_BANDS = 3
_S_XSTAR_MODES = 4


@dataclass(frozen=True)
class Problem:
    """Shape and recipe parameters of one synthetic operator."""

    nlon: int
    nlat: int
    nlev: int
    shift: float = 1e-3
    ratio: float = 1.1          # dz_{k+1} / dz_k
    perturb: float = 0.1        # relative size of the non-symmetric perturbation
    bands: bool = False         # banded vertical diffusivity (stress variant)
    seed: int = 0
    name: str = field(default="", compare=False)

    @property
    def n(self) -> int:
        return self.nlon * self.nlat * self.nlev

    @property
    def shape(self) -> tuple[int, int, int]:
        return (self.nlev, self.nlat, self.nlon)


def _stress_ratio() -> float:
    # 140 levels with the same top/bottom thickness ratio as 70 levels at r = 1.1
    return 1.1 ** (69.0 / 139.0)


CONFIGS: dict[str, Problem] = {
    # small correctness case (96 x 72 x 20, n = 138,240)
    "small_96x72x20": Problem(96, 72, 20, name="small_96x72x20"),
    # 640 x 480 x 70 (21.5M dof); right-hand side from a smooth manufactured solution
    "manufactured_640x480x70": Problem(640, 480, 70, name="manufactured_640x480x70"),
    # N1280-shaped grid 2560 x 1920 x 70 (344M dof)
    "n1280_2560x1920x70": Problem(2560, 1920, 70, name="n1280_2560x1920x70"),
    # learned-preconditioner case, same operator as the manufactured case
    "learned_640x480x70": Problem(640, 480, 70, name="learned_640x480x70"),
    # stress case 1280 x 960 x 140, near-singular shift, 1e4 diffusivity contrast
    "stress_1280x960x140": Problem(1280, 960, 140, shift=1e-6, ratio=_stress_ratio(), bands=True, name="stress_1280x960x140"),
}


def _rng(seed: int, stream: int, level: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(stream, level))))


def level_thickness(nlev: int, ratio: float) -> np.ndarray:
    """dz_k = dz_0 ratio^k, k = 0..nlev-1, summing to 80 km."""
    k = np.arange(nlev, dtype=np.float64)
    if ratio == 1.0:
        return np.full(nlev, Z_TOP / nlev)
    dz0 = Z_TOP * (ratio - 1.0) / (ratio ** nlev - 1.0)
    return dz0 * ratio ** k


def band_diffusivity(p: Problem) -> np.ndarray:
    """Per-level vertical diffusivity K_k (ones unless ``p.bands``).

    8 contiguous bands split at 7 distinct interior cut points; K_b = 10^U[-2, 2] with the
    smallest and largest draws pinned to 1e-2 and 1e2 (contrast exactly 1e4).
    """
    if not p.bands:
        return np.ones(p.nlev)
    nb = min(8, p.nlev)
    rng = _rng(p.seed, _S_BANDS)
    cuts = np.sort(rng.choice(np.arange(1, p.nlev), size=nb - 1, replace=False)) if nb > 1 else np.array([], int)
    kb = 10.0 ** rng.uniform(-2.0, 2.0, size=nb)
    if nb > 1:
        kb[np.argmin(kb)] = 1e-2
        kb[np.argmax(kb)] = 1e2
    band_of_level = np.searchsorted(cuts, np.arange(p.nlev), side="right")
    return kb[band_of_level]


def _grid(p: Problem):
    dlam = 2.0 * math.pi / p.nlon
    dphi = math.pi / p.nlat
    j = np.arange(p.nlat, dtype=np.float64)
    phi_c = -0.5 * math.pi + (j + 0.5) * dphi
    cos_c = np.cos(phi_c)
    jf = np.arange(p.nlat + 1, dtype=np.float64)
    cos_f = np.cos(-0.5 * math.pi + jf * dphi)
    cos_f[0] = 0.0
    cos_f[-1] = 0.0
    cos_f = np.maximum(cos_f, 0.0)
    dz = level_thickness(p.nlev, p.ratio)
    dmid = 0.5 * (dz[:-1] + dz[1:])          # d_{k+1/2}, k = 0..nlev-2
    return dlam, dphi, cos_c, cos_f, dz, dmid


def raw_couplings_level(p: Problem, k: int, grid=None, kdiff=None) -> np.ndarray:
    """Unscaled, unperturbed finite-volume couplings of level k: shape (6, nlat, nlon).

    This is the symmetric operator before row scaling: aE(i) = aW(i+1), aN(j) = aS(j+1),
    aU(k) = aD(k+1).
    """
    if grid is None:
        grid = _grid(p)
    if kdiff is None:
        kdiff = band_diffusivity(p)
    dlam, dphi, cos_c, cos_f, dz, dmid = grid
    nlat, nlon = p.nlat, p.nlon
    out = np.empty((6, nlat, nlon))
    ew = dphi * dz[k] / (cos_c * dlam)
    out[0] = ew[:, None]
    out[1] = ew[:, None]
    out[2] = (cos_f[:-1] * dlam * dz[k] / dphi)[:, None]
    out[3] = (cos_f[1:] * dlam * dz[k] / dphi)[:, None]
    vert = EARTH_RADIUS ** 2 * cos_c * dlam * dphi
    out[4] = (kdiff[k - 1] * vert / dmid[k - 1])[:, None] if k > 0 else 0.0
    out[5] = (kdiff[k] * vert / dmid[k])[:, None] if k < p.nlev - 1 else 0.0
    return out


def coeff_level(p: Problem, k: int, grid=None, kdiff=None) -> np.ndarray:
    """The seven coefficient planes of level k, shape (7, nlat, nlon), float64."""
    raw = raw_couplings_level(p, k, grid, kdiff)
    a = raw / raw.sum(axis=0, keepdims=True)
    if p.perturb:
        u = _rng(p.seed, _S_PERTURB, k).random((6, p.nlat, p.nlon))
        a *= 1.0 + p.perturb * (2.0 * u - 1.0)
    # zero-flux boundaries stay exactly zero (cos = 0 faces, top/bottom)
    out = np.empty((7, p.nlat, p.nlon))
    out[:6] = a
    out[6] = a.sum(axis=0) + p.shift
    return out


def iter_coeff_levels(p: Problem, threads: int = 8):
    """Yield ``(k, level_array)`` for k = 0..nlev-1 (level arrays built in a thread pool)."""
    grid = _grid(p)
    kdiff = band_diffusivity(p)
    if threads <= 1 or p.nlev == 1:
        for k in range(p.nlev):
            yield k, coeff_level(p, k, grid, kdiff)
        return
    with ThreadPoolExecutor(max_workers=threads) as ex:
        window = []
        for k in range(p.nlev):
            window.append(ex.submit(coeff_level, p, k, grid, kdiff))
            if len(window) >= 2 * threads:
                kk = k - len(window) + 1
                yield kk, window.pop(0).result()
        base = p.nlev - len(window)
        for off, f in enumerate(window):
            yield base + off, f.result()


def make_coeffs(p: Problem, threads: int = 8) -> np.ndarray:
    """All coefficients, shape (7, nlev, nlat, nlon), float64 (small and medium grids)."""
    out = np.empty((7, p.nlev, p.nlat, p.nlon))
    for k, lev in iter_coeff_levels(p, threads):
        out[:, k] = lev
    return out


def make_raw_coeffs(p: Problem) -> np.ndarray:
    """Symmetric unscaled couplings with C = sum + shift (used to test symmetry pins)."""
    grid = _grid(p)
    kdiff = band_diffusivity(p)
    out = np.empty((7, p.nlev, p.nlat, p.nlon))
    for k in range(p.nlev):
        raw = raw_couplings_level(p, k, grid, kdiff)
        out[:6, k] = raw
        out[6, k] = raw.sum(axis=0) + p.shift
    return out


def rhs_level(p: Problem, k: int, seed: int | None = None) -> np.ndarray:
    """b ~ N(0, 1) on level k, shape (nlat, nlon)."""
    return _rng(p.seed if seed is None else seed, _S_RHS, k).standard_normal((p.nlat, p.nlon))


def make_rhs(p: Problem, seed: int | None = None) -> np.ndarray:
    """b ~ N(0, 1), shape (nlev, nlat, nlon)."""
    out = np.empty(p.shape)
    for k in range(p.nlev):
        out[k] = rhs_level(p, k, seed)
    return out


def make_xstar(p: Problem, nmodes: int = 8, noise: float = 1e-3, seed: int | None = None) -> np.ndarray:
    """Smooth manufactured solution: a sum of ``nmodes`` spherical-harmonic-like modes plus
    N(0, noise) white noise (noise is a standard deviation).

    Mode q: integers m_q, l_q in {0..6}, v_q in {0..3}, amplitude A_q ~ N(0, 1), phase
    psi_q ~ U[0, 2 pi);  A_q cos^m(phi) cos(m lam + psi) cos(l (phi + pi/2))
    cos(pi v (k + 1/2) / nlev) with lam_i = (i + 1/2) dlam.  The cos^m(phi) factor keeps
    each mode regular at the poles.
    """
    s = p.seed if seed is None else seed
    rng = _rng(s, _S_XSTAR_MODES)
    m = rng.integers(0, 7, nmodes)
    l = rng.integers(0, 7, nmodes)
    v = rng.integers(0, 4, nmodes)
    amp = rng.standard_normal(nmodes)
    psi = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    dlam = 2.0 * math.pi / p.nlon
    dphi = math.pi / p.nlat
    lam = (np.arange(p.nlon) + 0.5) * dlam
    phi = -0.5 * math.pi + (np.arange(p.nlat) + 0.5) * dphi
    kk = np.arange(p.nlev) + 0.5
    out = np.zeros(p.shape)
    for q in range(nmodes):
        hor = (np.cos(phi) ** m[q] * np.cos(l[q] * (phi + 0.5 * math.pi)))[:, None] * np.cos(m[q] * lam + psi[q])[None, :]
        ver = np.cos(math.pi * v[q] * kk / p.nlev)
        out += amp[q] * ver[:, None, None] * hor[None, :, :]
    if noise:
        for k in range(p.nlev):
            out[k] += noise * _rng(s, _S_XSTAR_NOISE, k).standard_normal((p.nlat, p.nlon))
    return out


def constant_operator(nlon: int, nlat: int, nlev: int, ax: float, ay: float, az: float, shift: float,
                      ax_e: float | None = None) -> np.ndarray:
    """Constant-coefficient test operator with zero-flux lat/vertical boundaries.

    ``ax`` is the W coupling and ``ax_e`` (default ``ax``) the E coupling, so a lon-asymmetric
    operator can be built; S/N use ``ay`` and D/U use ``az`` except on boundary faces.
    """
    ax_e = ax if ax_e is None else ax_e
    c = np.zeros((7, nlev, nlat, nlon))
    c[0] = ax
    c[1] = ax_e
    c[2] = ay
    c[3] = ay
    c[2, :, 0, :] = 0.0
    c[3, :, nlat - 1, :] = 0.0
    c[4] = az
    c[5] = az
    c[4, 0] = 0.0
    c[5, nlev - 1] = 0.0
    c[6] = c[:6].sum(axis=0) + shift
    return c
