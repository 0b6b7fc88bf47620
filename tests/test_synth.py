"""Checks on the seeded input generator (shapes, boundaries, margins, recipe invariants)."""
import math

import numpy as np

import synth


def test_shapes_boundaries_margin():
    for p in (synth.CONFIGS["small_96x72x20"], synth.Problem(33, 17, 9, shift=1e-6, ratio=synth._stress_ratio(), bands=True)):
        c = synth.make_coeffs(p)
        assert c.shape == (7, p.nlev, p.nlat, p.nlon) and c.dtype == np.float64
        assert np.all(c[:6] >= 0)
        assert not np.any(c[2, :, 0, :]) and not np.any(c[3, :, -1, :])
        assert not np.any(c[4, 0]) and not np.any(c[5, -1])
        m = c[6] - c[:6].sum(axis=0)
        assert np.allclose(m, p.shift, rtol=0, atol=8 * np.finfo(float).eps * c[6].max())
        # scaled couplings sum to one before the +-10% perturbation
        s = c[:6].sum(axis=0)
        assert s.min() >= 0.9 - 1e-12 and s.max() <= 1.1 + 1e-12


def test_deterministic_and_level_streams():
    p = synth.Problem(20, 10, 6, seed=5)
    a = synth.make_coeffs(p, threads=1)
    b = synth.make_coeffs(p, threads=4)
    assert np.array_equal(a, b)
    assert np.array_equal(synth.coeff_level(p, 3), a[:, 3])
    assert not np.array_equal(synth.make_coeffs(synth.Problem(20, 10, 6, seed=6)), a)
    assert np.array_equal(synth.make_rhs(p), synth.make_rhs(p))


def test_levels_and_aspect():
    dz = synth.level_thickness(70, 1.1)
    assert math.isclose(dz.sum(), 80_000.0, rel_tol=1e-12)
    assert math.isclose(dz[1] / dz[0], 1.1, rel_tol=1e-12)
    dz5 = synth.level_thickness(140, synth._stress_ratio())
    assert math.isclose(dz5[-1] / dz5[0], dz[-1] / dz[0], rel_tol=1e-9)
    # near-pole cell aspect ratio of the 2560 x 1920 grid: cos(phi_0) dlam / dphi ~ 1.23e-3
    p = synth.CONFIGS["n1280_2560x1920x70"]
    dphi = math.pi / p.nlat
    dlam = 2 * math.pi / p.nlon
    asp = math.cos(-math.pi / 2 + 0.5 * dphi) * dlam / dphi
    assert 1.2e-3 < asp < 1.25e-3


def test_band_contrast():
    k = synth.band_diffusivity(synth.CONFIGS["stress_1280x960x140"])
    assert k.min() == 1e-2 and k.max() == 1e2
    assert len(np.unique(k)) <= 8
    # contiguous bands
    assert np.sum(np.diff(k) != 0) <= 7


def test_xstar_smooth_plus_noise():
    p = synth.CONFIGS["small_96x72x20"]
    x = synth.make_xstar(p)
    x0 = synth.make_xstar(p, noise=0.0)
    d = x - x0
    assert abs(d.std() - 1e-3) < 1e-4
    assert np.isfinite(x).all() and x0.std() > 0.1
