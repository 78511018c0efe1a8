"""Pins of the oracle's spherical-harmonic transforms (Section 3)."""
import math

import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import sh


@pytest.mark.parametrize("nlat", [16, 64, 128, 256])
def test_gauss_quadrature_exact_for_polynomials(nlat):
    mu, w = sh.gauss_latitudes(nlat)
    assert np.all(np.diff(mu) < 0)                       # north to south
    for k in range(0, 2 * nlat, 7):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * mu ** k) - exact) < 1e-14


def test_legendre_against_scipy():
    # scipy's normalised functions carry the Condon-Shortley phase (-1)^m.
    mu, _ = sh.gauss_latitudes(48)
    T = 40
    P = sh.legendre(T, mu)
    ref = sp.assoc_legendre_p_all(T, T, mu, norm=True)[0]
    err = 0.0
    for m in range(T + 1):
        for n in range(m, T + 1):
            err = max(err, np.max(np.abs(P[m][n - m] - (-1) ** m * ref[n][m])))
    assert err < 1e-13


def test_legendre_closed_forms():
    mu = np.linspace(-0.99, 0.99, 11)
    P = sh.legendre(2, mu)
    assert np.allclose(P[0][0], 1 / math.sqrt(2), rtol=0, atol=1e-15)
    assert np.allclose(P[0][1], math.sqrt(1.5) * mu, rtol=0, atol=1e-15)
    assert np.allclose(P[0][2], math.sqrt(2.5) * (1.5 * mu * mu - 0.5), rtol=0, atol=1e-15)
    assert np.allclose(P[1][0], math.sqrt(3) / 2 * np.sqrt(1 - mu * mu), rtol=0, atol=1e-15)


def test_orthonormality_t256():
    # Exact up to polynomial degree 2 nlat - 1 = 511, i.e. n, n' <= 255.
    mu, w = sh.gauss_latitudes(256)
    P = sh.legendre(256, mu)
    err = 0.0
    for m in range(256):
        G = (P[m] * w) @ P[m].T
        k = 256 - m
        err = max(err, np.max(np.abs(G[:k, :k] - np.eye(k))))
    assert err < 1e-13
    # Deep near the poles the seed underflows; values are flushed, never garbage.
    assert np.all(np.isfinite(np.concatenate([p.ravel() for p in P])))


def test_analysis_of_scipy_harmonics_gives_unit_coefficients():
    T, nlat, nlon = 10, 16, 32
    mu, _ = sh.gauss_latitudes(nlat)
    th = np.arccos(mu)
    lam = 2 * math.pi * np.arange(nlon) / nlon
    for (n, m) in [(0, 0), (3, 0), (3, 2), (7, 5), (10, 10)]:
        # scipy: Y_n^m = (-1)^m P_n^m(cos th) e^{im phi} / sqrt(2 pi) in this basis
        Y = sp.sph_harm_y(n, m, th[:, None], lam[None, :])
        base = math.sqrt(2 * math.pi) * (-1) ** m * Y
        field = base.real if m == 0 else 2 * base.real
        spec = sh.analysis(field[None], T)[0]
        expect = np.zeros(sh.nspec(T), dtype=complex)
        expect[sh.index(T, m, n)] = 1.0
        assert np.max(np.abs(spec - expect)) < 1e-13
        # imaginary part: field 2 Re(i base) = -2 Im(base) has coefficient i
        if m > 0:
            spec_i = sh.analysis((-2 * base.imag)[None], T)[0]
            assert abs(spec_i[sh.index(T, m, n)] - 1j) < 1e-13


def test_round_trip():
    T, nlat, nlon = 31, 32, 64
    u = synth.random_state(T, 2, 3).reshape(6, -1)
    g = sh.synthesis(u, T, nlat, nlon)
    back = sh.analysis(g, T)
    assert np.max(np.abs(back - u)) / np.max(np.abs(u)) < 1e-13


def test_truncation_limits_of_undersized_grids():
    # A 256x128 grid at T128 (and 512x256 at T256): Gauss quadrature with
    # nlat = T is exact only to degree 2T - 1, and m = nlon/2 is the Nyquist
    # wave whose imaginary part is invisible on the grid.  Everything below
    # both limits round-trips.
    T, nlat, nlon = 128, 128, 256
    u = synth.random_state(T, 1, 4).reshape(3, -1)
    back = sh.analysis(sh.synthesis(u, T, nlat, nlon), T)
    n = np.array([n for m in range(T + 1) for n in range(m, T + 1)])
    m = np.array([m for m in range(T + 1) for n in range(m, T + 1)])
    ok = (n < nlat) & (m < nlon // 2)
    assert np.max(np.abs(back[:, ok] - u[:, ok])) / np.max(np.abs(u)) < 1e-13
    assert np.max(np.abs(back[:, ~ok] - u[:, ~ok])) / np.max(np.abs(u[:, ~ok])) > 1e-3
