"""Pins of the oracle's vector transforms (Eq. (1), Section 3, Section 6.1).

The winds follow from V = k x grad(psi) + grad(chi) with lap psi = zeta,
lap chi = delta.  The oracle computes the latitude derivative of P_n^m by
differentiating its recurrence; these tests hold it to things fixed outside
that code: finite differences, a textbook identity, the solid-body rotation of
Section 6.1 and rotated/divergent versions of it in closed form, Parseval's
identity for the kinetic energy, and the exact round trip.
"""
import math

import numpy as np
import pytest

import synth
from oracle import sh as osh

A = synth.EARTH_RADIUS
U0 = 20.0


def _real_m0(vd, T):
    """Zonal (m = 0) coefficients of a real field are real."""
    vd = vd.copy()
    vd[..., :T + 1] = vd[..., :T + 1].real
    return vd


def _random_vd(T, B, seed):
    rng = np.random.default_rng(seed)
    n = synth.nspec(T)
    vd = (rng.standard_normal((B, 2, n)) + 1j * rng.standard_normal((B, 2, n))) * 1e-5
    vd[..., 0] = 0.0  # the (0, 0) vorticity / divergence of any wind is zero
    return _real_m0(vd, T)


def test_derivative_matches_finite_differences():
    T = 24
    mu = np.array([-0.93, -0.41, 0.07, 0.55, 0.88])
    _, H = osh.legendre(T, mu, with_h=True)
    d = 1e-4
    pts = [osh.legendre(T, mu + k * d) for k in (-2, -1, 1, 2)]
    for m in range(T + 1):
        fd = (pts[0][m] - 8 * pts[1][m] + 8 * pts[2][m] - pts[3][m]) / (12 * d)
        want = (1 - mu * mu) * fd
        scale = np.max(np.abs(H[m])) + 1e-300
        assert np.max(np.abs(H[m] - want)) / scale < 1e-8, m


def test_derivative_textbook_identity():
    # (1 - mu^2) dP_n^m/dmu = (n+1) eps_n P_{n-1} - n eps_{n+1} P_{n+1}
    T = 40
    mu, _ = osh.gauss_latitudes(48)
    P = osh.legendre(T + 1, mu)
    _, H = osh.legendre(T, mu, with_h=True)
    for m in range(T + 1):
        for n in range(m, T + 1):
            want = -n * math.sqrt(((n + 1) ** 2 - m * m) / (4.0 * (n + 1) ** 2 - 1)) * P[m][n + 1 - m]
            if n > m:
                want = want + (n + 1) * math.sqrt((n * n - m * m) / (4.0 * n * n - 1)) * P[m][n - 1 - m]
            assert np.max(np.abs(H[m][n - m] - want)) < 1e-12 * max(1.0, np.max(np.abs(want))), (m, n)


def _grid(nlat, nlon):
    mu, _ = osh.gauss_latitudes(nlat)
    lat = np.arcsin(mu)[:, None]
    lam = 2 * math.pi * np.arange(nlon)[None, :] / nlon
    return lat, lam


def test_solid_body_rotation_of_section_6_1():
    # u = u0 cos(lat), v = 0 (Section 6.1): psi = -a u0 sin(lat), so
    # zeta = 2 u0 sin(lat) / a = (2 u0 / a) P_1^0 / sqrt(3/2).
    T, nlat, nlon = 10, 12, 24
    vd = np.zeros((1, 2, synth.nspec(T)), dtype=np.complex128)
    vd[0, 0, osh.index(T, 0, 1)] = 2 * U0 / A / math.sqrt(1.5)
    uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    lat, lam = _grid(nlat, nlon)
    assert np.max(np.abs(uv[0, 0] - U0 * np.cos(lat) * np.ones_like(lam))) < 1e-12 * U0
    assert np.max(np.abs(uv[0, 1])) < 1e-12 * U0


def test_zonal_divergent_flow():
    # chi = a u0 sin(lat): v = u0 cos(lat), u = 0, delta = -2 u0 sin(lat) / a
    T, nlat, nlon = 10, 12, 24
    vd = np.zeros((1, 2, synth.nspec(T)), dtype=np.complex128)
    vd[0, 1, osh.index(T, 0, 1)] = -2 * U0 / A / math.sqrt(1.5)
    uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    lat, lam = _grid(nlat, nlon)
    assert np.max(np.abs(uv[0, 1] - U0 * np.cos(lat) * np.ones_like(lam))) < 1e-12 * U0
    assert np.max(np.abs(uv[0, 0])) < 1e-12 * U0


def test_rotation_about_an_equatorial_axis():
    # psi = a u0 cos(lat) cos(lam): u = u0 sin(lat) cos(lam), v = -u0 sin(lam).
    # chi = a u0 cos(lat) cos(lam): u = -u0 sin(lam), v = -u0 sin(lat) cos(lam).
    # cos(lat) cos(lam) has the single coefficient 1/sqrt(3) at (n, m) = (1, 1),
    # and lap = -2/a^2 on degree 1.
    T, nlat, nlon = 6, 8, 16
    lat, lam = _grid(nlat, nlon)
    c = -2.0 / A ** 2 * A * U0 / math.sqrt(3.0)
    for var in (0, 1):
        vd = np.zeros((1, 2, synth.nspec(T)), dtype=np.complex128)
        vd[0, var, osh.index(T, 1, 1)] = c
        uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
        if var == 0:
            u, v = U0 * np.sin(lat) * np.cos(lam), -U0 * np.sin(lam) * np.ones_like(lat)
        else:
            u, v = -U0 * np.sin(lam) * np.ones_like(lat), -U0 * np.sin(lat) * np.cos(lam)
        assert np.max(np.abs(uv[0, 0] - u)) < 1e-12 * U0, var
        assert np.max(np.abs(uv[0, 1] - v)) < 1e-12 * U0, var


def _point_fields(spec, T, lat, lam):
    """A real field of spectral coefficients `spec` at one point."""
    P = osh.legendre(T, np.array([math.sin(lat)]))
    val = 0.0
    for m in range(T + 1):
        s = np.dot(spec[osh.index(T, m, m):osh.index(T, m, m) + T + 1 - m], P[m][:, 0])
        val += s.real if m == 0 else 2 * (s * np.exp(1j * m * lam)).real
    return val


def test_winds_match_finite_differences_of_psi_and_chi():
    # u = -(1/a) dpsi/dlat + dchi/dlam / (a cos(lat)),
    # v = dpsi/dlam / (a cos(lat)) + (1/a) dchi/dlat, by central differences.
    T, nlat, nlon = 15, 16, 32
    vd = _random_vd(T, 1, 3)
    n = np.array([n for m in range(T + 1) for n in range(m, T + 1)], dtype=float)
    inv = np.where(n > 0, -A * A / np.maximum(n * (n + 1), 1), 0.0)
    psi, chi = vd[0, 0] * inv, vd[0, 1] * inv
    uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    lat, lam = _grid(nlat, nlon)
    d = 1e-4
    for j, k in [(0, 0), (3, 7), (8, 31), (11, 16), (15, 5)]:
        ph, la = lat[j, 0], lam[0, k]

        def dlat(f):
            return (f(ph - 2 * d, la) - 8 * f(ph - d, la) + 8 * f(ph + d, la) - f(ph + 2 * d, la)) / (12 * d)

        def dlam(f):
            return (f(ph, la - 2 * d) - 8 * f(ph, la - d) + 8 * f(ph, la + d) - f(ph, la + 2 * d)) / (12 * d)

        fpsi = lambda p, l: _point_fields(psi, T, p, l)  # noqa: E731
        fchi = lambda p, l: _point_fields(chi, T, p, l)  # noqa: E731
        u = -dlat(fpsi) / A + dlam(fchi) / (A * math.cos(ph))
        v = dlam(fpsi) / (A * math.cos(ph)) + dlat(fchi) / A
        scale = np.max(np.abs(uv))
        assert abs(uv[0, 0, j, k] - u) < 1e-8 * scale, (j, k)
        assert abs(uv[0, 1, j, k] - v) < 1e-8 * scale, (j, k)


def test_kinetic_energy_parseval():
    # int (u^2 + v^2) dmu dlam / (2 pi) = sum_{n,m} c_m n(n+1)/a^2 (|psi|^2 + |chi|^2),
    # c_0 = 1, c_m = 2 (orthonormal P, cross terms integrate to zero).
    T, nlat, nlon = 20, 24, 48
    vd = _random_vd(T, 2, 5)
    uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    _, w = osh.gauss_latitudes(nlat)
    grid_ke = np.einsum("j,bjk->b", w, uv[:, 0] ** 2 + uv[:, 1] ** 2) / nlon
    n = np.array([n for m in range(T + 1) for n in range(m, T + 1)], dtype=float)
    cm = np.array([1.0 if m == 0 else 2.0 for m in range(T + 1) for n in range(m, T + 1)])
    inv = np.where(n > 0, A * A / np.maximum(n * (n + 1), 1), 0.0)  # |psi|^2 n(n+1)/a^2 = a^2 |zeta|^2/(n(n+1))
    spec_ke = np.einsum("k,bvk->b", cm * inv, np.abs(vd) ** 2)
    assert np.allclose(grid_ke, spec_ke, rtol=1e-12, atol=0)


@pytest.mark.parametrize("T,nlat,nlon", [(15, 16, 32), (21, 30, 64), (31, 32, 64)])
def test_round_trip(T, nlat, nlon):
    vd = _random_vd(T, 2, T)
    uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    back = osh.uv_to_vortdiv(uv, T, A)
    assert np.max(np.abs(back - vd)) < 1e-12 * np.max(np.abs(vd))
    uv2 = osh.vortdiv_to_uv(back, T, nlat, nlon, A)
    assert np.max(np.abs(uv2 - uv)) < 1e-12 * np.max(np.abs(uv))


def test_curl_of_solid_body_rotation():
    # zeta of u = u0 cos(lat) is 2 u0 sin(lat) / a, and its divergence is zero.
    T, nlat, nlon = 8, 10, 20
    lat, lam = _grid(nlat, nlon)
    uv = np.stack([U0 * np.cos(lat) * np.ones_like(lam), np.zeros((nlat, nlon))])[None]
    vd = osh.uv_to_vortdiv(uv, T, A)
    want = np.zeros_like(vd)
    want[0, 0, osh.index(T, 0, 1)] = 2 * U0 / A / math.sqrt(1.5)
    assert np.max(np.abs(vd - want)) < 1e-13 * U0 / A
