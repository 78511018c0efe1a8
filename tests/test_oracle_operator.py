"""Pins of the oracle's spectral SWE operator (Eq. (1), Section 2)."""
import math

import numpy as np
import pytest
import scipy.special as sp
from scipy.linalg import eigvalsh

import synth
from oracle import operator as op

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH


def _J(T, m):
    """J = diag((-1)^n (1, -1, -1)) on the (Phi, zeta, delta) layout."""
    j = []
    for n in range(m, T + 1):
        s = (-1) ** n
        j += [s, -s, -s]
    return np.array(j, dtype=float)


@pytest.mark.parametrize("m", [0, 1, 7, 40, 63])
def test_scaled_operator_is_skew_hermitian_and_j_symmetric(m):
    T = 63
    L = op.scaled_block(T, m, A, OM, PB)
    assert np.max(np.abs(L + L.conj().T)) <= 1e-15 * np.max(np.abs(L))
    J = _J(T, m)
    assert np.array_equal(J[:, None] * np.conj(L) * J[None, :], -L)


@pytest.mark.parametrize("m", [0, 1, 5, 20])
def test_scaled_and_unscaled_forms_agree(m):
    T = 20
    Lh = op.scaled_block(T, m, A, OM, PB)
    L = op.unscaled_block(T, m, A, OM, PB)
    d = op.scaling_block(T, m, A, PB)
    assert np.max(np.abs(Lh / d[:, None] * d[None, :] - L)) <= 1e-15 * np.max(np.abs(L))


def test_balanced_jet_is_a_null_vector():
    # Section 6.1: the geostrophically balanced jet has zero time derivatives.
    T = 63
    x = synth.jet_state(T)
    L0 = op.unscaled_block(T, 0, A, OM, PB)
    X = op.block_of(x, T, 0)[:, 0]
    r = L0 @ X
    scale = np.abs(L0) @ np.abs(X)
    assert np.max(np.abs(r)) <= 1e-15 * np.max(scale)
    # A flipped Coriolis sign would break the balance.
    L0_wrong = op.unscaled_block(T, 0, A, -OM, PB)
    assert np.max(np.abs(L0_wrong @ X)) > 0.1 * np.max(scale)


def _scipy_grid(coef, T, P, dP, mu, lam, deriv=None):
    """Real grid field of spectral coefficients in scipy's basis.

    deriv: None, 'lam' (d/dlam) or 'mu' ((1-mu^2) d/dmu)."""
    out = np.zeros((len(mu), len(lam)))
    for m in range(T + 1):
        o = m * (T + 1) - m * (m - 1) // 2
        c = coef[o:o + T + 1 - m]
        base = P if deriv != "mu" else dP
        Fm = np.einsum("n,nj->j", c, base[m:T + 1, m, :])
        if deriv == "lam":
            Fm = 1j * m * Fm
        if deriv == "mu":
            Fm = (1 - mu * mu) * Fm
        ph = np.exp(1j * m * lam)
        out += (Fm.real[:, None] * np.ones_like(lam)[None, :]) if m == 0 else 2 * np.real(Fm[:, None] * ph[None, :])
    return out


def _scipy_analysis(field, T, P, mu, w, lam):
    nlon = len(lam)
    out = np.zeros((T + 1) * (T + 2) // 2, dtype=complex)
    for m in range(T + 1):
        o = m * (T + 1) - m * (m - 1) // 2
        Fm = field @ np.exp(-1j * m * lam) / nlon
        out[o:o + T + 1 - m] = np.einsum("nj,j,j->n", P[m:T + 1, m, :], w, Fm)
    return out


def test_operator_matches_pseudo_spectral_tendencies_of_eq1():
    """Evaluate Eq. (1) on a Gauss grid (scipy Legendre functions and their
    derivatives, grid products), project back, compare with the blocks."""
    T, nlat, nlon = 12, 24, 48
    mu, w = sp.roots_legendre(nlat)
    lam = 2 * math.pi * np.arange(nlon) / nlon
    Pall = sp.assoc_legendre_p_all(T + 1, T + 1, mu, norm=True, diff_n=1)
    P = Pall[0]                      # [n][m][j], m >= 0 at index m
    dP = Pall[1]
    st = synth.random_state(T, 1, 11)[0]
    phi, zeta, delta = st
    n_of = np.array([n for m in range(T + 1) for n in range(m, T + 1)], dtype=float)
    inv_lap = np.where(n_of > 0, -A * A / np.maximum(n_of * (n_of + 1), 1), 0.0)
    psi, chi = inv_lap * zeta, inv_lap * delta
    g = lambda c, d=None: _scipy_grid(c, T, P, dP, mu, lam, d)
    U = (g(chi, "lam") - g(psi, "mu")) / A
    V = (g(psi, "lam") + g(chi, "mu")) / A
    f = (2 * OM * mu)[:, None]
    lap_phi = g(-n_of * (n_of + 1) / (A * A) * phi)
    zeta_t = -f * g(delta) - (2 * OM / A) * V
    delta_t = f * g(zeta) - (2 * OM / A) * U - lap_phi
    phi_t = -PB * g(delta)
    got = np.stack([_scipy_analysis(x, T, P, mu, w, lam) for x in (phi_t, zeta_t, delta_t)])[None]
    want = np.zeros_like(got)
    for m in range(T + 1):
        X = op.block_of(st[None], T, m)
        op.scatter_block(want, op.unscaled_block(T, m, A, OM, PB) @ X, T, m)
    for v in range(3):
        assert np.linalg.norm(got[0, v] - want[0, v]) <= 1e-12 * np.linalg.norm(want[0, v])


def test_no_rotation_closed_form():
    # Omega = 0: per degree a (Phi, delta) gravity-wave pair at +-i w_n, zeta frozen.
    T, m = 20, 3
    L = op.scaled_block(T, m, A, 0.0, PB)
    ev = np.sort(eigvalsh(1j * L))
    wn = np.array([math.sqrt(PB * n * (n + 1)) / A for n in range(m, T + 1)])
    want = np.sort(np.concatenate([wn, -wn, np.zeros(T + 1 - m)]))
    assert np.max(np.abs(ev - want)) < 1e-15 * wn.max() * 10


def test_f_sphere_closed_form():
    # Section 4.3: with a constant f0 the eigenvalues are 0 and +-i sqrt(f0^2 + w_n^2).
    T, m, f0 = 16, 2, 2 * OM
    L = op.scaled_block(T, m, A, OM, PB, fsphere=f0)
    ev = np.sort(eigvalsh(1j * L))
    wn = np.array([math.sqrt(f0 * f0 + PB * n * (n + 1) / A ** 2) for n in range(m, T + 1)])
    want = np.sort(np.concatenate([wn, -wn, np.zeros(T + 1 - m)]))
    assert np.max(np.abs(ev - want)) < 1e-14 * wn.max()


@pytest.mark.parametrize("T", [63, 128])
def test_spectral_radius_close_to_top_gravity_wave(T):
    wT = math.sqrt(PB * T * (T + 1)) / A
    r = max(np.max(np.abs(eigvalsh(1j * op.scaled_block(T, m, A, OM, PB)))) for m in range(T + 1))
    assert wT <= r < 1.001 * wT
