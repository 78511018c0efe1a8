"""Spherical-harmonic transforms, plain FP64 (Section 3).

Test infrastructure: see the package docstring.

Synthesis (Section 3):  xi(lam, mu) = sum_r sum_{s>=|r|} xi_s^r P_s^r(mu) e^{i r lam}.
Analysis  (Section 3):  xi_s^r = int_{-1}^{1} (1/2pi) int_0^{2pi} xi e^{-i r lam} dlam P_s^r(mu) dmu.
For this pair to be inverse to each other the P_s^r must be orthonormal on
[-1, 1] (int P^2 dmu = 1); no Condon-Shortley phase is used.  The latitude
integral is Gauss-Legendre quadrature on the Gaussian latitudes (Section 3),
the longitude integral the trapezoid rule on nlon equispaced points, written
here as a plain DFT sum (no FFT).

Triangular truncation: 0 <= m <= n <= T.  Real fields: xi^{-m} = conj(xi^m),
so only m >= 0 is stored and synthesis returns
  sum_n Re(xi_n^0) P_n^0 + 2 Re sum_{m>0} sum_n xi_n^m P_n^m e^{i m lam}.
Grid layout: [B][nlat][nlon], latitude j = 0 northernmost (mu descending),
lam_k = 2 pi k / nlon.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_legendre


def nspec(T: int) -> int:
    return (T + 1) * (T + 2) // 2


def index(T: int, m: int, n: int) -> int:
    """Position of (n, m) in the m-major triangular list."""
    return m * (T + 1) - m * (m - 1) // 2 + (n - m)


def _legendre_pn(n, x):
    """P_n(x) and P_{n-1}(x) by Bonnet's recurrence k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2}."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, p0


def gauss_latitudes(nlat: int):
    """Gauss-Legendre nodes mu_j = sin(lat_j), north to south, and weights.

    The nodes are the roots of P_nlat.  scipy's roots serve as starting
    guesses and are refined by Newton's method; the weights are
    w_j = 2 / ((1 - x_j^2) P'_nlat(x_j)^2) with P'_n = n (x P_n - P_{n-1})/(x^2 - 1).
    (scipy's own weights lose ~1e-10 relative accuracy at nlat = 256.)
    """
    x, _ = roots_legendre(nlat)
    for _ in range(3):
        pn, pm = _legendre_pn(nlat, x)
        dp = nlat * (x * pn - pm) / (x * x - 1.0)
        x = x - pn / dp
    pn, pm = _legendre_pn(nlat, x)
    dp = nlat * (x * pn - pm) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    return x[::-1].copy(), w[::-1].copy()


def _eps(n, m):
    return math.sqrt((n * n - m * m) / (4.0 * n * n - 1.0))


def legendre(T: int, mu: np.ndarray):
    """Orthonormal P_n^m(mu_j) for 0 <= m <= T, n = m..T.

    Returns a list P with P[m] of shape (T+1-m, len(mu)).  Three-term
    recurrence in n,  mu P_{n-1}^m = eps_n^m P_n^m + eps_{n-1}^m P_{n-2}^m,
    eps_n^m = sqrt((n^2-m^2)/(4n^2-1)), seeded with
    P_m^m = sqrt(prod_{k=1}^{m} (2k+1)/(2k)) (1-mu^2)^{m/2} / sqrt(2).
    The seed is formed in logarithms with a per-column power-of-two offset so
    that columns whose seed underflows (large m near the poles) are still
    carried exactly through the recurrence; values below 1e-300 are returned
    as zero.
    """
    mu = np.asarray(mu, dtype=np.float64)
    s2 = np.maximum(1.0 - mu * mu, 0.0)
    logsin = 0.5 * np.log(s2)
    out = []
    logc = -0.5 * math.log(2.0)
    for m in range(T + 1):
        if m > 0:
            logc += 0.5 * math.log((2.0 * m + 1.0) / (2.0 * m))
        logseed = logc + m * logsin
        # Offset: carry values scaled by 2^-e so the seed is O(1).
        e = np.floor(logseed / math.log(2.0))
        scaled = np.exp(logseed - e * math.log(2.0))
        col = np.zeros((T + 1 - m, len(mu)))
        p_prev2 = np.zeros_like(mu)
        p_prev = scaled
        vals = [p_prev]
        for n in range(m + 1, T + 1):
            em = _eps(n - 1, m) if n - 1 > m else 0.0
            pn = (mu * p_prev - em * p_prev2) / _eps(n, m)
            # Renormalise the running pair when it grows large, moving the
            # factor into the exponent (keeps the recurrence in range).
            big = np.abs(pn) > 1e200
            if np.any(big):
                f = np.where(big, 2.0 ** -600, 1.0)
                pn = pn * f
                p_prev = p_prev * f
                vals = [v * f for v in vals]
                e = e + np.where(big, 600.0, 0.0)
            p_prev2, p_prev = p_prev, pn
            vals.append(pn)
        for i, v in enumerate(vals):
            with np.errstate(over="ignore", under="ignore"):
                col[i] = np.where(e > -1000, np.ldexp(v, np.clip(e, -2000, 2000).astype(np.int64)), 0.0)
        col[np.abs(col) < 1e-300] = 0.0
        out.append(col)
    return out


def analysis(grid: np.ndarray, T: int) -> np.ndarray:
    """Grid [B][nlat][nlon] (real) -> spectral [B][nspec] (complex128)."""
    grid = np.asarray(grid, dtype=np.float64)
    B, nlat, nlon = grid.shape
    mu, w = gauss_latitudes(nlat)
    P = legendre(T, mu)
    k = np.arange(nlon)
    m = np.arange(T + 1)
    E = np.exp(-1j * 2.0 * math.pi * np.outer(m, k) / nlon) / nlon      # [T+1][nlon]
    F = np.einsum("bjk,mk->bjm", grid, E)                                  # (1/2pi) int dlam
    out = np.zeros((B, nspec(T)), dtype=np.complex128)
    for mm in range(T + 1):
        o = index(T, mm, mm)
        out[:, o:o + T + 1 - mm] = np.einsum("nj,j,bj->bn", P[mm], w, F[:, :, mm])
    return out


def synthesis(spec: np.ndarray, T: int, nlat: int, nlon: int) -> np.ndarray:
    """Spectral [B][nspec] -> real grid [B][nlat][nlon] (direct double sum)."""
    spec = np.asarray(spec, dtype=np.complex128)
    B = spec.shape[0]
    mu, _ = gauss_latitudes(nlat)
    P = legendre(T, mu)
    k = np.arange(nlon)
    out = np.zeros((B, nlat, nlon))
    for mm in range(T + 1):
        o = index(T, mm, mm)
        Fm = np.einsum("bn,nj->bj", spec[:, o:o + T + 1 - mm], P[mm])     # [B][nlat]
        if mm == 0:
            out += Fm.real[:, :, None] * np.ones(nlon)[None, None, :]
        else:
            ph = np.exp(1j * 2.0 * math.pi * mm * k / nlon)
            out += 2.0 * np.real(Fm[:, :, None] * ph[None, None, :])
    return out
