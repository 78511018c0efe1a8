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

Vector transforms (Eq. (1), Section 3): winds (u, v) from vorticity and
divergence through the stream function and velocity potential, and back, with
the latitude derivative of P_n^m taken from the differentiated recurrence.
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


def legendre(T: int, mu: np.ndarray, with_h: bool = False):
    """Orthonormal P_n^m(mu_j) for 0 <= m <= T, n = m..T.

    Returns a list P with P[m] of shape (T+1-m, len(mu)).  Three-term
    recurrence in n,  mu P_{n-1}^m = eps_n^m P_n^m + eps_{n-1}^m P_{n-2}^m,
    eps_n^m = sqrt((n^2-m^2)/(4n^2-1)), seeded with
    P_m^m = sqrt(prod_{k=1}^{m} (2k+1)/(2k)) (1-mu^2)^{m/2} / sqrt(2).
    The seed is formed in logarithms with a per-column power-of-two offset so
    that columns whose seed underflows (large m near the poles) are still
    carried exactly through the recurrence; values below 1e-300 are returned
    as zero.

    with_h: also return H[m], H_n^m = (1 - mu^2) dP_n^m/dmu, obtained by
    differentiating the same recurrence (times 1 - mu^2):
      eps_n H_n = (1 - mu^2) P_{n-1} + mu H_{n-1} - eps_{n-1} H_{n-2},
    seeded with H_m^m = -m mu P_m^m.  Returns (P, H) then.
    """
    mu = np.asarray(mu, dtype=np.float64)
    s2 = np.maximum(1.0 - mu * mu, 0.0)
    logsin = 0.5 * np.log(s2)
    out, outh = [], []
    logc = -0.5 * math.log(2.0)
    for m in range(T + 1):
        if m > 0:
            logc += 0.5 * math.log((2.0 * m + 1.0) / (2.0 * m))
        logseed = logc + m * logsin
        # Offset: carry values scaled by 2^-e so the seed is O(1).
        e = np.floor(logseed / math.log(2.0))
        scaled = np.exp(logseed - e * math.log(2.0))
        p_prev2 = np.zeros_like(mu)
        p_prev = scaled
        g_prev2 = np.zeros_like(mu)
        g_prev = -m * mu * scaled
        vals = [p_prev]
        hvals = [g_prev]
        for n in range(m + 1, T + 1):
            em = _eps(n - 1, m) if n - 1 > m else 0.0
            en = _eps(n, m)
            pn = (mu * p_prev - em * p_prev2) / en
            gn = (s2 * p_prev + mu * g_prev - em * g_prev2) / en
            # Renormalise the running values when they grow large, moving the
            # factor into the exponent (keeps the recurrence in range).
            big = np.maximum(np.abs(pn), np.abs(gn)) > 1e200
            if np.any(big):
                f = np.where(big, 2.0 ** -600, 1.0)
                pn, p_prev, gn, g_prev = pn * f, p_prev * f, gn * f, g_prev * f
                vals = [v * f for v in vals]
                hvals = [v * f for v in hvals]
                e = e + np.where(big, 600.0, 0.0)
            p_prev2, p_prev = p_prev, pn
            g_prev2, g_prev = g_prev, gn
            vals.append(pn)
            hvals.append(gn)

        def unscale(vs):
            col = np.zeros((T + 1 - m, len(mu)))
            for i, v in enumerate(vs):
                with np.errstate(over="ignore", under="ignore"):
                    col[i] = np.where(e > -1000, np.ldexp(v, np.clip(e, -2000, 2000).astype(np.int64)), 0.0)
            col[np.abs(col) < 1e-300] = 0.0
            return col

        out.append(unscale(vals))
        if with_h:
            outh.append(unscale(hvals))
    return (out, outh) if with_h else out


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


def vortdiv_to_uv(vd: np.ndarray, T: int, nlat: int, nlon: int, radius: float) -> np.ndarray:
    """Winds from vorticity and divergence (Eq. (1), Section 3).

    vd: spectral [B][2][nspec] (zeta, delta).  Returns the grid [B][2][nlat][nlon]
    of (u, v) in the units of radius * zeta.  With V = k x grad(psi) + grad(chi),
    lap psi = zeta, lap chi = delta (lap -> -n(n+1)/a^2 on degree n; the n = 0
    part carries no wind), and the cos(lat)-scaled winds U = u cos(lat),
    V = v cos(lat) of Section 3:
      U = -(1/a) (1 - mu^2) dpsi/dmu + (1/a) dchi/dlam,
      V =  (1/a) dpsi/dlam + (1/a) (1 - mu^2) dchi/dmu,
    summed directly over the modes with H_n^m = (1 - mu^2) dP_n^m/dmu from the
    differentiated recurrence, then u = U / cos(lat), v = V / cos(lat).
    """
    vd = np.asarray(vd, dtype=np.complex128)
    B = vd.shape[0]
    mu, _ = gauss_latitudes(nlat)
    P, Hm = legendre(T, mu, with_h=True)
    k = np.arange(nlon)
    U = np.zeros((B, nlat, nlon))
    V = np.zeros((B, nlat, nlon))
    for mm in range(T + 1):
        o = index(T, mm, mm)
        n = np.arange(mm, T + 1)
        inv_lap = np.zeros(len(n))
        inv_lap[n > 0] = -radius * radius / (n[n > 0] * (n[n > 0] + 1.0))
        psi = vd[:, 0, o:o + T + 1 - mm] * inv_lap
        chi = vd[:, 1, o:o + T + 1 - mm] * inv_lap
        Um = (-np.einsum("bn,nj->bj", psi, Hm[mm]) + 1j * mm * np.einsum("bn,nj->bj", chi, P[mm])) / radius
        Vm = (1j * mm * np.einsum("bn,nj->bj", psi, P[mm]) + np.einsum("bn,nj->bj", chi, Hm[mm])) / radius
        if mm == 0:
            U += Um.real[:, :, None]
            V += Vm.real[:, :, None]
        else:
            ph = np.exp(1j * 2.0 * math.pi * mm * k / nlon)
            U += 2.0 * np.real(Um[:, :, None] * ph[None, None, :])
            V += 2.0 * np.real(Vm[:, :, None] * ph[None, None, :])
    cosl = np.sqrt(1.0 - mu * mu)[None, :, None]
    return np.stack([U / cosl, V / cosl], axis=1)


def uv_to_vortdiv(uv: np.ndarray, T: int, radius: float) -> np.ndarray:
    """Vorticity and divergence of the winds (Eq. (1), Section 3).

    uv: grid [B][2][nlat][nlon] of (u, v).  Returns spectral [B][2][nspec] of
    zeta = k . curl V and delta = div V:
      zeta = (1/(a (1 - mu^2))) dV/dlam - (1/a) dU/dmu,
      delta = (1/(a (1 - mu^2))) dU/dlam + (1/a) dV/dmu   (U, V = u, v times cos(lat)).
    The analysis integral of the mu-derivative is taken by parts (U and V
    vanish at the poles), so with u~ = u / cos(lat), v~ = v / cos(lat) and
    their longitude coefficients u~_m, v~_m:
      zeta_n^m = (1/a) sum_j w_j (i m v~_m P_n^m + u~_m H_n^m)(mu_j),
      delta_n^m = (1/a) sum_j w_j (i m u~_m P_n^m - v~_m H_n^m)(mu_j).
    """
    uv = np.asarray(uv, dtype=np.float64)
    B, _, nlat, nlon = uv.shape
    mu, w = gauss_latitudes(nlat)
    P, Hm = legendre(T, mu, with_h=True)
    cosl = np.sqrt(1.0 - mu * mu)[None, :, None]
    k = np.arange(nlon)
    m = np.arange(T + 1)
    E = np.exp(-1j * 2.0 * math.pi * np.outer(m, k) / nlon) / nlon
    Fu = np.einsum("bjk,mk->bjm", uv[:, 0] / cosl, E)
    Fv = np.einsum("bjk,mk->bjm", uv[:, 1] / cosl, E)
    out = np.zeros((B, 2, nspec(T)), dtype=np.complex128)
    for mm in range(T + 1):
        o = index(T, mm, mm)
        sl = slice(o, o + T + 1 - mm)
        out[:, 0, sl] = (1j * mm * np.einsum("nj,j,bj->bn", P[mm], w, Fv[:, :, mm])
                         + np.einsum("nj,j,bj->bn", Hm[mm], w, Fu[:, :, mm])) / radius
        out[:, 1, sl] = (1j * mm * np.einsum("nj,j,bj->bn", P[mm], w, Fu[:, :, mm])
                         - np.einsum("nj,j,bj->bn", Hm[mm], w, Fv[:, :, mm])) / radius
    return out
