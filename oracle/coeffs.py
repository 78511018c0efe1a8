"""REXI coefficients, plain FP64 (Section 4.1 and Section 6.1).

Test infrastructure: see the package docstring.

Steps, in the paper's order and notation:

1. Rational approximation of the Gaussian (Section 4.1, first display):
   psi_h(x) = (4 pi)^{-1/2} exp(-x^2/(4h^2)) ~ Re sum_{l=-K}^{K} a_l / (i x/h + mu + i l).
   The paper takes mu and a_l from Haut et al. (their Table 1), which is not
   available here, so the coefficients are fitted: a_{-l} = conj(a_l) (the
   Gaussian is even and real), so a_0 is real and there are 2K+1 real unknowns;
   for a fixed real mu < 0 the fit is a linear least-squares problem on a grid
   of y = x/h, and mu is chosen by a scan that minimises the maximum error.
2. Gaussian sum for the oscillation (Section 4.1, Eq. (2)):
   e^{ix} ~ sum_{m=-M}^{M} b_m psi_h(x + m h) with b_m = e^{h^2} e^{-imh}.
   The paper does not print b_m; this value follows from Poisson summation and
   the Fourier transform of the Gaussian, int psi_h(t) e^{-i xi t} dt = h e^{-h^2 xi^2}.
3. Merge: inserting step 1 into step 2 gives poles alpha_n = h (mu + i n),
   n = -(M+K)..(M+K), with beta^c_n = h sum_{m+l=n} Re(b_m) a_l for the real
   part (cos x ~ Re sum beta^c_n/(ix + alpha_n)) and beta^s_n the same with
   Im(b_m) for the imaginary part.
4. Taking the real part of a rational function of x adds the mirrored poles.
   Merging the real-part and imaginary-part approximations therefore gives the
   two-sided form  e^{z} ~ sum_n beta+_n/(z + alpha_n) + sum_n beta-_n/(alpha_n - z),
   beta+-_n = (beta^c_n +- i beta^s_n)/2, valid for z = i x and, by the spectral
   theorem, for z = dt L with L skew-Hermitian.
5. Renormalisation (Section 6.1): the sum at x = 0 is g(0) = sum_n beta^c_n/alpha_n
   instead of 1; dividing every beta by g(0) makes stationary modes exact.
"""
from __future__ import annotations

import functools
import math

import numpy as np


def _gauss_target(y):
    return np.exp(-0.25 * y * y) / math.sqrt(4.0 * math.pi)


def _fit_basis(y, mu, K):
    """Columns of Re sum a_l/(iy + mu + il) in the real unknowns.

    Unknowns: a_0 (real), then (Re a_l, Im a_l) for l = 1..K.  With
    a_{-l} = conj(a_l), the pair (l, -l) contributes
    Re a_l * [mu/(mu^2+(y+l)^2) + mu/(mu^2+(y-l)^2)]
      + Im a_l * [(y+l)/(mu^2+(y+l)^2) - (y-l)/(mu^2+(y-l)^2)].
    """
    cols = [mu / (mu * mu + y * y)]
    for l in range(1, K + 1):
        dp = mu * mu + (y + l) ** 2
        dm = mu * mu + (y - l) ** 2
        cols.append(mu / dp + mu / dm)
        cols.append((y + l) / dp - (y - l) / dm)
    return np.stack(cols, axis=1)


def _unpack(c, K):
    a = np.zeros(2 * K + 1, dtype=np.complex128)
    a[K] = c[0]
    for l in range(1, K + 1):
        a[K + l] = c[2 * l - 1] + 1j * c[2 * l]
        a[K - l] = np.conj(a[K + l])
    return a


def gaussian_rational(y, mu, a):
    """Evaluate Re sum_{l=-K}^{K} a_l / (i y + mu + i l) (a indexed l = -K..K)."""
    K = (len(a) - 1) // 2
    y = np.asarray(y, dtype=np.float64)
    l = np.arange(-K, K + 1)
    return np.real((a[None, :] / (1j * y[:, None] + mu + 1j * l[None, :])).sum(axis=1))


FIT_YMAX = 80.0
FIT_NY = 8001
CHECK_YMAX = 200.0
CHECK_NY = 100001


@functools.lru_cache(maxsize=8)
def fit_gaussian(K: int = 11, mu_lo: float = -5.5, mu_hi: float = -3.5, mu_step: float = 0.01):
    """Least-squares fit of the Gaussian by 2K+1 conjugate-symmetric poles.

    Returns (mu, a, max_err) with a indexed l = -K..K and max_err the largest
    absolute error on y in [0, 200] (the error is even in y).
    """
    y = np.linspace(0.0, FIT_YMAX, FIT_NY)
    b = _gauss_target(y)
    yc = np.linspace(0.0, CHECK_YMAX, CHECK_NY)
    bc = _gauss_target(yc)
    best = None
    for mu in np.arange(mu_lo, mu_hi + 0.5 * mu_step, mu_step):
        c, *_ = np.linalg.lstsq(_fit_basis(y, mu, K), b, rcond=None)
        err = float(np.max(np.abs(_fit_basis(yc, mu, K) @ c - bc)))
        if best is None or err < best[2]:
            best = (float(mu), c, err)
    mu, c, err = best
    return mu, _unpack(c, K), err


def gaussian_sum_weights(M: int, h: float):
    """b_m = e^{h^2} e^{-imh}, m = -M..M (Section 4.1, Eq. (2))."""
    m = np.arange(-M, M + 1)
    return math.exp(h * h) * np.exp(-1j * m * h)


def rexi_coefficients(M: int, h: float, K: int = 11, normalize: bool = True, fit=None):
    """Poles and two-sided weights of T-REXI.

    Returns a dict with ``n`` (pole index -(M+K)..(M+K)), ``alpha``,
    ``beta_plus``, ``beta_minus`` (so that e^{z} ~ sum beta+/(z+alpha) +
    sum beta-/(alpha-z)), ``beta_c``, ``beta_s``, ``g0`` (the sum at x = 0 before
    renormalisation) and the fit used.
    """
    if fit is None:
        fit = fit_gaussian(K)
    mu, a, _ = fit
    b = gaussian_sum_weights(M, h)
    n = np.arange(-(M + K), M + K + 1)
    beta_c = np.zeros(len(n), dtype=np.complex128)
    beta_s = np.zeros(len(n), dtype=np.complex128)
    for mi, m in enumerate(range(-M, M + 1)):
        for li, l in enumerate(range(-K, K + 1)):
            beta_c[m + l + M + K] += h * b[mi].real * a[li]
            beta_s[m + l + M + K] += h * b[mi].imag * a[li]
    alpha = h * (mu + 1j * n)
    g0 = complex(np.sum(beta_c / alpha))
    if normalize:
        beta_c = beta_c / g0
        beta_s = beta_s / g0
    return dict(n=n, alpha=alpha, beta_plus=0.5 * (beta_c + 1j * beta_s),
                beta_minus=0.5 * (beta_c - 1j * beta_s), beta_c=beta_c, beta_s=beta_s,
                g0=g0, mu=mu, a=a)


def rexi_scalar(x, co):
    """The two-sided sum at z = i x: an approximation of e^{ix}."""
    z = 1j * np.asarray(x, dtype=np.float64)[:, None]
    al = co["alpha"][None, :]
    return (co["beta_plus"][None, :] / (z + al)).sum(axis=1) + \
        (co["beta_minus"][None, :] / (al - z)).sum(axis=1)


def steps_to_error(eps: float, eps_T: float) -> float:
    """Number of steps N with (1 - eps)^N - 1 = -eps_T ... (Section 6.1).

    The paper writes N = log_{1+eps} |1 - eps_T|; this is that expression.
    """
    return math.log(abs(1.0 - eps_T)) / math.log(1.0 + eps)
