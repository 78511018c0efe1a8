"""Linear SWE operator in spherical-harmonic space, plain FP64 (Section 2, Eq. (1)).

Test infrastructure: see the package docstring.

Eq. (1), with f = 2 Omega mu and mu = sin(lat):
    zeta_t  = -f delta - V . grad f
    delta_t =  f zeta + k . (grad f x V) - lap Phi
    Phi_t   = -Phibar delta
Writing U = u cos(lat) = (1/a)[chi_lam - (1-mu^2) psi_mu] and
V = v cos(lat) = (1/a)[psi_lam + (1-mu^2) chi_mu] (zeta = lap psi, delta = lap chi),
the Coriolis terms become -(2 Omega/a) V and -(2 Omega/a) U.  In the
orthonormal basis P_n^m(mu) e^{i m lam} (Section 3) the identities
    mu P_n^m             = eps_{n+1} P_{n+1}^m + eps_n P_{n-1}^m,
    (1-mu^2) dP_n^m/dmu  = -n eps_{n+1} P_{n+1}^m + (n+1) eps_n P_{n-1}^m,
    lap Y_n^m            = -n(n+1)/a^2 Y_n^m,           eps_n = sqrt((n^2-m^2)/(4n^2-1)),
give, coefficient by coefficient at fixed m (the operator is block diagonal in m):
    Phi_t(n)   = -Phibar delta_n
    zeta_t(n)  = i theta_n zeta_n - 2 Omega [ (n+1)/n eps_n delta_{n-1} + n/(n+1) eps_{n+1} delta_{n+1} ]
    delta_t(n) = i theta_n delta_n + 2 Omega [ (n+1)/n eps_n zeta_{n-1} + n/(n+1) eps_{n+1} zeta_{n+1} ]
                 + n(n+1)/a^2 Phi_n
with theta_n = 2 Omega m / (n(n+1)).  The sign of i theta follows from the
e^{+i m lam} convention of Section 3 (Rossby-Haurwitz waves move west).

Energy scaling: zeta^ = s_n zeta, delta^ = s_n delta, Phi^ = Phi with
s_n = a sqrt(Phibar / (n(n+1))).  In these variables the operator L^ is
skew-Hermitian:
    Phi^_t(n)   = -w_n delta^_n,                      w_n = sqrt(Phibar n(n+1))/a
    zeta^_t(n)  =  i theta zeta^_n - 2 Omega (k_n delta^_{n-1} + k_{n+1} delta^_{n+1})
    delta^_t(n) =  i theta delta^_n + 2 Omega (k_n zeta^_{n-1} + k_{n+1} zeta^_{n+1}) + w_n Phi^_n
with k_n = eps_n sqrt(n^2-1)/n.  Truncation is Galerkin: couplings to n < m or
n > T are dropped.  The (n=0, m=0) mode is left unchanged by the operator (its
vorticity and divergence carry no flow and w_0 = 0); its scale is s_0 = 1.

Optional f-sphere variant (Section 4.3): a constant f0 replaces 2 Omega mu, so
grad f = 0 and the couplings become zeta_t = -f0 delta, delta_t = f0 zeta + ...;
its eigenvalues per n are 0 and +-i sqrt(f0^2 + w_n^2).

Block layout: unknowns interleaved by degree, (Phi_n, zeta_n, delta_n) for
n = m..T, i.e. position 3 (n - m) + v with v = 0, 1, 2.
"""
from __future__ import annotations

import math

import numpy as np


def eps(n: int, m: int) -> float:
    if n <= 0 or n < m:
        return 0.0
    return math.sqrt((n * n - m * m) / (4.0 * n * n - 1.0))


def scale(n: int, a: float, phibar: float) -> float:
    """s_n: vorticity/divergence multiplier to energy variables (1 at n = 0)."""
    if n == 0:
        return 1.0
    return a * math.sqrt(phibar / (n * (n + 1.0)))


def scaling_block(T: int, m: int, a: float, phibar: float) -> np.ndarray:
    """Diagonal of D for the block of order m, layout (Phi, zeta, delta) per n."""
    d = np.ones(3 * (T + 1 - m))
    for n in range(m, T + 1):
        s = scale(n, a, phibar)
        d[3 * (n - m) + 1] = s
        d[3 * (n - m) + 2] = s
    return d


def unscaled_block(T: int, m: int, a: float, omega: float, phibar: float) -> np.ndarray:
    """Dense operator block L_m in physical units (the formulas above)."""
    K = T + 1 - m
    A = np.zeros((3 * K, 3 * K), dtype=np.complex128)
    P, Z, D = 0, 1, 2

    def at(n, v):
        return 3 * (n - m) + v

    for n in range(m, T + 1):
        if n == 0:
            continue
        th = 2.0 * omega * m / (n * (n + 1.0))
        A[at(n, P), at(n, D)] = -phibar
        A[at(n, Z), at(n, Z)] = 1j * th
        A[at(n, D), at(n, D)] = 1j * th
        A[at(n, D), at(n, P)] = n * (n + 1.0) / (a * a)
        if n - 1 >= max(m, 1):
            cm = (n + 1.0) / n * eps(n, m)
            A[at(n, Z), at(n - 1, D)] = -2.0 * omega * cm
            A[at(n, D), at(n - 1, Z)] = 2.0 * omega * cm
        if n + 1 <= T:
            cp = n / (n + 1.0) * eps(n + 1, m)
            A[at(n, Z), at(n + 1, D)] = -2.0 * omega * cp
            A[at(n, D), at(n + 1, Z)] = 2.0 * omega * cp
    return A


def scaled_block(T: int, m: int, a: float, omega: float, phibar: float,
                 fsphere: float | None = None) -> np.ndarray:
    """Dense L^_m in energy variables (skew-Hermitian), written out directly."""
    K = T + 1 - m
    A = np.zeros((3 * K, 3 * K), dtype=np.complex128)
    P, Z, D = 0, 1, 2

    def at(n, v):
        return 3 * (n - m) + v

    for n in range(m, T + 1):
        if n == 0:
            continue
        w = math.sqrt(phibar * n * (n + 1.0)) / a
        A[at(n, P), at(n, D)] = -w
        A[at(n, D), at(n, P)] = w
        if fsphere is not None:
            A[at(n, Z), at(n, D)] = -fsphere
            A[at(n, D), at(n, Z)] = fsphere
            continue
        th = 2.0 * omega * m / (n * (n + 1.0))
        A[at(n, Z), at(n, Z)] = 1j * th
        A[at(n, D), at(n, D)] = 1j * th
        if n - 1 >= max(m, 1):
            k = eps(n, m) * math.sqrt(n * n - 1.0) / n
            A[at(n, Z), at(n - 1, D)] = -2.0 * omega * k
            A[at(n, D), at(n - 1, Z)] = 2.0 * omega * k
        if n + 1 <= T:
            k1 = eps(n + 1, m) * math.sqrt((n + 1.0) ** 2 - 1.0) / (n + 1.0)
            A[at(n, Z), at(n + 1, D)] = -2.0 * omega * k1
            A[at(n, D), at(n + 1, Z)] = 2.0 * omega * k1
    return A


def block_of(state: np.ndarray, T: int, m: int) -> np.ndarray:
    """Gather the (Phi, zeta, delta) interleaved block of order m.

    ``state`` has shape [S][3][nspec]; the result has shape [3(T+1-m)][S].
    """
    o = m * (T + 1) - m * (m - 1) // 2
    K = T + 1 - m
    S = state.shape[0]
    out = np.zeros((3 * K, S), dtype=np.complex128)
    for v in range(3):
        out[v::3, :] = state[:, v, o:o + K].T
    return out


def scatter_block(state: np.ndarray, blk: np.ndarray, T: int, m: int) -> None:
    o = m * (T + 1) - m * (m - 1) // 2
    K = T + 1 - m
    for v in range(3):
        state[:, v, o:o + K] = blk[v::3, :].T
