"""Seeded synthetic inputs for the T-REXI shallow-water hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
none of the method's arithmetic: no transforms, no operator, no REXI
coefficients.  It only draws random spectral states, writes down the initial
conditions the paper prints in closed form, and names the workloads.

Spectral layout (the same for every producer of states): complex128 arrays of
shape [S][3][nspec] with the variables ordered (Phi, vort, div) and the
triangular coefficient list ordered m-major, ``idx(m, n) = m(T+1) - m(m-1)/2 +
(n - m)`` for ``0 <= m <= n <= T``; ``nspec = (T+1)(T+2)/2``.  Only m >= 0 is
stored; m = 0 coefficients describe real fields.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

# Physical constants of the numerical tests (Section 6, first paragraph).
EARTH_RADIUS = 6.37122e6      # m
EARTH_OMEGA = 7.292e-5        # 1/s
GRAVITY = 9.80616             # m/s^2
MEAN_DEPTH = 1.0e4            # m


@dataclass(frozen=True)
class Workload:
    """One named workload: truncation, grid, time step, REXI size, batch."""
    name: str
    T: int
    nlat: int
    nlon: int
    dt: float
    M: int
    h: float = 0.2
    L: int = 11
    states: int = 1
    steps: int = 1
    checkpoint_every: int = 0
    kind: str = "random"          # "random" | "jet" | "bumps"

    def as_dict(self):
        return asdict(self)


# The five workloads the hot path is specified on.  They share the Earth
# constants above; h = 0.2 and a rational basis half-width of 11 throughout.
WORKLOADS = {
    "t63_single": Workload("t63_single", 63, 64, 128, 3600.0, 64, states=1, steps=1),
    "t63_jet": Workload("t63_jet", 63, 64, 128, 7200.0, 128, states=1, steps=24, kind="jet"),
    "t128_batched": Workload("t128_batched", 128, 128, 256, 3600.0, 256, states=8, steps=1),
    "t128_adjoint": Workload("t128_adjoint", 128, 128, 256, 1800.0, 192, states=1, steps=48,
                             checkpoint_every=8),
    "t256_fwd_adj": Workload("t256_fwd_adj", 256, 256, 512, 10800.0, 1024, states=4, steps=16,
                             checkpoint_every=4),
}


# The propagating Gaussian bumps of Section 6.2 over 1.5 days (129600 s) at the
# paper's T128 (degrees n <= 127), with the T-REXI settings of its timing study
# (Section 6.4): 800 s steps with M = 512, 1600 s steps with M = 1024, and one
# 1.5-day step with M = 4096.  Fields at rest with the bump height.
BUMP_WORKLOADS = {
    "t127_bumps_dt800": Workload("t127_bumps_dt800", 127, 128, 256, 800.0, 512, steps=162, kind="bumps"),
    "t127_bumps_dt1600": Workload("t127_bumps_dt1600", 127, 128, 256, 1600.0, 1024, steps=81, kind="bumps"),
    "t127_bumps_1step": Workload("t127_bumps_1step", 127, 128, 256, 129600.0, 4096, steps=1, kind="bumps"),
}


# Numerical dispersion analysis (Section 6.3): T16, steps of at most 400 s, on
# the f-sphere (Section 4.3).  The paper does not print f0 or M; f0 = 2 Omega
# (the pole value) and M = 32 (h M = 6.4 covers dt sqrt(f0^2 + w_16^2) = 0.33)
# are this build's choice.
DISPERSION_WORKLOAD = Workload("t16_fsphere_dispersion", 16, 0, 0, 400.0, 32)
FSPHERE_F0 = 2.0 * EARTH_OMEGA


def nspec(T: int) -> int:
    return (T + 1) * (T + 2) // 2


def _degrees_orders(T: int):
    """Arrays n[i], m[i] for the m-major triangular list."""
    ms, ns = [], []
    for m in range(T + 1):
        for n in range(m, T + 1):
            ms.append(m)
            ns.append(n)
    return np.array(ns, dtype=np.int64), np.array(ms, dtype=np.int64)


# Amplitudes of the random states: a geopotential of 1e3 m^2/s^2 and a
# vorticity / divergence of 1e-5 1/s at the largest scale, both decaying as
# (n+1)^-2, so that the three variables carry comparable energy.
PHI_AMPLITUDE = 1.0e3
VORTDIV_AMPLITUDE = 1.0e-5


def random_state(T: int, states: int, seed: int) -> np.ndarray:
    """Seeded random spectral states, shape [states][3][nspec], complex128.

    Each coefficient is amplitude * (n+1)^-2 * z with z = (x + i y)/sqrt(2),
    x, y standard normal, drawn from numpy's PCG64 generator seeded with
    ``seed``: state by state, variable by variable (Phi, vort, div), all real
    parts of a variable first, then all imaginary parts.  m = 0 coefficients
    are made real, and the (n=0, m=0) vorticity and divergence are zero (the
    mean of a Laplacian vanishes on the sphere).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ns, ms = _degrees_orders(T)
    K = len(ns)
    decay = 1.0 / (ns + 1.0) ** 2
    amp = (PHI_AMPLITUDE, VORTDIV_AMPLITUDE, VORTDIV_AMPLITUDE)
    out = np.zeros((states, 3, K), dtype=np.complex128)
    for s in range(states):
        for v in range(3):
            x = rng.standard_normal(K)
            y = rng.standard_normal(K)
            z = (x + 1j * y) / math.sqrt(2.0)
            z[ms == 0] = z[ms == 0].real
            out[s, v] = amp[v] * decay * z
        out[s, 1, 0] = 0.0
        out[s, 2, 0] = 0.0
    return out


def random_grid(nlat: int, nlon: int, fields: int, seed: int) -> np.ndarray:
    """Seeded standard-normal grid-point fields, shape [fields][nlat][nlon]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((fields, nlat, nlon))


# Linearised geostrophic balance (Section 6.1): u = u0 cos(lat), v = 0,
# Phi = g H + u0 a Omega cos^2(lat).  The workload uses u0 = 20 m/s.
JET_U0 = 20.0


def jet_grid(mu: np.ndarray, nlon: int, u0: float = JET_U0, a: float = EARTH_RADIUS,
             omega: float = EARTH_OMEGA, g: float = GRAVITY, H: float = MEAN_DEPTH):
    """Grid-point (Phi, vort, div, u, v) of the balanced zonal jet.

    ``mu`` are the sines of the grid latitudes.  The vorticity of u = u0 cos(lat)
    is 2 u0 sin(lat) / a and its divergence is zero.
    """
    mu = np.asarray(mu, dtype=np.float64)
    cos2 = 1.0 - mu * mu
    one = np.ones((len(mu), nlon))
    phi = (g * H + u0 * a * omega * cos2)[:, None] * one
    vort = (2.0 * u0 * mu / a)[:, None] * one
    div = np.zeros_like(one)
    u = (u0 * np.sqrt(cos2))[:, None] * one
    v = np.zeros_like(one)
    return phi, vort, div, u, v


def jet_state(T: int, u0: float = JET_U0, a: float = EARTH_RADIUS, omega: float = EARTH_OMEGA,
              g: float = GRAVITY, H: float = MEAN_DEPTH) -> np.ndarray:
    """Closed-form spectral coefficients of the balanced jet, shape [1][3][nspec].

    With the basis orthonormal on [-1, 1] (P_0^0 = 1/sqrt2, P_1^0 = sqrt(3/2) mu,
    P_2^0 = sqrt(5/2) (3 mu^2 - 1)/2):  mu = sqrt(2/3) P_1^0, 1 = sqrt2 P_0^0 and
    1 - mu^2 = (2/3) sqrt2 P_0^0 - (2/3) sqrt(2/5) P_2^0.
    """
    assert T >= 2
    out = np.zeros((1, 3, nspec(T)), dtype=np.complex128)
    c = u0 * a * omega
    out[0, 0, 0] = math.sqrt(2.0) * (g * H + (2.0 / 3.0) * c)          # (n=0, m=0)
    out[0, 0, 2] = -(2.0 / 3.0) * math.sqrt(2.0 / 5.0) * c              # (n=2, m=0)
    out[0, 1, 1] = (2.0 * u0 / a) * math.sqrt(2.0 / 3.0)                # (n=1, m=0)
    return out


def bump_height(mu: np.ndarray, nlon: int, H: float = MEAN_DEPTH) -> np.ndarray:
    """Height field of three Gaussian bumps (Section 6.2) on the grid, [nlat][nlon].

    psi(lam, phi; lam_c, phi_c, p) = exp(-d^2 p) * 0.1 H, with d the great-circle
    angle to the bump centre; centres and widths as printed in Section 6.2.
    """
    phi = np.arcsin(np.asarray(mu, dtype=np.float64))[:, None]
    lam = (2.0 * np.pi * np.arange(nlon) / nlon)[None, :]
    out = np.full((len(mu), nlon), H)
    for lc, pc, p in ((0.2 * np.pi, np.pi / 3.0, 20.0), (1.2 * np.pi, -np.pi / 5.0, 80.0),
                      (1.6 * np.pi, -np.pi / 4.0, 360.0)):
        cosd = np.sin(pc) * np.sin(phi) + np.cos(pc) * np.cos(phi) * np.cos(lam - lc)
        d = np.arccos(np.clip(cosd, -1.0, 1.0))
        out = out + np.exp(-d * d * p) * 0.1 * H
    return out


def gauss_nodes(nlat: int) -> np.ndarray:
    """sin(latitude) of the nlat Gauss-Legendre grid rows, north to south
    (numpy's Gauss-Legendre nodes; the grid the inputs are sampled on)."""
    x, _ = np.polynomial.legendre.leggauss(nlat)
    return np.sort(x)[::-1].copy()


def bump_fields(nlat: int, nlon: int, g: float = GRAVITY, H: float = MEAN_DEPTH) -> np.ndarray:
    """Initial grid fields of the bump test, [3][nlat][nlon]: the geopotential
    perturbation g (h - H) of ``bump_height`` and zero vorticity and divergence
    (the fluid starts at rest)."""
    mu = gauss_nodes(nlat)
    out = np.zeros((3, nlat, nlon))
    out[0] = g * (bump_height(mu, nlon, H) - H)
    return out

