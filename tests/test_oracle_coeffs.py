"""Pins of the oracle's REXI coefficients (Section 4.1, Section 6.1)."""
import math

import numpy as np
import pytest

import synth
from oracle import coeffs
from tests.golden.read import load

PAPER = load("paper_section6.txt")
PHIBAR = synth.GRAVITY * synth.MEAN_DEPTH


def x_max(w):
    """Largest |frequency * dt| of the truncated operator, with margin.

    The gravity-wave frequency of the top degree is w_T = sqrt(Phibar T(T+1))/a;
    the spectral radius of the full operator exceeds it by less than 1e-3
    relative (checked in test_oracle_operator)."""
    return 1.001 * math.sqrt(PHIBAR * w.T * (w.T + 1)) / synth.EARTH_RADIUS * w.dt


def test_gaussian_fit_near_double_precision():
    # Section 4.1: K = 11 keeps the rational fit of the Gaussian close to double precision.
    K = int(PAPER["rational_half_width"])
    mu, a, err = coeffs.fit_gaussian(K)
    y = np.linspace(-150.0, 150.0, 60001)
    exact = np.exp(-y * y / 4.0) / math.sqrt(4.0 * math.pi)
    got = coeffs.gaussian_rational(y, mu, a)
    assert np.max(np.abs(got - exact)) < 1e-12
    assert mu < 0.0
    assert np.allclose(a[::-1], np.conj(a), rtol=0, atol=0)


def test_gaussian_sum_weights_reproduce_oscillation_with_exact_gaussians():
    # b_m = e^{h^2} e^{-imh}: with exact Gaussians psi_h the sum reproduces
    # e^{ix} (Poisson summation), away from the ends of [-hM, hM].
    h, M = 0.2, 64
    b = coeffs.gaussian_sum_weights(M, h)
    x = np.linspace(-h * (M - 14), h * (M - 14), 2001)
    m = np.arange(-M, M + 1)
    psi = np.exp(-((x[:, None] + m[None, :] * h) ** 2) / (4 * h * h)) / math.sqrt(4 * math.pi)
    approx = (psi * b[None, :]).sum(axis=1)
    assert np.max(np.abs(approx - np.exp(1j * x))) < 1e-13
    # A wrong sign of the phase fails by O(1).
    approx_wrong = (psi * np.conj(b)[None, :]).sum(axis=1)
    assert np.max(np.abs(approx_wrong - np.exp(1j * x))) > 0.5


@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_two_sided_rexi_matches_exponential_over_the_spectrum(name):
    w = synth.WORKLOADS[name]
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    assert len(co["alpha"]) == 2 * (w.M + w.L) + 1
    xm = x_max(w)
    assert xm < w.h * w.M
    x = np.linspace(-xm, xm, 6001)
    err = np.max(np.abs(coeffs.rexi_scalar(x, co) - np.exp(1j * x)))
    # t63_single spans 11.25+0.5 of hM = 12.8: the Gaussian sum is cut near its end.
    bound = 2e-9 if name == "t63_single" else 6e-12
    assert err < bound, err


def test_one_sided_merge_fails():
    # Merging the cos- and sin-coefficient lists without the mirrored poles
    # (a one-sided sum over the same N poles) is wrong by O(1e-2) or worse:
    # only the two-sided form reproduces e^{ix}.
    co = coeffs.rexi_coefficients(128, 0.2)
    x = np.linspace(-20, 20, 2001)
    one_sided = ((co["beta_c"] + 1j * co["beta_s"])[None, :] / (1j * x[:, None] + co["alpha"][None, :])).sum(1)
    assert np.max(np.abs(one_sided - np.exp(1j * x))) > 1e-2


def test_renormalisation_makes_zero_frequency_exact():
    # Section 6.1: before renormalisation sum beta/alpha misses 1 by a small
    # residual (the paper prints -1.56e-11 for M = 128 with Haut's
    # coefficients); after it the x = 0 response is 1.
    co_raw = coeffs.rexi_coefficients(128, 0.2, normalize=False)
    eps = 1.0 - co_raw["g0"].real
    assert 1e-13 < abs(eps) < 1e-10
    assert abs(math.log10(abs(eps)) - math.log10(abs(PAPER["epsilon_M128"]))) < 1.5
    assert abs(co_raw["g0"].imag) < 1e-14
    co = coeffs.rexi_coefficients(128, 0.2, normalize=True)
    g = coeffs.rexi_scalar(np.array([0.0]), co)[0]
    assert abs(g - 1.0) < 1e-14


def test_error_growth_estimate_arithmetic():
    # Section 6.1: with eps = 1.559e-11, about 60000 steps reach 1e-6.
    n = abs(coeffs.steps_to_error(abs(PAPER["epsilon_M128"]), 1e-6))
    assert abs(n - PAPER["steps_to_1e-6"]) / PAPER["steps_to_1e-6"] < 0.1
    # and (1 - eps)^N - 1 at that N is the target error
    assert abs((1 - abs(PAPER["epsilon_M128"])) ** n - 1 + 1e-6) < 1e-9


def test_coefficient_conjugate_symmetry():
    co = coeffs.rexi_coefficients(64, 0.2)
    n = co["n"]
    assert np.all(n == -n[::-1])
    assert np.allclose(co["alpha"][::-1], np.conj(co["alpha"]), rtol=0, atol=1e-15)
    for key in ("beta_plus", "beta_minus"):
        b = co[key]
        assert np.max(np.abs(b[::-1] - np.conj(b))) < 1e-14 * np.max(np.abs(b))
