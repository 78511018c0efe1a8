"""The Gaussian-bump workload (Section 6.2) on the oracle: coverage of the
spectrum by the REXI sum, and the 1.5-day step against the exact exponential."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import coeffs, operator as op, rexi as orexi, sh as osh

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH


@pytest.mark.parametrize("name", list(synth.BUMP_WORKLOADS))
def test_rexi_covers_the_bump_spectrum(name):
    # every frequency of the T127 operator, |x| <= dt omega_T, lies inside the
    # covered range [-hM, hM] and is reproduced to the fit accuracy
    w = synth.BUMP_WORKLOADS[name]
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    xm = np.sqrt(PB * w.T * (w.T + 1)) / A * w.dt
    assert xm < w.h * w.M
    x = np.linspace(-xm, xm, 8001)
    assert np.max(np.abs(coeffs.rexi_scalar(x, co) - np.exp(1j * x))) < 5e-12


def test_grid_nodes_are_the_gauss_latitudes():
    mu, _ = osh.gauss_latitudes(128)
    assert np.max(np.abs(mu - synth.gauss_nodes(128))) < 1e-15


def test_one_step_of_one_and_a_half_days_matches_the_exponential():
    # one T-REXI step of 129600 s with M = 4096 against expm(dt L) of the
    # assembled block, on the bump state (Section 6.2 / 6.4)
    w = synth.BUMP_WORKLOADS["t127_bumps_1step"]
    u0 = osh.analysis(synth.bump_fields(w.nlat, w.nlon), w.T)[None]
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    for m in (20, 64, 100, 127):
        got = op.block_of(orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, orders=[m]), w.T, m)
        Lh = op.scaled_block(w.T, m, A, OM, PB)
        d = op.scaling_block(w.T, m, A, PB)[:, None]
        want = (expm(w.dt * Lh) @ (d * op.block_of(u0, w.T, m))) / d
        assert np.linalg.norm(got - want) <= 5e-11 * np.linalg.norm(want), m


def test_propagator_is_the_step():
    # rexi_propagator(m) applied to a state equals rexi_step on that order
    w = synth.Workload("p", T=24, nlat=0, nlon=0, dt=1800.0, M=32)
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    u0 = synth.random_state(w.T, 1, 7)
    for m in (0, 5, 24):
        R = orexi.rexi_propagator(w.T, m, w.dt, co, A, OM, PB)
        want = op.block_of(orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, orders=[m]), w.T, m)
        got = R @ op.block_of(u0, w.T, m)
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
