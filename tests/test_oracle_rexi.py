"""Pins of the oracle's T-REXI step (Sections 4.2, 5, 6.1)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import coeffs, operator as op, rexi

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH


def _expm_step(u, T, dt, adjoint=False):
    out = np.zeros_like(u)
    for m in range(T + 1):
        Lh = op.scaled_block(T, m, A, OM, PB)
        d = op.scaling_block(T, m, A, PB)[:, None]
        X = op.block_of(u, T, m)
        E = expm(dt * Lh)
        Y = (E @ (d * X)) / d if not adjoint else d * (E.conj().T @ (X / d))
        op.scatter_block(out, Y, T, m)
    return out


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dt,M", [(3600.0, 64), (7200.0, 128), (1800.0, 192), (10800.0, 1024)])
def test_step_matches_matrix_exponential(dt, M):
    T = 15
    co = coeffs.rexi_coefficients(M, 0.2)
    u0 = synth.random_state(T, 2, 1)
    got = rexi.rexi_step(u0, T, dt, co, A, OM, PB)
    want = _expm_step(u0, T, dt)
    for s in range(2):
        for v in range(3):
            assert _rel(got[s, v], want[s, v]) < 1e-11


def test_step_matches_at_the_edge_of_the_covered_spectrum():
    # t63_single: the top gravity wave sits at 11.25 of hM = 12.8.
    w = synth.WORKLOADS["t63_single"]
    co = coeffs.rexi_coefficients(w.M, w.h)
    u0 = synth.random_state(w.T, 1, 0)
    ms = [0, 1, 31, 62, 63]
    got = rexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, orders=ms)
    want = np.zeros_like(u0)
    for m in ms:
        Lh = op.scaled_block(w.T, m, A, OM, PB)
        d = op.scaling_block(w.T, m, A, PB)[:, None]
        op.scatter_block(want, (expm(w.dt * Lh) @ (d * op.block_of(u0, w.T, m))) / d, w.T, m)
    for v in range(3):
        assert _rel(got[0, v], want[0, v]) < 3e-9


def test_banded_lu_equals_dense_solves():
    T, dt = 10, 7200.0
    co = coeffs.rexi_coefficients(32, 0.2)
    u0 = synth.random_state(T, 1, 2)
    got = rexi.rexi_step(u0, T, dt, co, A, OM, PB)
    want = np.zeros_like(u0)
    for m in range(T + 1):
        X = op.block_of(u0, T, m)
        op.scatter_block(want, rexi.rexi_block_matrix(T, m, dt, co, A, OM, PB) @ X, T, m)
    assert _rel(got, want) < 1e-13


@pytest.mark.parametrize("normalize", [True, False])
def test_balanced_jet_stays_steady(normalize):
    # Section 6.1: with renormalised betas the geostrophic state is kept to
    # round-off over 24 long steps; without it the x = 0 residual of the REXI
    # sum accumulates step after step (the paper's finding).
    w = synth.WORKLOADS["t63_jet"]
    co = coeffs.rexi_coefficients(w.M, w.h, normalize=normalize)
    u0 = synth.jet_state(w.T)
    u = rexi.rexi_run(u0, w.steps, w.T, w.dt, co, A, OM, PB)
    change = np.linalg.norm(u - u0) / np.linalg.norm(u0)
    eps = abs(1 - coeffs.rexi_coefficients(w.M, w.h, normalize=False)["g0"].real)
    if normalize:
        assert change < 1e-12
    else:
        assert change > 1e-12
        assert abs(change - w.steps * eps) < 0.1 * w.steps * eps


def _energy(u, T):
    e = 0.0
    for m in range(T + 1):
        d = op.scaling_block(T, m, A, PB)[:, None]
        e += np.sum(np.abs(d * op.block_of(u, T, m)) ** 2)
    return e


def test_energy_preserved_to_rexi_accuracy():
    T, dt = 15, 7200.0
    co = coeffs.rexi_coefficients(128, 0.2)
    u0 = synth.random_state(T, 1, 7)
    u1 = rexi.rexi_step(u0, T, dt, co, A, OM, PB)
    e0, e1 = _energy(u0, T), _energy(u1, T)
    assert abs(e1 / e0 - 1) < 1e-11


def test_adjoint_dot_product():
    T, dt = 12, 3600.0
    co = coeffs.rexi_coefficients(64, 0.2)
    x = synth.random_state(T, 2, 20)
    y = synth.random_state(T, 2, 21)
    Rx = rexi.rexi_step(x, T, dt, co, A, OM, PB)
    RHy = rexi.rexi_step(y, T, dt, co, A, OM, PB, adjoint=True)
    assert abs(np.vdot(y, Rx) - np.vdot(RHy, x)) < 1e-13 * abs(np.vdot(y, Rx))


def test_adjoint_matches_exponential_adjoint_and_dense_adjoint():
    T, dt = 15, 1800.0
    co = coeffs.rexi_coefficients(192, 0.2)
    g = synth.random_state(T, 1, 30)
    got = rexi.rexi_step(g, T, dt, co, A, OM, PB, adjoint=True)
    assert _rel(got, _expm_step(g, T, dt, adjoint=True)) < 1e-11
    dense = rexi.dense_adjoint_run(g, 1, T, dt, co, A, OM, PB)
    assert _rel(got, dense) < 1e-13


def test_step_is_unitary_in_energy_variables_to_rexi_accuracy():
    T, dt, m = 15, 3600.0, 2
    co = coeffs.rexi_coefficients(64, 0.2)
    R = rexi.rexi_block_matrix(T, m, dt, co, A, OM, PB)
    d = op.scaling_block(T, m, A, PB)
    Rh = (R * d[:, None]) / d[None, :]
    assert np.max(np.abs(Rh.conj().T @ Rh - np.eye(len(d)))) < 1e-11
