"""Shared helpers of the GPU tests (inputs from synth, expectations from the oracle)."""
import functools

import numpy as np

import synth
from oracle import coeffs

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH
TOL = 1e-10      # relative L2 per variable and state, FP64


@functools.lru_cache(maxsize=16)
def oracle_coeffs(M, h, L=11, normalize=True):
    return coeffs.rexi_coefficients(M, h, L, normalize=normalize)


def rel_err(got, want):
    d = np.linalg.norm(want)
    return np.linalg.norm(got - want) / (d if d > 0 else 1.0)


def assert_parity(got, want, tol=TOL, what=""):
    S = want.shape[0]
    for s in range(S):
        for v in range(3):
            e = rel_err(got[s, v], want[s, v])
            assert e <= tol, f"{what}: state {s} variable {v}: rel L2 {e:.3e} > {tol:.0e}"


def block_mask(T, orders):
    """Boolean mask over the m-major spectral list selecting the given orders."""
    mask = np.zeros(synth.nspec(T), dtype=bool)
    for m in orders:
        o = m * (T + 1) - m * (m - 1) // 2
        mask[o:o + T + 1 - m] = True
    return mask
