"""f-sphere dispersion (Sections 4.3 and 6.3) on the oracle: the T-REXI step
matrix has eigenvalues exp(i dt nu) with nu the exact f-sphere frequencies."""
import numpy as np

import synth
from oracle import coeffs, rexi as orexi

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH


def test_oracle_step_reproduces_the_f_sphere_frequencies():
    w = synth.DISPERSION_WORKLOAD
    f0 = synth.FSPHERE_F0
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    worst = 0.0
    for m in (0, 1, 7, 16):
        E = orexi.rexi_propagator(w.T, m, w.dt, co, A, OM, PB, fsphere=f0)
        nu = np.sort(np.log(np.linalg.eigvals(E)).imag / w.dt)
        # closed form: per degree 0 and +-sqrt(f0^2 + Phibar n(n+1)/a^2); n = 0 has none
        ex = []
        for n in range(m, w.T + 1):
            if n == 0:
                ex += [0.0, 0.0, 0.0]
            else:
                s = np.sqrt(f0 ** 2 + PB * n * (n + 1) / A ** 2)
                ex += [-s, 0.0, s]
        ex = np.sort(ex)
        scale = np.max(np.abs(ex))
        worst = max(worst, np.max(np.abs(nu - ex)) / scale)
        # no growth or decay beyond the REXI error
        assert np.max(np.abs(np.abs(np.linalg.eigvals(E)) - 1.0)) < 1e-10
    assert worst < 1e-9, worst
