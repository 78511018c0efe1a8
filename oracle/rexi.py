"""One T-REXI time step in spherical-harmonic space, plain FP64.

Test infrastructure: see the package docstring.

Section 4.2: U_{n+1} ~ sum_k beta_k (dt L + alpha_k I)^{-1} U_n.  With the
two-sided coefficient list of ``oracle.coeffs`` (poles alpha_k used with +dt L
and with -dt L), one step is
    u1 = D^{-1} [ sum_k beta+_k (alpha_k I + dt L^)^{-1} + sum_k beta-_k (alpha_k I - dt L^)^{-1} ] D u0
for every zonal order m separately (the matrix is blocked by m, Section 5 /
Fig. 1), where L^ is the energy-scaled operator of ``oracle.operator`` and D
the scaling.  Every one of the 2N shifted systems is solved on its own by
LAPACK's banded LU with partial pivoting (scipy.linalg.solve_banded; the
interleaved (Phi, zeta, delta) ordering has 4 sub- and 4 super-diagonals), and
the weighted solutions are summed in pole order, + terms first, as the
"parallel reduce" of Algorithm 1 does.

The adjoint step is the conjugate transpose of that linear map:
    g0 = D [ sum_k conj(beta+_k) (conj(alpha_k) I + dt L^H)^{-1}
           + sum_k conj(beta-_k) (conj(alpha_k) I - dt L^H)^{-1} ] D^{-1} g1,
with L^H formed as the conjugate transpose of the assembled block.  For a real
loss of complex u1 the gradient dL/dRe + i dL/dIm obeys g0 = R^H g1.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from . import operator as op

KL = KU = 4


def _band(A: np.ndarray) -> np.ndarray:
    n = A.shape[0]
    ab = np.zeros((KL + KU + 1, n), dtype=np.complex128)
    for i in range(n):
        for j in range(max(0, i - KL), min(n, i + KU + 1)):
            ab[KU + i - j, j] = A[i, j]
    assert np.count_nonzero(A) == np.count_nonzero(
        [A[i, j] for i in range(n) for j in range(max(0, i - KL), min(n, i + KU + 1))])
    return ab


def _rexi_block(X, Aband, alphas, betas_plus, betas_minus):
    """sum_k beta+_k (alpha_k + A)^{-1} X + sum_k beta-_k (alpha_k - A)^{-1} X."""
    acc = np.zeros_like(X)
    for al, bp in zip(alphas, betas_plus):
        ab = Aband.copy()
        ab[KU] += al
        acc += bp * solve_banded((KL, KU), ab, X)
    for al, bm in zip(alphas, betas_minus):
        ab = -Aband
        ab[KU] += al
        acc += bm * solve_banded((KL, KU), ab, X)
    return acc


def rexi_step(u0, T, dt, co, a, omega, phibar, adjoint=False, orders=None, fsphere=None):
    """One forward (or adjoint) T-REXI step of states u0 [S][3][nspec].

    ``co`` is a coefficient dict from ``oracle.coeffs.rexi_coefficients``.
    ``orders`` restricts the work to the listed zonal orders (other orders
    are returned as zero); blocks whose input is exactly zero give zero.
    """
    u0 = np.asarray(u0, dtype=np.complex128)
    out = np.zeros_like(u0)
    ms = range(T + 1) if orders is None else orders
    alpha = co["alpha"]
    bp = co["beta_plus"]
    bm = co["beta_minus"]
    for m in ms:
        U = op.block_of(u0, T, m)
        if not np.any(U):
            continue
        Lh = op.scaled_block(T, m, a, omega, phibar, fsphere=fsphere)
        d = op.scaling_block(T, m, a, phibar)[:, None]
        if not adjoint:
            Y = _rexi_block(d * U, _band(dt * Lh), alpha, bp, bm) / d
        else:
            Y = d * _rexi_block(U / d, _band(dt * Lh.conj().T), np.conj(alpha), np.conj(bp), np.conj(bm))
        op.scatter_block(out, Y, T, m)
    return out


def rexi_run(u0, nsteps, T, dt, co, a, omega, phibar, adjoint=False, orders=None, fsphere=None):
    """Repeat the step ``nsteps`` times (the map is linear and time invariant)."""
    u = np.asarray(u0, dtype=np.complex128)
    for _ in range(nsteps):
        u = rexi_step(u, T, dt, co, a, omega, phibar, adjoint=adjoint, orders=orders, fsphere=fsphere)
    return u


def rexi_block_matrix(T, m, dt, co, a, omega, phibar, fsphere=None):
    """Dense matrix of the step restricted to order m, in physical units.

    R_m = D^{-1} [ sum_k beta+_k (alpha_k + dt L^)^{-1} + sum_k beta-_k (alpha_k - dt L^)^{-1} ] D,
    each shifted block inverted densely (numpy.linalg.inv).  Used for dense
    adjoints (R_m^H) and for building the propagator column by column.
    """
    Lh = op.scaled_block(T, m, a, omega, phibar, fsphere=fsphere)
    d = op.scaling_block(T, m, a, phibar)
    I = np.eye(Lh.shape[0])
    R = np.zeros_like(Lh)
    for al, bp in zip(co["alpha"], co["beta_plus"]):
        R += bp * np.linalg.inv(al * I + dt * Lh)
    for al, bm in zip(co["alpha"], co["beta_minus"]):
        R += bm * np.linalg.inv(al * I - dt * Lh)
    return (R / d[:, None]) * d[None, :]


def rexi_propagator(T, m, dt, co, a, omega, phibar, fsphere=None):
    """The step restricted to order m as a dense matrix, physical units: the
    banded solves of ``rexi_step`` applied to the identity (every column at once)."""
    Lh = op.scaled_block(T, m, a, omega, phibar, fsphere=fsphere)
    d = op.scaling_block(T, m, a, phibar)
    Rs = _rexi_block(np.eye(Lh.shape[0], dtype=np.complex128), _band(dt * Lh),
                     co["alpha"], co["beta_plus"], co["beta_minus"])
    return (Rs / d[:, None]) * d[None, :]


def dense_adjoint_run(g, nsteps, T, dt, co, a, omega, phibar):
    """g0 = (R^H)^nsteps g for every order m, with R_m^H = conj(R_m).T."""
    g = np.asarray(g, dtype=np.complex128)
    out = np.zeros_like(g)
    for m in range(T + 1):
        G = op.block_of(g, T, m)
        if not np.any(G):
            continue
        RH = rexi_block_matrix(T, m, dt, co, a, omega, phibar).conj().T
        for _ in range(nsteps):
            G = RH @ G
        op.scatter_block(out, G, T, m)
    return out
