"""Numerical dispersion analysis of the T-REXI step (Section 6.3).

The step matrix E (U_{n+1} = E U_n) is built column by column: every spectral
unknown (variable, n, m) is switched on alone and stepped once with
``rexi_step`` on the GPU, in batches of the plan's ``max_states``.  E is block
diagonal in the zonal order m.  The logarithm of each eigenvalue of a block,
divided by i dt, is a numerical frequency; on the f-sphere the exact ones per
(n, m) are 0 and +-sqrt(f0^2 + Phibar n(n+1)/a^2) (all zero at n = 0).  Only
the eigen-decomposition of the small blocks runs on the host; the steps run in
the library's kernels.
"""
from __future__ import annotations

import numpy as np


def _index(T: int, m: int, n: int) -> int:
    return m * (T + 1) - m * (m - 1) // 2 + (n - m)


def step_matrix_blocks(plan, T: int, device):
    """{m: E_m} with E_m the (3L x 3L) block of the step for order m, unknowns
    ordered (Phi, vort, div) per degree n = m..T, in physical units."""
    import torch
    S = plan.params.max_states
    ns = plan.nspec
    blocks = {}
    for m in range(T + 1):
        idx = [(v, _index(T, m, n)) for n in range(m, T + 1) for v in range(3)]
        K = len(idx)
        E = np.zeros((K, K), dtype=np.complex128)
        rows_v = torch.tensor([v for v, _ in idx], device=device)
        rows_i = torch.tensor([i for _, i in idx], device=device)
        for c0 in range(0, K, S):
            chunk = idx[c0:c0 + S]
            U = torch.zeros((len(chunk), 3, ns), dtype=torch.complex128, device=device)
            for s, (v, i) in enumerate(chunk):
                U[s, v, i] = 1.0
            Y = plan.step(U)
            E[:, c0:c0 + len(chunk)] = Y[:, rows_v, rows_i].T.cpu().numpy()
        blocks[m] = E
    return blocks


def exact_frequencies(T: int, m: int, f0: float, phibar: float, a: float) -> np.ndarray:
    """Sorted exact frequencies of the f-sphere block of order m."""
    out = []
    for n in range(m, T + 1):
        if n == 0:
            out += [0.0, 0.0, 0.0]
            continue
        w = np.sqrt(f0 * f0 + phibar * n * (n + 1.0) / (a * a))
        out += [-w, 0.0, w]
    return np.sort(np.array(out))


def analyse(plan, T: int, dt: float, f0: float, phibar: float, a: float, device):
    """Numerical vs exact frequencies of every mode.

    Returns a dict: per-mode arrays ``m``, ``exact``, ``numerical`` (rad/s,
    matched by sorting within each block), ``growth`` (Re log(lambda)/dt, 1/s),
    and the summary ``max_rel_phase_error`` over the non-zero modes and
    ``max_abs_zero_mode`` (|frequency| of the geostrophic modes, rad/s)."""
    blocks = step_matrix_blocks(plan, T, device)
    ms, ex, nu, gr = [], [], [], []
    for m, E in blocks.items():
        lam = np.linalg.eigvals(E)
        lg = np.log(lam)
        order = np.argsort(lg.imag)
        ms += [m] * len(lam)
        ex.append(exact_frequencies(T, m, f0, phibar, a))
        nu.append(lg.imag[order] / dt)
        gr.append(lg.real[order] / dt)
    ex, nu, gr = np.concatenate(ex), np.concatenate(nu), np.concatenate(gr)
    nz = ex != 0.0
    return {
        "m": np.array(ms), "exact": ex, "numerical": nu, "growth": gr,
        "max_rel_phase_error": float(np.max(np.abs(nu[nz] - ex[nz]) / np.abs(ex[nz]))),
        "max_abs_zero_mode": float(np.max(np.abs(nu[~nz]))) if np.any(~nz) else 0.0,
        "max_abs_growth": float(np.max(np.abs(gr))),
    }
