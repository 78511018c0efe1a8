"""Physical-space diagnostics of spectral states (Eq. (1), Section 3).

``grid_fields(plan, u)`` returns the geopotential perturbation Phi and the
winds (u, v) of states [S][3][nspec] on the plan's Gaussian grid (SH synthesis
and the vector transform, both in the library's kernels).

``energy(plan, u)`` returns, per state, the area mean of the linear
shallow-water energy density, (1/2) (Phibar |V|^2 + Phi^2), integrated with
the Gauss weights in latitude and the trapezoid rule in longitude.  It is the
quantity the linear operator conserves (it is skew-Hermitian in the
energy-scaled variables).  For a state truncated at T on a grid with
nlat >= T + 1 and nlon > 2 T the quadrature is exact, and the value equals
(1/4) sum_{n,m} c_m [Phibar a^2 / (n(n+1)) (|zeta|^2 + |delta|^2) + |Phi|^2],
c_0 = 1, c_m = 2.  The final weighted sums are torch reductions on the GPU.

``spectral_energy(plan, u)`` is that sum itself, exact at any grid size; on a
grid with nlat < T + 1 (such as 512 x 256 at T256) the grid quadrature is not
exact for the top degrees, and ``energy`` then carries a bias for states with
much energy there.
"""
import numpy as np

from . import rexi


def _gauss_weights(nlat, device):
    import torch
    _, w = np.polynomial.legendre.leggauss(nlat)  # symmetric about the equator
    return torch.from_numpy(np.ascontiguousarray(w)).to(device)


def spectral_energy(plan: rexi.Plan, u):
    """(1/4) sum c_m [Phibar a^2/(n(n+1)) (|zeta|^2 + |delta|^2) + |Phi|^2] of
    each state u [S][3][nspec] (the same quantity as ``energy``, exactly)."""
    import torch
    p = plan.params
    phibar = p.gravity * p.mean_depth
    T = p.T
    n = np.concatenate([np.arange(m, T + 1) for m in range(T + 1)]).astype(float)
    cm = np.concatenate([np.full(T + 1 - m, 1.0 if m == 0 else 2.0) for m in range(T + 1)])
    s2 = np.where(n > 0, phibar * p.radius ** 2 / np.maximum(n * (n + 1), 1.0), 0.0)
    cm_t = torch.from_numpy(cm).to(u.device)
    s2_t = torch.from_numpy(s2).to(u.device)
    a2 = (u.real ** 2 + u.imag ** 2)  # [S][3][nspec]
    return 0.25 * ((a2[:, 0] + s2_t * (a2[:, 1] + a2[:, 2])) * cm_t).sum(-1)


def grid_fields(plan: rexi.Plan, u):
    """(Phi [S][nlat][nlon], winds [S][2][nlat][nlon]) of states u [S][3][nspec]."""
    phi = plan.sh_inverse(u[:, 0].contiguous())
    winds = plan.vortdiv_to_uv(u)
    return phi, winds


def energy(plan: rexi.Plan, u):
    """Area-mean energy (1/2) <Phibar |V|^2 + Phi^2> of each state (m^4 s^-4)."""
    p = plan.params
    phibar = p.gravity * p.mean_depth
    phi, winds = grid_fields(plan, u)
    dens = 0.5 * (phibar * (winds * winds).sum(1) + phi * phi)  # [S][nlat][nlon]
    w = _gauss_weights(p.nlat, u.device)
    # (1/4 pi) int f dOmega = sum_j w_j (1/nlon) sum_k f_jk / 2
    return (dens.sum(-1) * w).sum(-1) / (2.0 * p.nlon)
