"""GPU: physical-space energy of states against its spectral value and across a REXI step."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
A, PB = synth.EARTH_RADIUS, synth.GRAVITY * synth.MEAN_DEPTH


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


def _spectral_energy(u, T):
    """(1/4) sum c_m [Phibar a^2/(n(n+1)) (|zeta|^2 + |delta|^2) + |Phi|^2]."""
    n = np.array([n for m in range(T + 1) for n in range(m, T + 1)], dtype=float)
    cm = np.array([1.0 if m == 0 else 2.0 for m in range(T + 1) for n in range(m, T + 1)])
    s2 = np.where(n > 0, PB * A * A / np.maximum(n * (n + 1), 1), 0.0)
    return 0.25 * (np.abs(u[:, 0]) ** 2 * cm).sum(-1) + 0.25 * ((np.abs(u[:, 1]) ** 2 + np.abs(u[:, 2]) ** 2) * cm * s2).sum(-1)


def test_energy_matches_spectral_value_and_is_kept_by_the_step():
    import torch
    import paper_1812_03431_amd as rexi
    from paper_1812_03431_amd import diagnostics
    dev = torch.device("cuda:0")
    T, S = 63, 3
    w = synth.Workload("energy", T=T, nlat=64, nlon=128, dt=3600.0, M=128, states=S)
    plan = rexi.plan_for(w)
    u0 = synth.random_state(T, S, 77)
    ut = torch.from_numpy(u0).to(dev)
    e0 = diagnostics.energy(plan, ut).cpu().numpy()
    want = _spectral_energy(u0, T)
    assert np.max(np.abs(e0 - want) / want) < 1e-12
    assert np.max(np.abs(diagnostics.spectral_energy(plan, ut).cpu().numpy() - want) / want) < 1e-14
    # the linear operator conserves it; one REXI step changes it by its error only
    e1 = diagnostics.energy(plan, plan.step(ut)).cpu().numpy()
    assert np.max(np.abs(e1 / e0 - 1)) < 1e-10
    # the balanced jet's energy: Phi of the jet and u = u0 cos(lat)
    phi, winds = diagnostics.grid_fields(plan, torch.from_numpy(synth.jet_state(T)).to(dev))
    _, _, _, u, v = synth.jet_grid(synth.gauss_nodes(64), 128)
    assert np.max(np.abs(winds[0, 0].cpu().numpy() - u)) < 1e-12 * synth.JET_U0
