"""GPU parity of sh_forward / sh_inverse (FFT + FP64-MFMA Legendre) with the oracle."""
import numpy as np
import pytest

import synth
from oracle import sh as osh

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


@pytest.mark.parametrize("T,nlat,nlon,B", [(15, 16, 32, 2), (63, 64, 128, 3), (128, 128, 256, 6),
                                           (256, 256, 512, 12), (20, 22, 64, 1), (63, 64, 128, 40),
                                           (40, 44, 128, 13), (33, 36, 64, 9)])
def test_transforms_match_oracle(T, nlat, nlon, B):
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    w = synth.Workload("sh", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=B)
    grid = synth.random_grid(nlat, nlon, B, T)
    got = plan.sh_forward(torch.from_numpy(grid).to(dev)).cpu().numpy()
    want = osh.analysis(grid, T)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert err < 1e-12, f"sh_forward rel max err {err}"
    spec = synth.random_state(T, 1, T).reshape(3, -1)[:1].repeat(B, axis=0)
    got_g = plan.sh_inverse(torch.from_numpy(np.ascontiguousarray(spec)).to(dev)).cpu().numpy()
    want_g = osh.synthesis(spec, T, nlat, nlon)
    err = np.max(np.abs(got_g - want_g)) / np.max(np.abs(want_g))
    assert err < 1e-12, f"sh_inverse rel max err {err}"


def test_round_trip_on_gpu():
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    w = synth.Workload("rt", T=63, nlat=64, nlon=128, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=3)
    u = synth.random_state(63, 1, 5).reshape(3, -1)
    g = plan.sh_inverse(torch.from_numpy(u).to(dev))
    back = plan.sh_forward(g).cpu().numpy()
    assert np.max(np.abs(back - u)) / np.max(np.abs(u)) < 1e-13
