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


@pytest.mark.parametrize("T,nlat,nlon,B", [(300, 320, 1024, 3), (1, 2, 4, 1), (3, 4, 8, 2)])
def test_transforms_match_oracle_more_grids(T, nlat, nlon, B):
    # 160 northern latitudes: the forward kernel's two-block path; and the
    # smallest grids the plan accepts
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    w = synth.Workload("sh", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=2 * B)
    grid = synth.random_grid(nlat, nlon, B, T + 1)
    got = plan.sh_forward(torch.from_numpy(grid).to(dev)).cpu().numpy()
    want = osh.analysis(grid, T)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-12
    spec = synth.random_state(T, B, T + 2)[:, 0]
    got_g = plan.sh_inverse(torch.from_numpy(np.ascontiguousarray(spec)).to(dev)).cpu().numpy()
    want_g = osh.synthesis(spec, T, nlat, nlon)
    assert np.max(np.abs(got_g - want_g)) / np.max(np.abs(want_g)) < 1e-12


def test_round_trip_at_the_largest_grid():
    # T1023 on 4096 x 2048: sh_forward(sh_inverse(s)) = s exactly (n < nlat,
    # m < nlon/2), on the largest sizes the plan accepts
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    T, nlat, nlon = 1023, 2048, 4096
    w = synth.Workload("max", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=2)
    u = torch.from_numpy(synth.random_state(T, 1, 9).reshape(3, -1)[:2].copy()).to(dev)
    g = plan.sh_inverse(u)
    back = plan.sh_forward(g)
    err = (back - u).abs().max().item() / u.abs().max().item()
    assert err < 1e-11, err


def test_round_trip_many_fields_at_t1023():
    # T1023 on 2048 x 1024 with 16 fields (32 real columns): the workspace
    # planes are a power of two apart before padding, 512 row pairs fill the
    # XCD-ordered FFT blocks, and every order has up to 8 partial slots
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    T, nlat, nlon, B = 1023, 1024, 2048, 16
    w = synth.Workload("big", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=B)
    u = torch.from_numpy(synth.random_state(T, 6, 11).reshape(18, -1)[:B].copy()).to(dev)
    g = plan.sh_inverse(u)
    back = plan.sh_forward(g)
    err = ((back - u).abs().amax(1) / u.abs().amax(1)).max().item()
    assert err < 1e-11, err
    # a second call of the same plan with fewer fields (one column tile)
    u3 = u[:3].contiguous()
    back3 = plan.sh_forward(plan.sh_inverse(u3))
    err3 = ((back3 - u3).abs().amax(1) / u3.abs().amax(1)).max().item()
    assert err3 < 1e-11, err3


def _random_shapes(n, seed=2024):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        nlon = int(2 ** rng.integers(2, 11))          # 4 .. 1024
        T = int(rng.integers(1, min(nlon - 1, 200) + 1))
        nlat = int(2 * rng.integers(1, 151))           # 2 .. 300, even
        B = int(rng.integers(1, 21))
        out.append((T, nlat, nlon, B))
    return out


@pytest.mark.parametrize("T,nlat,nlon,B", _random_shapes(16))
def test_transforms_random_shapes(T, nlat, nlon, B):
    # scalar and vector transforms on seeded random shapes (T above or below
    # nlat, ragged column chunks) against the oracle
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    w = synth.Workload("rnd", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=2 * B)
    grid = synth.random_grid(nlat, nlon, B, T + nlat)
    got = plan.sh_forward(torch.from_numpy(grid).to(dev)).cpu().numpy()
    want = osh.analysis(grid, T)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-12
    spec = synth.random_state(T, B, T + nlon)[:, 0]
    got_g = plan.sh_inverse(torch.from_numpy(np.ascontiguousarray(spec)).to(dev)).cpu().numpy()
    want_g = osh.synthesis(spec, T, nlat, nlon)
    assert np.max(np.abs(got_g - want_g)) / np.max(np.abs(want_g)) < 1e-12
    vd = synth.random_state(T, B, T + 7)[:, 1:]
    uv = plan.vortdiv_to_uv(torch.from_numpy(np.ascontiguousarray(vd)).to(dev)).cpu().numpy()
    want_uv = osh.vortdiv_to_uv(vd, T, nlat, nlon, synth.EARTH_RADIUS)
    assert np.max(np.abs(uv - want_uv)) / np.max(np.abs(want_uv)) < 1e-11
    winds = synth.random_grid(nlat, nlon, 2 * B, T + 9).reshape(B, 2, nlat, nlon)
    got_vd = plan.uv_to_vortdiv(torch.from_numpy(winds).to(dev)).cpu().numpy()
    want_vd = osh.uv_to_vortdiv(winds, T, synth.EARTH_RADIUS)
    assert np.max(np.abs(got_vd - want_vd)) / np.max(np.abs(want_vd)) < 1e-11
