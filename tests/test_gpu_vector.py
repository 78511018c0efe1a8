"""GPU parity of the vector transforms sh_vortdiv_to_uv / sh_uv_to_vortdiv with the oracle."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import sh as osh

pytestmark = pytest.mark.gpu
A = synth.EARTH_RADIUS


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


def _plan(T, nlat, nlon, max_fields):
    import paper_1812_03431_amd as rexi
    w = synth.Workload("vec", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    return rexi.plan_for(w, max_fields=max_fields)


def _relmax(got, want):
    return np.max(np.abs(got - want)) / np.max(np.abs(want))


# the bump grid (T127, 256 x 128) and the benchmark grid (T256, 512 x 256)
# among them; B pairs need 2 B <= max_fields
@pytest.mark.parametrize("T,nlat,nlon,B", [(15, 16, 32, 1), (63, 64, 128, 3), (40, 44, 128, 5),
                                           (127, 128, 256, 2), (256, 256, 512, 6), (20, 22, 64, 17),
                                           (300, 320, 1024, 2), (1, 2, 4, 1)])
def test_vector_transforms_match_oracle(T, nlat, nlon, B):
    import torch
    dev = torch.device("cuda:0")
    plan = _plan(T, nlat, nlon, 2 * B)
    vd = synth.random_state(T, B, 11 + T)[:, 1:]
    uv = plan.vortdiv_to_uv(torch.from_numpy(np.ascontiguousarray(vd)).to(dev)).cpu().numpy()
    want = osh.vortdiv_to_uv(vd, T, nlat, nlon, A)
    assert _relmax(uv, want) < 1e-11
    winds = synth.random_grid(nlat, nlon, 2 * B, 7 + T).reshape(B, 2, nlat, nlon)
    got = plan.uv_to_vortdiv(torch.from_numpy(winds).to(dev)).cpu().numpy()
    want_vd = osh.uv_to_vortdiv(winds, T, A)
    assert _relmax(got, want_vd) < 1e-11


def test_balanced_jet_winds():
    # Section 6.1: the balanced jet's vorticity gives u = u0 cos(lat), v = 0
    import torch
    dev = torch.device("cuda:0")
    T, nlat, nlon = 63, 64, 128
    plan = _plan(T, nlat, nlon, 2)
    st = torch.from_numpy(synth.jet_state(T)).to(dev)
    uv = plan.vortdiv_to_uv(st).cpu().numpy()
    _, _, _, u, v = synth.jet_grid(synth.gauss_nodes(nlat), nlon)
    assert np.max(np.abs(uv[0, 0] - u)) < 1e-12 * synth.JET_U0
    assert np.max(np.abs(uv[0, 1] - v)) < 1e-12 * synth.JET_U0


def test_round_trip_and_state_layout():
    import torch
    dev = torch.device("cuda:0")
    T, nlat, nlon, S = 63, 64, 128, 3
    plan = _plan(T, nlat, nlon, 2 * S)
    st = torch.from_numpy(synth.random_state(T, S, 21)).to(dev)
    uv_state = plan.vortdiv_to_uv(st)
    uv_pairs = plan.vortdiv_to_uv(st[:, 1:].contiguous())
    assert torch.equal(uv_state, uv_pairs)
    # back into a state tensor: Phi is left alone, zeta and delta come back
    out = torch.full_like(st, 7.0 + 3.0j)
    plan.uv_to_vortdiv(uv_state, out=out)
    assert torch.all(out[:, 0] == 7.0 + 3.0j)
    back = out[:, 1:].cpu().numpy()
    want = st[:, 1:].cpu().numpy()
    assert _relmax(back, want) < 1e-12


def test_vector_argument_errors():
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    T, nlat, nlon = 15, 16, 32
    plan = _plan(T, nlat, nlon, 2)
    ns = plan.nspec
    vd = torch.zeros((2, 2, ns), dtype=torch.complex128, device=dev)
    with pytest.raises(rexi.RexiError, match="max_fields"):
        plan.vortdiv_to_uv(vd)
    uv = torch.zeros((1, 2, nlat, nlon), dtype=torch.float64, device=dev)
    lib, h = plan._lib, plan._h
    with pytest.raises(rexi.RexiError, match="stride"):
        rexi.rexi._check(lib.sh_vortdiv_to_uv(h, ctypes.c_void_p(vd.data_ptr()), 2 * ns - 1,
                                              ctypes.c_void_p(uv.data_ptr()), 1, None), "sh_vortdiv_to_uv")
    # output spectral pair overlapping the input winds
    buf = torch.zeros(2 * nlat * nlon + 4 * ns, dtype=torch.float64, device=dev)
    with pytest.raises(rexi.RexiError, match="overlaps"):
        rexi.rexi._check(lib.sh_uv_to_vortdiv(h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr() + 8),
                                              2 * ns, 1, None), "sh_uv_to_vortdiv")
    one = _plan(T, nlat, nlon, 1)
    with pytest.raises(rexi.RexiError, match="max_fields"):
        one.vortdiv_to_uv(vd[:1])


def test_vector_round_trip_at_the_largest_grid():
    # T1023 on 4096 x 2048 (degree 1024 inside the transforms): the winds of a
    # T-truncated state give the state back exactly, as nlat >= T + 1
    import torch
    dev = torch.device("cuda:0")
    T, nlat, nlon = 1023, 2048, 4096
    plan = _plan(T, nlat, nlon, 2)
    vd = torch.from_numpy(np.ascontiguousarray(synth.random_state(T, 1, 5)[:, 1:])).to(dev)
    back = plan.uv_to_vortdiv(plan.vortdiv_to_uv(vd))
    err = (back - vd).abs().max().item() / vd.abs().max().item()
    assert err < 1e-11, err
