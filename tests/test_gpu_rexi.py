"""GPU parity of rexi_step / rexi_step_adjoint / rexi_step_per_term with the oracle."""
import numpy as np
import pytest

import synth
from oracle import rexi as orexi
from tests.gpu_common import A, OM, PB, TOL, assert_parity, block_mask, oracle_coeffs, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


def _plan(w, **kw):
    import paper_1812_03431_amd as rexi
    return rexi.plan_for(w, **kw)


def _gpu(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _oracle_step(u0, w, nsteps=1, adjoint=False, orders=None, normalize=True):
    co = oracle_coeffs(w.M, w.h, w.L, normalize)
    return orexi.rexi_run(u0, nsteps, w.T, w.dt, co, A, OM, PB, adjoint=adjoint, orders=orders)


def test_step_t63_every_schedule(torch_dev):
    w = synth.WORKLOADS["t63_single"]
    u0 = synth.random_state(w.T, 1, 0)
    want = _oracle_step(u0, w)
    plan = _plan(w, grid=False)
    n = plan.schedule_count(1)
    assert n >= 3
    for i in range(n):
        plan.set_schedule(1, i)
        print(f"  schedule {i}", flush=True)
        got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got, want, what=f"t63 schedule {i}")


@pytest.mark.parametrize("T,S,M,dt", [(40, 3, 32, 3600.0), (7, 5, 16, 7200.0), (1, 2, 8, 1800.0),
                                      (33, 4, 48, 10800.0)])
def test_step_ragged_and_partial_tiles(torch_dev, T, S, M, dt):
    w = synth.Workload("ragged", T=T, nlat=0, nlon=0, dt=dt, M=M, states=S)
    u0 = synth.random_state(T, S, 100 + T)
    want = _oracle_step(u0, w)
    plan = _plan(w, grid=False)
    for i in range(plan.schedule_count(S)):
        plan.set_schedule(S, i)
        got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got, want, what=f"T{T} S{S} schedule {i}")
    got = plan.step_per_term(_gpu(u0, torch_dev)).cpu().numpy()
    assert_parity(got, want, what=f"T{T} S{S} per-term")


@pytest.mark.parametrize("T,S,M,dt,orders", [
    (160, 2, 32, 600.0, [0, 1, 31, 32, 33, 63, 95, 96, 97, 159, 160]),
    (255, 1, 24, 300.0, [0, 1, 2, 64, 126, 127, 128, 191, 254, 255]),
])
def test_step_long_chains_every_schedule(torch_dev, T, S, M, dt, orders):
    # chains of up to 255 elements: 32-lane groups over row pairs and the
    # 12/16-element row tilings, for every policy, both directions
    w = synth.Workload("long", T=T, nlat=0, nlon=0, dt=dt, M=M, states=S)
    u0 = synth.random_state(T, S, 200 + T)
    mask = block_mask(T, orders)
    want = _oracle_step(u0, w, orders=orders)
    want_a = _oracle_step(u0, w, adjoint=True, orders=orders)
    plan = _plan(w, grid=False)
    for i in range(plan.schedule_count(S)):
        plan.set_schedule(S, i)
        print(f"  schedule {i}", flush=True)
        got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got[:, :, mask], want[:, :, mask], what=f"T{T} schedule {i}")
        got_a = plan.step_adjoint(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got_a[:, :, mask], want_a[:, :, mask], what=f"T{T} adjoint schedule {i}")
    got = plan.step_per_term(_gpu(u0, torch_dev)).cpu().numpy()
    assert_parity(got[:, :, mask], want[:, :, mask], what=f"T{T} per-term")


def test_step_chains_beyond_256_elements(torch_dev):
    # T400: chains of up to 400 elements run 16 elements per lane over 32
    # lanes with ds_bpermute moves, under every policy
    T, S, M, dt = 400, 1, 16, 120.0
    orders = [0, 1, 143, 144, 145, 399, 400]
    w = synth.Workload("vlong", T=T, nlat=0, nlon=0, dt=dt, M=M, states=S)
    u0 = synth.random_state(T, S, 400)
    mask = block_mask(T, orders)
    want = _oracle_step(u0, w, orders=orders)
    want_a = _oracle_step(u0, w, adjoint=True, orders=orders)
    plan = _plan(w, grid=False)
    for i in range(plan.schedule_count(S)):
        plan.set_schedule(S, i)
        print(f"  schedule {i}", flush=True)
        got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got[:, :, mask], want[:, :, mask], what=f"T{T} schedule {i}")
        got_a = plan.step_adjoint(_gpu(u0, torch_dev)).cpu().numpy()
        assert_parity(got_a[:, :, mask], want_a[:, :, mask], what=f"T{T} adjoint schedule {i}")


def test_step_at_the_largest_truncation(torch_dev):
    # T1023, the largest truncation a plan accepts: chains of up to 1023
    # elements over 64 lanes of 16 elements (ds_bpermute moves), forward and
    # adjoint on sampled orders.  dt = 60 s keeps dt * omega_T near 3, inside
    # h M = 6.4.
    T, S, M, dt = 1023, 1, 32, 60.0
    orders = [0, 1, 2, 511, 1021, 1022, 1023]
    w = synth.Workload("tmax", T=T, nlat=0, nlon=0, dt=dt, M=M, states=S)
    u0 = synth.random_state(T, S, 1023)
    mask = block_mask(T, orders)
    plan = _plan(w, grid=False)
    got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
    want = _oracle_step(u0, w, orders=orders)
    assert_parity(got[:, :, mask], want[:, :, mask], what="T1023")
    got_a = plan.step_adjoint(_gpu(u0, torch_dev)).cpu().numpy()
    want_a = _oracle_step(u0, w, adjoint=True, orders=orders)
    assert_parity(got_a[:, :, mask], want_a[:, :, mask], what="T1023 adjoint")


def test_zero_steps_copy_the_state(torch_dev):
    w = synth.Workload("zero", T=20, nlat=0, nlon=0, dt=3600.0, M=16, states=2)
    plan = _plan(w, grid=False)
    u0 = _gpu(synth.random_state(w.T, 2, 5), torch_dev)
    assert np.array_equal(plan.step(u0, nsteps=0).cpu().numpy(), u0.cpu().numpy())
    assert np.array_equal(plan.step_adjoint(u0, nsteps=0).cpu().numpy(), u0.cpu().numpy())


def test_multistep_and_adjoint(torch_dev):
    w = synth.Workload("ms", T=20, nlat=0, nlon=0, dt=3600.0, M=64, states=2)
    u0 = synth.random_state(w.T, 2, 7)
    plan = _plan(w, grid=False)
    got = plan.step(_gpu(u0, torch_dev), nsteps=5).cpu().numpy()
    assert_parity(got, _oracle_step(u0, w, 5), what="5 steps")
    got = plan.step_adjoint(_gpu(u0, torch_dev), nsteps=3).cpu().numpy()
    assert_parity(got, _oracle_step(u0, w, 3, adjoint=True), what="3 adjoint steps")
    # nsteps = 0 copies
    got = plan.step(_gpu(u0, torch_dev), nsteps=0).cpu().numpy()
    assert np.array_equal(got, u0)


def test_adjoint_dot_product_on_gpu(torch_dev):
    w = synth.Workload("dot", T=31, nlat=0, nlon=0, dt=1800.0, M=192, states=2)
    x = synth.random_state(w.T, 2, 1)
    y = synth.random_state(w.T, 2, 2)
    plan = _plan(w, grid=False)
    Rx = plan.step(_gpu(x, torch_dev), nsteps=2).cpu().numpy()
    RHy = plan.step_adjoint(_gpu(y, torch_dev), nsteps=2).cpu().numpy()
    lhs, rhs = np.vdot(y, Rx), np.vdot(RHy, x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_balanced_jet_steady_for_24_steps(torch_dev):
    w = synth.WORKLOADS["t63_jet"]
    u0 = synth.jet_state(w.T)
    plan = _plan(w, grid=False)
    got = plan.step(_gpu(u0, torch_dev), nsteps=w.steps).cpu().numpy()
    assert np.linalg.norm(got - u0) / np.linalg.norm(u0) < 1e-12
    # the non-constant part of the jet (vorticity, Phi at n = 2) is kept too
    for v, i in ((1, 1), (0, 2)):
        assert abs(got[0, v, i] - u0[0, v, i]) <= 1e-12 * abs(u0[0, v, i])
    want = _oracle_step(u0, w, w.steps, orders=[0])
    # Phi and vorticity: relative; divergence is exactly zero, so bound it by
    # the vorticity scale (same units) instead of its own norm.
    assert rel_err(got[0, 0], want[0, 0]) < 1e-12 and rel_err(got[0, 1], want[0, 1]) < 1e-12
    assert np.linalg.norm(got[0, 2] - want[0, 2]) <= 1e-12 * np.linalg.norm(u0[0, 1])


def test_determinism(torch_dev):
    w = synth.Workload("det", T=47, nlat=0, nlon=0, dt=3600.0, M=64, states=2)
    u0 = _gpu(synth.random_state(w.T, 2, 3), torch_dev)
    plan = _plan(w, grid=False)
    a = plan.step(u0).cpu().numpy()
    b = plan.step(u0).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name,orders,seed", [
    ("t128_batched", [0, 1, 2, 63, 64, 65, 127, 128], 0),
    ("t256_fwd_adj", [0, 1, 2, 127, 128, 129, 200, 255, 256], 0),
])
def test_full_size_forward_sampled_orders(torch_dev, name, orders, seed):
    w = synth.WORKLOADS[name]
    u0 = synth.random_state(w.T, w.states, seed)
    plan = _plan(w, grid=False)
    got = plan.step(_gpu(u0, torch_dev)).cpu().numpy()
    assert np.all(np.isfinite(got))
    mask = block_mask(w.T, orders)
    want = _oracle_step(u0, w, orders=orders)
    assert_parity(got[:, :, mask], want[:, :, mask], what=f"{name} orders {orders}")
    got_a = plan.step_adjoint(_gpu(u0, torch_dev)).cpu().numpy()
    want_a = _oracle_step(u0, w, adjoint=True, orders=orders)
    assert_parity(got_a[:, :, mask], want_a[:, :, mask], what=f"{name} adjoint orders {orders}")


def test_t128_adjoint_48_steps_sampled_orders(torch_dev):
    w = synth.WORKLOADS["t128_adjoint"]
    g = synth.random_state(w.T, 1, 100)
    plan = _plan(w, grid=False)
    got = plan.step_adjoint(_gpu(g, torch_dev), nsteps=w.steps).cpu().numpy()
    orders = [0, 64, 128]
    mask = block_mask(w.T, orders)
    want = _oracle_step(g, w, w.steps, adjoint=True, orders=orders)
    assert_parity(got[:, :, mask], want[:, :, mask], what="t128 adjoint 48 steps")


def test_argument_errors(torch_dev):
    import torch
    import paper_1812_03431_amd as rexi
    w = synth.Workload("err", T=8, nlat=0, nlon=0, dt=3600.0, M=8, states=2)
    plan = _plan(w, grid=False)
    u = torch.zeros((3, 3, plan.nspec), dtype=torch.complex128, device=torch_dev)
    with pytest.raises(rexi.RexiError, match="max_states"):
        plan.step(u)
    u = torch.zeros((2, 3, plan.nspec), dtype=torch.complex128, device=torch_dev)
    with pytest.raises(rexi.RexiError, match="overlaps"):
        plan.step(u, out=u)
    with pytest.raises(rexi.RexiError, match="without a grid"):
        rexi.rexi._check(plan._lib.sh_forward(plan._h, None, None, 1, None), "sh_forward")


def test_graph_replays_match_direct_launches(torch_dev):
    import torch
    w = synth.Workload("graph", T=47, nlat=0, nlon=0, dt=3600.0, M=64, states=2)
    plan = _plan(w, grid=False)
    u0 = _gpu(synth.random_state(w.T, 2, 9), torch_dev)
    plan.set_graphs(False)
    want = plan.step(u0, nsteps=3).cpu().numpy()
    want_a = plan.step_adjoint(u0, nsteps=2).cpu().numpy()
    plan.set_graphs(True)
    for rep in range(4):
        got = plan.step(u0, nsteps=3)
        torch.cuda.synchronize()
        scratch = (u0 * 2).sum()           # eager work between the replays
        assert np.array_equal(got.cpu().numpy(), want), rep
        got_a = plan.step_adjoint(u0, nsteps=2).cpu().numpy()
        assert np.array_equal(got_a, want_a), rep
        del scratch


def test_persistent_and_regular_schedules_agree(torch_dev):
    w = synth.WORKLOADS["t128_batched"]
    plan = _plan(w, grid=False)
    u0 = _gpu(synth.random_state(w.T, w.states, 0), torch_dev)
    n = plan.schedule_count(w.states)
    assert n % 2 == 0
    ref = None
    for i in (0, 2, n // 2, n // 2 + 2):    # regular and persistent variants of two policies
        plan.set_schedule(w.states, i)
        got = plan.step(u0).cpu().numpy()
        if ref is None:
            ref = got
        else:
            assert rel_err(got, ref) < 1e-13


def test_concurrent_and_serial_class_launches_agree(torch_dev):
    # every tile class writes its own partials, so running the classes on
    # side streams must give the serial result bit for bit, directly and
    # replayed from graphs
    import torch
    w = synth.WORKLOADS["t128_batched"]
    plan = _plan(w, grid=False)
    u0 = _gpu(synth.random_state(w.T, w.states, 3), torch_dev)
    plan.set_graphs(False)
    plan.set_streams(False)
    ref = plan.step(u0, nsteps=2).cpu().numpy()
    ref_a = plan.step_adjoint(u0).cpu().numpy()
    plan.set_streams(True)
    for graphs in (False, True):
        plan.set_graphs(graphs)
        for rep in range(3):
            assert np.array_equal(plan.step(u0, nsteps=2).cpu().numpy(), ref), (graphs, rep)
            torch.cuda.synchronize()
            assert np.array_equal(plan.step_adjoint(u0).cpu().numpy(), ref_a), (graphs, rep)

