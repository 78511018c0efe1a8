"""The f-sphere variant on the GPU (Section 4.3) and the dispersion analysis
built on it (Section 6.3), against the oracle."""
import numpy as np
import pytest

import synth
from oracle import rexi as orexi
from tests.gpu_common import A, OM, PB, assert_parity, oracle_coeffs, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


def _plan(w, S, f0):
    import paper_1812_03431_amd as rexi
    return rexi.plan_for(w, max_states=S, grid=False, fsphere=f0)


def test_fsphere_steps_match_oracle():
    import torch
    dev = torch.device("cuda:0")
    f0 = synth.FSPHERE_F0
    w = synth.Workload("fs", T=40, nlat=0, nlon=0, dt=3600.0, M=64, states=3)
    u0 = synth.random_state(w.T, 3, 11)
    co = oracle_coeffs(w.M, w.h, w.L)
    plan = _plan(w, 3, f0)
    got = plan.step(torch.from_numpy(u0).to(dev)).cpu().numpy()
    want = orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, fsphere=f0)
    assert_parity(got, want, w.T, what="f-sphere forward")
    got_a = plan.step_adjoint(torch.from_numpy(u0).to(dev)).cpu().numpy()
    want_a = orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, adjoint=True, fsphere=f0)
    assert_parity(got_a, want_a, w.T, what="f-sphere adjoint")


def test_fsphere_adjoint_dot_product_and_multistep():
    import torch
    dev = torch.device("cuda:0")
    w = synth.Workload("fs", T=20, nlat=0, nlon=0, dt=7200.0, M=48, states=2)
    plan = _plan(w, 2, synth.FSPHERE_F0)
    u = torch.from_numpy(synth.random_state(w.T, 2, 1)).to(dev)
    g = torch.from_numpy(synth.random_state(w.T, 2, 2)).to(dev)
    lhs = torch.vdot(g.flatten(), plan.step(u).flatten()).item()
    rhs = torch.vdot(plan.step_adjoint(g).flatten(), u.flatten()).item()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    three = plan.step(u, 3).cpu().numpy()
    one = plan.step(plan.step(plan.step(u))).cpu().numpy()
    assert np.array_equal(three, one)
    assert np.array_equal(plan.step(u, 0).cpu().numpy(), u.cpu().numpy())


def test_fsphere_plan_rejects_schedule_calls():
    import torch
    import paper_1812_03431_amd as rexi
    w = synth.Workload("fs", T=8, nlat=0, nlon=0, dt=3600.0, M=8, states=1)
    plan = _plan(w, 1, synth.FSPHERE_F0)
    with pytest.raises(rexi.RexiError, match="f-sphere"):
        plan.autotune(1)
    u = torch.zeros((1, 3, plan.nspec), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(rexi.RexiError, match="f-sphere"):
        plan.step_per_term(u)


def test_dispersion_matrix_and_frequencies():
    import torch
    from paper_1812_03431_amd import dispersion
    dev = torch.device("cuda:0")
    w = synth.DISPERSION_WORKLOAD
    f0 = synth.FSPHERE_F0
    plan = _plan(w, 64, f0)
    blocks = dispersion.step_matrix_blocks(plan, w.T, dev)
    co = oracle_coeffs(w.M, w.h, w.L)
    for m in (0, 1, 9, 16):
        want = orexi.rexi_propagator(w.T, m, w.dt, co, A, OM, PB, fsphere=f0)
        assert rel_err(blocks[m], want) < 1e-10, m
    res = dispersion.analyse(plan, w.T, w.dt, f0, PB, A, dev)
    assert res["max_rel_phase_error"] < 1e-9
    assert res["max_abs_zero_mode"] < 1e-12
    assert res["max_abs_growth"] < 1e-12
