"""Differentiation through the hand-written adjoint (autograd.Function).

Loss = ||Phi(T) - Phi_target||^2 over the stored spectral coefficients after
48 steps (t128_adjoint workload), gradients with checkpoint segments of 8.
Checked against central finite differences (eps = 1e-6) on 32 seeded
directions, and against the oracle's dense adjoint at T31."""
import numpy as np
import pytest

import synth
from oracle import rexi as orexi
from tests.gpu_common import A, OM, PB, oracle_coeffs, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)


def _grad(plan, u0_np, target_np, nsteps, ck):
    import torch
    import paper_1812_03431_amd as rexi
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(u0_np).to(dev).requires_grad_(True)
    tgt = torch.from_numpy(target_np).to(dev)
    u = rexi.run(plan, u0, nsteps, checkpoint_every=ck)
    loss = (u[:, 0] - tgt).abs().pow(2).sum()
    loss.backward()
    return float(loss.detach()), u0.grad.detach().cpu().numpy()


def test_gradient_matches_central_differences_t128():
    import torch
    import paper_1812_03431_amd as rexi
    w = synth.WORKLOADS["t128_adjoint"]
    ndir = 32
    plan = rexi.plan_for(w, grid=False, max_states=2 * ndir)
    u0 = synth.random_state(w.T, 1, 0)
    target = synth.random_state(w.T, 1, 100)[:, 0].copy()
    _, g = _grad(plan, u0, target, w.steps, w.checkpoint_every)
    dirs = np.concatenate([synth.random_state(w.T, 1, 200 + i) for i in range(ndir)])
    an = np.array([np.real(np.vdot(g[0], d)) for d in dirs])
    # The loss is quadratic in u0 (the step is linear), so central differences
    # equal the directional derivative for every eps; what remains is
    # rounding.  Each loss carries the steps' own rounding, about 1e-13 of the
    # loss and different for u0 + eps d and u0 - eps d, so the difference
    # quotient errs by up to about 1e-13 / eps: 1e-7 at the workload's
    # eps = 1e-6 (measured 2.6e-8; bound 2e-7) and 1e-11 at eps = 1e-2
    # (measured 1.2e-12; bound 1e-9).
    for eps, bound in ((1e-6, 2e-7), (1e-2, 1e-9)):
        batch = np.concatenate([u0 + eps * dirs, u0 - eps * dirs])   # [2 ndir][3][nspec]
        with torch.no_grad():
            out = plan.step(torch.from_numpy(batch).cuda(), w.steps).cpu().numpy()
        loss = np.sum(np.abs(out[:, 0] - target) ** 2, axis=1)
        fd = (loss[:ndir] - loss[ndir:]) / (2 * eps)
        err = np.abs(fd - an) / np.maximum(np.abs(an), 1e-300)
        print(f"  eps {eps:.0e}: max rel error {np.max(err):.2e}", flush=True)
        assert np.max(err) < bound, (eps, err)


def test_gradient_matches_dense_adjoint_t31():
    import paper_1812_03431_amd as rexi
    w0 = synth.WORKLOADS["t128_adjoint"]
    w = synth.Workload("adj31", T=31, nlat=0, nlon=0, dt=w0.dt, M=w0.M, states=1)
    plan = rexi.plan_for(w, grid=False)
    u0 = synth.random_state(w.T, 1, 0)
    target = synth.random_state(w.T, 1, 100)[:, 0].copy()
    _, g = _grad(plan, u0, target, w0.steps, w0.checkpoint_every)
    from oracle import operator as op
    co = oracle_coeffs(w.M, w.h, w.L)
    # dense step matrices R_m of the oracle: u(T) = R^48 u0, grad = (R^H)^48 2 (Phi(T) - target)
    R = [orexi.rexi_block_matrix(w.T, m, w.dt, co, A, OM, PB) for m in range(w.T + 1)]
    uT = np.zeros_like(u0)
    for m in range(w.T + 1):
        X = op.block_of(u0, w.T, m)
        for _ in range(w0.steps):
            X = R[m] @ X
        op.scatter_block(uT, X, w.T, m)
    seed = np.zeros_like(uT)
    seed[:, 0] = 2.0 * (uT[:, 0] - target)
    want = np.zeros_like(seed)
    for m in range(w.T + 1):
        G = op.block_of(seed, w.T, m)
        for _ in range(w0.steps):
            G = R[m].conj().T @ G
        op.scatter_block(want, G, w.T, m)
    for v in range(3):
        assert rel_err(g[0, v], want[0, v]) < 1e-10, v


def test_checkpoint_segmentation_does_not_change_the_gradient():
    import paper_1812_03431_amd as rexi
    w = synth.Workload("seg", T=24, nlat=0, nlon=0, dt=1800.0, M=64, states=1)
    plan = rexi.plan_for(w, grid=False)
    u0 = synth.random_state(w.T, 1, 5)
    target = synth.random_state(w.T, 1, 6)[:, 0].copy()
    l1, g1 = _grad(plan, u0, target, 12, 0)
    l2, g2 = _grad(plan, u0, target, 12, 4)
    l3, g3 = _grad(plan, u0, target, 12, 5)
    assert abs(l1 - l2) <= 1e-13 * abs(l1) and abs(l1 - l3) <= 1e-13 * abs(l1)
    assert rel_err(g2, g1) < 1e-12 and rel_err(g3, g1) < 1e-12
