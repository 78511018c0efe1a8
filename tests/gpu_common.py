"""Shared helpers of the GPU tests (inputs from synth, expectations from the oracle)."""
import functools
import multiprocessing
import os

import numpy as np

import synth
from oracle import coeffs
from oracle import rexi as orexi

A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH
TOL = 1e-10      # relative L2 per variable and state, FP64


@functools.lru_cache(maxsize=16)
def oracle_coeffs(M, h, L=11, normalize=True):
    return coeffs.rexi_coefficients(M, h, L, normalize=normalize)


def rel_err(got, want):
    d = np.linalg.norm(want)
    return np.linalg.norm(got - want) / (d if d > 0 else 1.0)


def order_slice(T, m):
    o = m * (T + 1) - m * (m - 1) // 2
    return slice(o, o + T + 1 - m)


def block_mask(T, orders):
    """Boolean mask over the m-major spectral list selecting the given orders."""
    mask = np.zeros(synth.nspec(T), dtype=bool)
    for m in orders:
        mask[order_slice(T, m)] = True
    return mask


def parity_errors(got, want, T, orders=None):
    """Relative L2 errors of got against want, [S][3][nspec] each.

    Returns (worst over (state, variable) of the error over the selected
    orders, worst over (state, variable, order) of the error within one
    order's block).  A block whose expected values are all zero is measured
    against the norm of its variable over the selected orders instead."""
    ms = range(T + 1) if orders is None else orders
    mask = block_mask(T, ms)
    worst_var, worst_blk = 0.0, 0.0
    for s in range(want.shape[0]):
        for v in range(3):
            g, w = got[s, v], want[s, v]
            scale = np.linalg.norm(w[mask])
            worst_var = max(worst_var, np.linalg.norm(g[mask] - w[mask]) / (scale if scale > 0 else 1.0))
            for m in ms:
                sl = order_slice(T, m)
                d = np.linalg.norm(w[sl])
                den = d if d > 0 else (scale if scale > 0 else 1.0)
                worst_blk = max(worst_blk, np.linalg.norm(g[sl] - w[sl]) / den)
    return worst_var, worst_blk


def assert_parity(got, want, T, orders=None, tol=TOL, what="", blocks=True):
    """got matches want to ``tol`` relative L2 per (state, variable) over the
    selected orders (all if None) and, with ``blocks``, per (state, variable,
    order) within each order's block, so that an error confined to the small
    high-order blocks cannot hide behind the large low-order ones.  (Without
    ``blocks`` only where the two sides start from inputs that differ by
    rounding, e.g. two independent transforms of one grid: a block far below
    the variable's norm then carries that input difference, not a step error.)"""
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    ms = list(range(T + 1) if orders is None else orders)
    mask = block_mask(T, ms)
    for s in range(want.shape[0]):
        for v in range(3):
            g, w = got[s, v], want[s, v]
            scale = np.linalg.norm(w[mask])
            e = np.linalg.norm(g[mask] - w[mask]) / (scale if scale > 0 else 1.0)
            assert e <= tol, f"{what}: state {s} variable {v}: rel L2 {e:.3e} > {tol:.0e}"
            for m in (ms if blocks else ()):
                sl = order_slice(T, m)
                d = np.linalg.norm(w[sl])
                den = d if d > 0 else (scale if scale > 0 else 1.0)
                e = np.linalg.norm(g[sl] - w[sl]) / den
                assert e <= tol, f"{what}: state {s} variable {v} order {m}: block rel L2 {e:.3e} > {tol:.0e}"


# ---------------------------------------------------------------- oracle pool
def _oracle_orders(args):
    u0, nsteps, T, dt, co, adjoint, orders = args
    return orexi.rexi_run(u0, nsteps, T, dt, co, A, OM, PB, adjoint=adjoint, orders=orders)


def oracle_workers():
    """Worker processes for the oracle: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_run_parallel(u0, w, nsteps=1, adjoint=False, orders=None, workers=None):
    """The oracle's nsteps-step run of states u0 [S][3][nspec] for workload w
    on the listed orders (all if None), the orders spread over worker
    processes.  Every order is its own independent block (the operator is
    block diagonal in m), so each block's arithmetic is the oracle's own,
    unchanged; the blocks are only computed in different processes.
    Workers are started with 'spawn' (a forked child of a process that has
    initialised the GPU must not touch it; these never import torch)."""
    T = w.T
    ms = list(range(T + 1) if orders is None else orders)
    ms.sort()                                   # longest chains (small m) first
    n = workers or oracle_workers()
    chunks = [ms[i::n] for i in range(n) if ms[i::n]]
    co = oracle_coeffs(w.M, w.h, w.L)       # fitted once here, passed to the workers
    jobs = [(u0, nsteps, T, w.dt, co, adjoint, c) for c in chunks]
    if len(jobs) == 1:
        return _oracle_orders(jobs[0])
    ctx = multiprocessing.get_context("spawn")
    # one BLAS thread per worker: the workers already use every CPU given
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        with ctx.Pool(len(jobs)) as pool:
            parts = pool.map(_oracle_orders, jobs, chunksize=1)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out = np.zeros_like(np.asarray(u0, dtype=np.complex128))
    for c, part in zip(chunks, parts):
        for m in c:
            sl = order_slice(T, m)
            out[..., sl] = part[..., sl]
    return out
