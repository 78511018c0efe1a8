#!/usr/bin/env python3
"""Benchmark of the T-REXI hot path on one MI355X.

One "step" of this benchmark is the whole job of the T256 workload on one
batch of synthetic input, already resident in HBM:
  SH analysis of 4 states x (Phi, vort, div) from a 512x256 Gaussian grid,
  16 forward T-REXI steps (dt = 10800 s, M = 1024 -> 2071 poles) kept as
  segments of 4 (checkpoints at segment boundaries),
  the gradient of ||Phi(T) - Phi_target||^2,
  16 adjoint steps, and SH synthesis of the resulting gradient.
The metric is (pole, m)-block solves per second over the timed region:
2 x 16 x 2071 x 257 blocks per step.

Also reported: live HIP-event timing of the fused solve kernel (roofline
against the FP64 vector peak), the FP64-MFMA Legendre kernels, the plain
per-term launch form for comparison, the vector transforms, the energy drift
of the benchmark states over the 16 steps, the wall-clock of the Gaussian-bump
workload over 1.5 days (Section 6.2), the f-sphere dispersion errors of the
step (Section 6.3), the Legendre kernels at T1023 on a 2048 x 1024 grid with
16 fields (where the contraction is large; context, not the benchmark
workload), and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK = 78.6     # TFLOP/s, MI355X (256 CUs x 2.4 GHz x 128 FP64 flop/clk)
FP64_MFMA_PEAK = 78.6       # TFLOP/s, MI355X dense FP64 matrix
HBM_PEAK = 8000.0           # GB/s


def solve_flops_per_launch(N, T, S):
    """Algorithmic FP64 flops of one forward REXI step of S states, as the
    measurement contract counts them: nspec N (40 + 156 S), i.e. per pole and
    per (n, m) 40 flops of factorisation and 156 per state (both signs' right-
    hand sides, Phi elimination, sweeps and the weighted accumulation)."""
    nspec = (T + 1) * (T + 2) // 2
    return float(nspec) * N * (40 + 156 * S)


def solve_flops_thomas(N, T, S):
    """The same step by a plain Thomas count: per pole and per (n, m) !=
    (0, 0), both parity chains hold one element each; factorisation 2 x 16
    flops (diagonal, pivot update, complex reciprocal, multiplier) and per
    right-hand side (2 per state) 2 x 34 flops (Phi elimination, forward
    sweep, back substitution, weighted accumulation)."""
    nspec = (T + 1) * (T + 2) // 2
    return float(N) * (nspec - 1) * (32 + 136 * S)


def legendre_flops(T, nlat, fields):
    """Algorithmic flops of one Legendre contraction (either direction), using
    the equatorial symmetry: 2 x (nlat/2) x (2 fields) per coefficient."""
    nspec = (T + 1) * (T + 2) // 2
    return 2.0 * (nlat // 2) * (2 * fields) * nspec


def legendre_large_run(rexi, synth, torch, dev, reps=5):
    """HIP-event time of the Legendre kernels at T1023 on a 2048 x 1024 grid
    with 16 fields, where the contraction (17.2 GFLOP per call) is large
    enough that launch and load burst no longer weigh as much as the MFMA
    work.  A transform-only plan: the smallest REXI tables, one state."""
    T, nlat, nlon, B = 1023, 1024, 2048, 16
    w = synth.Workload("t1023_transforms", T=T, nlat=nlat, nlon=nlon, dt=3600.0, M=8, states=1)
    plan = rexi.plan_for(w, max_fields=B)
    grid = torch.from_numpy(synth.random_grid(nlat, nlon, B, 1)).to(dev)
    spec = plan.sh_forward(grid)
    back = plan.sh_inverse(spec)
    torch.cuda.synchronize()
    plan.set_timing(True)
    for _ in range(reps):
        plan.sh_forward(grid, out=spec)
        plan.sh_inverse(spec, out=back)
    torch.cuda.synchronize()
    plan.set_timing(False)
    f_ms, f_n = plan.kernel_time(plan.KERNEL_LEGENDRE_FWD)
    i_ms, i_n = plan.kernel_time(plan.KERNEL_LEGENDRE_INV)
    fl = legendre_flops(T, nlat, B)
    a_f = fl / (f_ms / 1e3 / f_n) / 1e12
    a_i = fl / (i_ms / 1e3 / i_n) / 1e12
    out = {"T": T, "grid": f"{nlon}x{nlat}", "fields": B, "flops_per_launch": fl, "unit": "TFLOP/s",
           "peak": FP64_MFMA_PEAK, "forward_avg_ms": round(f_ms / f_n, 4), "inverse_avg_ms": round(i_ms / i_n, 4),
           "forward_achieved": round(a_f, 3), "forward_frac": round(a_f / FP64_MFMA_PEAK, 4),
           "inverse_achieved": round(a_i, 3), "inverse_frac": round(a_i / FP64_MFMA_PEAK, 4),
           "note": "context: the same kernels where the contraction is large; not the benchmark workload"}
    del plan, grid, spec, back
    torch.cuda.empty_cache()
    return out


def kernel_source_digest():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1812_03431_amd", "csrc", "rexi_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_summary(name, digest, schedule_name=None):
    """A committed counter summary from profiles/, if it was taken on the
    current solve kernel source and, where a schedule is given, on that
    schedule (matched by name: indices move when the candidate list
    changes); otherwise None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != digest:
        return None
    if schedule_name is not None and d.get("schedule_name") != schedule_name:
        return None
    return d


def cpu_baseline(w, budget_s, gpu_fwd=None, gpu_adj=None):
    """The oracle, as is, on a bounded sample of the workload's orders.  When
    the GPU's step and adjoint of the same states are given, the oracle's
    results on the sampled orders double as an accuracy check of them."""
    import numpy as np
    import synth
    from oracle import coeffs, rexi as orexi
    A, OM, PB = synth.EARTH_RADIUS, synth.EARTH_OMEGA, synth.GRAVITY * synth.MEAN_DEPTH
    co = coeffs.rexi_coefficients(w.M, w.h, w.L)
    N = len(co["alpha"])
    u0 = synth.random_state(w.T, w.states, 0)
    stride = 8  # 33 of 257 orders at T256, about 15 s of oracle time on one core
    orders = list(range(0, w.T + 1, stride))
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    t0, c0 = time.perf_counter(), time.process_time()
    done = []
    fwd = np.zeros_like(u0)
    adj = np.zeros_like(u0)
    for m in orders:
        fwd += orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, orders=[m])
        adj += orexi.rexi_step(u0, w.T, w.dt, co, A, OM, PB, orders=[m], adjoint=True)
        done.append(m)
        if time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    blocks = 2 * N * len(done)
    out = {"value": blocks / wall, "unit": "blocks/s", "cores": max(1, round(cpu / wall)), "kind": "oracle",
           "cpu_count": os.cpu_count(), "cpus_allowed": affinity,
           "cores_note": "cores = CPU time / wall time of the sample (threads actually used); cpu_count = "
                         "os.cpu_count() of the host",
           "sample": f"one forward and one adjoint step of {w.states} states for orders m = "
                     f"{done[0]}..{done[-1]} step {stride} ({len(done)} of {w.T + 1} orders, mean chain "
                     f"length {np.mean([w.T + 1 - m for m in done]):.0f}); {wall:.1f} s wall"}
    if gpu_fwd is not None:
        mask = np.zeros(u0.shape[-1], dtype=bool)
        for m in done:
            o = m * (w.T + 1) - m * (m - 1) // 2
            mask[o:o + w.T + 1 - m] = True

        def worst(got, want):
            var = max(float(np.linalg.norm(got[s, v, mask] - want[s, v, mask]) / np.linalg.norm(want[s, v, mask]))
                      for s in range(u0.shape[0]) for v in range(3))
            blk = 0.0
            for s in range(u0.shape[0]):
                for v in range(3):
                    for m in done:
                        o = m * (w.T + 1) - m * (m - 1) // 2
                        sl = slice(o, o + w.T + 1 - m)
                        d = np.linalg.norm(want[s, v, sl])
                        if d > 0:
                            blk = max(blk, float(np.linalg.norm(got[s, v, sl] - want[s, v, sl]) / d))
            return var, blk
        fv, fb = worst(gpu_fwd, fwd)
        av, ab = worst(gpu_adj, adj)
        ok = max(fv, fb, av, ab) <= 1e-10
        out["gpu_parity"] = {"orders": f"{done[0]}..{done[-1]} step {stride}",
                             "max_rel_l2_forward": fv, "max_rel_l2_adjoint": av,
                             "max_block_rel_l2_forward": fb, "max_block_rel_l2_adjoint": ab,
                             "per": "state and variable over the sampled orders, and within each order's block",
                             "bound": 1e-10, "ok": ok}
        if not ok:
            print(f"bench.py: GPU step differs from the oracle beyond 1e-10: {out['gpu_parity']}", file=sys.stderr)
    return out


def graph_replay_medians(plan, u, reps=25):
    """Median of `reps` graph replays of one forward and one adjoint step
    (HIP events around each replay on the launch stream)."""
    import torch
    plan.set_timing(False)
    plan.set_graphs(True)
    out = {}
    for name, fn in (("forward_ms", plan.step), ("adjoint_ms", plan.step_adjoint)):
        fn(u)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn(u)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        out[name] = sorted(times)[len(times) // 2]
    out["replays"] = reps
    out["note"] = "each replay includes the layout conversions into and out of the chain layout"
    return out


def bump_runs(rexi, synth, torch, dev, reps=3):
    """Wall-clock of the Gaussian-bump workload (Section 6.2) over 1.5 days on
    one GPU: SH analysis of the bump fields, the T-REXI steps, SH synthesis of
    the geopotential; inputs resident in HBM, plan built beforehand."""
    out = {}
    for name, w in synth.BUMP_WORKLOADS.items():
        plan = rexi.plan_for(w, max_states=1, max_fields=3)
        plan.autotune(1)
        grid = torch.from_numpy(synth.bump_fields(w.nlat, w.nlon)).to(dev)

        def run():
            u = plan.sh_forward(grid).view(1, 3, plan.nspec)
            u = plan.step(u, w.steps)
            return plan.sh_inverse(u.view(3, plan.nspec)[:1])

        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            h = run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert torch.isfinite(h).all()
        out[name] = {"seconds_per_1.5_days": dt, "steps": w.steps, "dt_s": w.dt, "M": w.M, "poles": plan.n_poles,
                     "T": w.T, "grid": f"{w.nlon}x{w.nlat}"}
        del plan
    out["paper_context"] = ("Cheyenne, Section 6.4 (other hardware, up to 512 MPI ranks; context only): "
                            "13.5 s for the best T-REXI run with M = 512, 2.02 s for one 1.5-day step with M = 4096")
    return out


def vector_run(plan, u, T, nlat, torch, reps=25):
    """Vector transforms of the benchmark states (winds from vorticity and
    divergence and back, Eq. (1)), median event time per call over `reps`
    calls.  Both run the Legendre contraction at degree T + 1 on 2 S fields."""
    S = u.shape[0]
    uv = plan.vortdiv_to_uv(u)
    back = torch.empty_like(u)
    plan.uv_to_vortdiv(uv, out=back)
    torch.cuda.synchronize()
    out = {}
    for name, fn in (("vortdiv_to_uv_ms", lambda: plan.vortdiv_to_uv(u, out=uv)),
                     ("uv_to_vortdiv_ms", lambda: plan.uv_to_vortdiv(uv, out=back))):
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        out[name] = sorted(times)[len(times) // 2]
    out["pairs"] = S
    out["legendre_flops_per_call"] = legendre_flops(T + 1, nlat, 2 * S)
    out["note"] = "each call: one spectral recombination, FFTs and the Legendre contraction at degree T + 1"
    return out


def dispersion_run(rexi, synth, torch, dev):
    """Numerical dispersion of the step on the f-sphere (Section 6.3): every
    mode stepped once on the GPU, log-eigenvalues against the exact frequencies."""
    from paper_1812_03431_amd import dispersion
    w, f0 = synth.DISPERSION_WORKLOAD, synth.FSPHERE_F0
    plan = rexi.plan_for(w, max_states=64, grid=False, fsphere=f0)
    t0 = time.perf_counter()
    res = dispersion.analyse(plan, w.T, w.dt, f0, synth.GRAVITY * synth.MEAN_DEPTH, synth.EARTH_RADIUS, dev)
    return {"T": w.T, "dt_s": w.dt, "M": w.M, "f0": f0, "modes": int(len(res["exact"])),
            "max_rel_phase_error": res["max_rel_phase_error"], "max_abs_zero_mode_rad_s": res["max_abs_zero_mode"],
            "max_abs_growth_per_s": res["max_abs_growth"], "seconds": time.perf_counter() - t0}


def stage(msg):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="t256_fwd_adj")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-bumps", action="store_true", help="skip the Gaussian-bump wall-clock runs")
    ap.add_argument("--no-large-transform", action="store_true",
                    help="skip the Legendre kernels at T1023 (2048 x 1024, 16 fields)")
    ap.add_argument("--schedule", type=int, default=-1, help="use this schedule index instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs the whole "
              f"step on a single MI355X (sharding by zonal order is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1812_03431_amd as rexi

    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    S = w.states
    B = 3 * S
    plan = rexi.plan_for(w, max_states=S, max_fields=B)
    N, T = plan.n_poles, w.T
    ck = w.checkpoint_every or w.steps
    nseg = w.steps // ck

    grid = torch.from_numpy(synth.random_grid(w.nlat, w.nlon, B, 0)).to(dev)
    target = torch.from_numpy(synth.random_state(T, S, 100)[:, 0].copy()).to(dev)
    stage("plan built")
    if args.schedule >= 0:
        plan.set_schedule(S, args.schedule)
        chosen = args.schedule
    elif not args.no_autotune:
        chosen = plan.autotune(S)
    else:
        chosen = plan.chosen_schedule(S)
    sched_name = plan.schedule_name(S, chosen)
    sched_classes = plan.schedule_classes(S, chosen)
    torch.cuda.synchronize()

    def job():
        u = plan.sh_forward(grid).view(S, 3, plan.nspec)
        boundaries = [u]
        for _ in range(nseg):
            u = plan.step(u, ck)
            boundaries.append(u)
        g = torch.zeros_like(u)
        g[:, 0] = 2.0 * (u[:, 0] - target)
        for _ in range(nseg):
            g = plan.step_adjoint(g, ck)
        return plan.sh_inverse(g.view(B, plan.nspec))

    stage(f"schedule {chosen} ({sched_name}); warm-up")
    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    # the timed region runs the product path (captured step graphs); the plan
    # brackets each step's graph replay and each Legendre launch with a HIP
    # event pair on the launch stream
    plan.set_graphs(True)
    plan.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = job()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_timing(False)
    solve_ms, solve_n = plan.kernel_time(plan.KERNEL_SOLVE)
    lf_ms, lf_n = plan.kernel_time(plan.KERNEL_LEGENDRE_FWD)
    li_ms, li_n = plan.kernel_time(plan.KERNEL_LEGENDRE_INV)
    assert torch.isfinite(out).all()

    elapsed = t1 - t0
    blocks_per_job = 2 * w.steps * N * (T + 1)
    value = blocks_per_job * args.steps / elapsed

    stage(f"timed {args.steps} steps: {elapsed / args.steps * 1e3:.2f} ms each")
    # the plain per-term launch form vs the batched form, one forward step each
    u = plan.sh_forward(grid).view(S, 3, plan.nspec)
    plan.step(u, 1)
    plan.step_per_term(u)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    plan.step(u, 1)
    e[1].record()
    e[2].record()
    plan.step_per_term(u)
    e[3].record()
    torch.cuda.synchronize()
    batched_ms, per_term_ms = e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3])

    avg_solve_s = solve_ms / 1e3 / max(1, solve_n)
    fl = solve_flops_per_launch(N, T, S)
    achieved = fl / avg_solve_s / 1e12
    fl_thomas = solve_flops_thomas(N, T, S)
    digest = kernel_source_digest()
    tr = load_summary("k_solve_t256_fwd_adj_traffic.json", digest, sched_name)
    traffic = tr.get("traffic_bytes_per_launch") if tr else None
    state_bytes = 2.0 * S * 3 * plan.nspec * 16       # state in and out of one step
    ctr = load_summary("k_solve_t256_fwd_adj_counters.json", digest, sched_name)
    pt = load_summary("per_term_t256_traffic.json", digest)
    per_term_hbm = None
    if pt:
        b_step = pt["bytes_per_step"]
        per_term_hbm = {"bytes_per_step": b_step, "achieved_GBps": b_step / (per_term_ms / 1e3) / 1e9,
                        "peak_GBps": HBM_PEAK, "frac": b_step / (per_term_ms / 1e3) / 1e9 / HBM_PEAK,
                        "source": "profiles/per_term_t256_traffic.json (FETCH_SIZE + WRITE_SIZE of one "
                                  "per-term step, scaled by a copy kernel's reading); time: this run"}
    lflops = legendre_flops(T, w.nlat, B)
    leg = {}
    if lf_n and li_n:
        a_f = lflops / (lf_ms / 1e3 / lf_n) / 1e12
        a_i = lflops / (li_ms / 1e3 / li_n) / 1e12
        # the measurement contract counts the contraction unfolded,
        # 2 nlat C nspec per direction, twice the folded work the kernels do
        lflops_u = 2.0 * lflops
        leg = {"bound": "mfma", "unit": "TFLOP/s", "peak": FP64_MFMA_PEAK,
               "forward_achieved": round(a_f, 3), "forward_frac": round(a_f / FP64_MFMA_PEAK, 4),
               "inverse_achieved": round(a_i, 3), "inverse_frac": round(a_i / FP64_MFMA_PEAK, 4),
               "forward_avg_ms": round(lf_ms / lf_n, 4), "inverse_avg_ms": round(li_ms / li_n, 4),
               "flops_per_launch": lflops,
               "flop_count": "folded: 2 (nlat/2) (2 fields) nspec per direction (the kernels use the "
                             "equatorial symmetry)",
               "flops_per_launch_unfolded": lflops_u,
               "forward_frac_unfolded": round(2 * a_f / FP64_MFMA_PEAK, 4),
               "inverse_frac_unfolded": round(2 * a_i / FP64_MFMA_PEAK, 4),
               "timing": "HIP events around each Legendre launch inside the timed job"}

    rec = {
        "metric": "REXI (term,m)-block solves/s and step time fwd+adjoint at T256, <=1e-10 rel L2",
        "value": value,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded random Gaussian-grid fields (SH analysis input) and a seeded random "
                "spectral Phi target",
        "config": {"workload": w.name, "T": T, "grid": f"{w.nlon}x{w.nlat}", "dt_s": w.dt, "M": w.M,
                   "h": w.h, "poles": N, "states": S, "forward_steps": w.steps, "adjoint_steps": w.steps,
                   "checkpoint_every": ck, "sh_fields": B, "blocks_per_step": blocks_per_job},
        "schedule": chosen,
        "schedule_name": sched_name,
        "schedule_classes": [list(c) for c in sched_classes],
        "timed_path": "step graphs on; HIP events around each step graph and Legendre launch",
        "rexi_step_ms": avg_solve_s * 1e3,
        "fwd_plus_adjoint_step_ms": 2 * avg_solve_s * 1e3,
        "batched_step_ms": batched_ms,
        "per_term_step_ms": per_term_ms,
        "batched_vs_per_term": per_term_ms / batched_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK, "traffic": traffic, "kernel": "k_solve",
                     "flops_per_launch": fl, "flop_count": "nspec N (40 + 156 S) per forward step",
                     "avg_launch_ms": avg_solve_s * 1e3, "launches": solve_n,
                     "launch": "one step: the captured graph of the solve class launches and the reduction",
                     "thomas_flops_per_launch": fl_thomas, "thomas_achieved": fl_thomas / avg_solve_s / 1e12,
                     "thomas_frac": fl_thomas / avg_solve_s / 1e12 / FP64_VECTOR_PEAK,
                     "algorithmic_bytes_per_launch": state_bytes,
                     "algorithmic_GBps": state_bytes / avg_solve_s / 1e9,
                     "traffic_GBps": (traffic / avg_solve_s / 1e9) if traffic else None,
                     "traffic_k_solve_classes": tr.get("k_solve_classes_bytes_per_launch") if tr else None,
                     "traffic_earlier_MB": ([(r["kernel_source_sha256_16"], r["schedule"], r["MB_per_step"], r["what"])
                                             for r in tr.get("earlier_readings", {}).get("runs", [])] if tr else None),
                     "executed_fp64_flops_per_launch": ctr.get("executed_fp64_flops_per_step") if ctr else None,
                     "kernel_source_sha256_16": digest},
        "per_term_hbm": per_term_hbm,
        "legendre": leg,
    }
    if args.copy_calibration:
        # one elementwise kernel that reads 1 GiB and writes 1 GiB: the scale of
        # the FETCH_SIZE / WRITE_SIZE counters for known traffic
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 1 << 30
    stage("per-term form and extras")
    if not args.no_bumps:
        rec["bumps"] = bump_runs(rexi, synth, torch, dev)
        rec["dispersion"] = dispersion_run(rexi, synth, torch, dev)
    rec["graph_replay_median"] = graph_replay_medians(plan, u)
    rec["vector_transforms"] = vector_run(plan, u, T, w.nlat, torch)
    if not args.no_large_transform:
        rec["legendre_large"] = legendre_large_run(rexi, synth, torch, dev)
    # physical check of the timed run: the linear operator conserves the
    # energy, so 16 REXI steps may change it by the REXI error only (the
    # spectral sum: the 512 x 256 grid is not exact for the top degree)
    from paper_1812_03431_amd import diagnostics
    e0 = diagnostics.spectral_energy(plan, u)
    e1 = diagnostics.spectral_energy(plan, plan.step(u, w.steps))
    rec["energy_drift"] = {"steps": w.steps, "max_rel_change": float((e1 / e0 - 1).abs().max().item()),
                           "quantity": "(1/4) sum c_m [Phibar a^2/(n(n+1)) (|zeta|^2+|delta|^2) + |Phi|^2] "
                                       "of the 4 benchmark states"}
    if not args.no_cpu_baseline:
        stage("oracle on the host")
        us = torch.from_numpy(synth.random_state(T, S, 0)).to(dev)
        gf = plan.step(us).cpu().numpy()
        ga = plan.step_adjoint(us).cpu().numpy()
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, gf, ga)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
