"""Run the spherical-harmonic transforms of a named workload, for profiling.

``python -m paper_1812_03431_amd.profile_sh --workload t256_fwd_adj --reps 5``
builds the workload's plan, then runs ``reps`` analyses and syntheses of its
transform fields (3 per state) on seeded random inputs and prints the mean
HIP-event time of the Legendre kernels, with their algorithmic FP64 rate
against the chip's FP64 matrix peak.  It is meant to run under rocprofv3, so
that the trace or the counters hold the transform kernels alone.

``--T``, ``--nlat``, ``--nlon`` and ``--fields`` replace the workload's
truncation, grid and field count (for example ``--T 1023 --nlat 1024 --nlon
2048 --fields 16``), to see how the contraction behaves where it is large.
"""
import argparse
from dataclasses import replace

import synth

from . import rexi

FP64_MFMA_PEAK = 78.6  # TFLOP/s, dense FP64 matrix peak of the MI355X


def legendre_flops(T, nlat, fields):
    """Algorithmic flops of one Legendre contraction (either direction), using
    the equatorial symmetry: 2 x (nlat/2) x (2 fields) per coefficient."""
    nspec = (T + 1) * (T + 2) // 2
    return 2.0 * (nlat // 2) * (2 * fields) * nspec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="t256_fwd_adj")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--T", type=int, default=None)
    ap.add_argument("--nlat", type=int, default=None)
    ap.add_argument("--nlon", type=int, default=None)
    ap.add_argument("--fields", type=int, default=None)
    args = ap.parse_args()
    import torch
    w = synth.WORKLOADS[args.workload]
    B = 3 * w.states
    if args.T is not None or args.nlat is not None or args.nlon is not None:
        # a transform-only plan: the smallest REXI tables, one state
        w = replace(w, name=f"{w.name}_resized", T=args.T if args.T is not None else w.T,
                    nlat=args.nlat if args.nlat is not None else w.nlat,
                    nlon=args.nlon if args.nlon is not None else w.nlon, M=8, states=1, steps=1)
    if args.fields is not None:
        B = args.fields
    plan = rexi.plan_for(w, max_states=w.states, max_fields=B)
    dev = torch.device("cuda:0")
    print(f"T{w.T} on {w.nlon} x {w.nlat}, {B} fields, {args.reps} reps", flush=True)
    grid = torch.from_numpy(synth.random_grid(w.nlat, w.nlon, B, 0)).to(dev)
    spec = plan.sh_forward(grid)
    back = plan.sh_inverse(spec)
    torch.cuda.synchronize()
    plan.set_timing(True)
    for _ in range(args.reps):
        plan.sh_forward(grid, out=spec)
        plan.sh_inverse(spec, out=back)
    torch.cuda.synchronize()
    plan.set_timing(False)
    f_ms, f_n = plan.kernel_time(plan.KERNEL_LEGENDRE_FWD)
    i_ms, i_n = plan.kernel_time(plan.KERNEL_LEGENDRE_INV)
    fl = legendre_flops(w.T, w.nlat, B)
    f_us, i_us = 1e3 * f_ms / f_n, 1e3 * i_ms / i_n
    f_tf, i_tf = fl / (f_us * 1e-6) / 1e12, fl / (i_us * 1e-6) / 1e12
    print(f"{w.name}: T{w.T} on {w.nlon} x {w.nlat}, {B} fields: Legendre forward {f_us:.1f} us "
          f"({f_tf:.1f} TF/s, {f_tf / FP64_MFMA_PEAK:.1%} of FP64 MFMA peak), inverse {i_us:.1f} us "
          f"({i_tf:.1f} TF/s, {i_tf / FP64_MFMA_PEAK:.1%}) (HIP events, mean of {args.reps}; "
          f"{fl:.3e} flops per call)", flush=True)


if __name__ == "__main__":
    main()
