"""Run the spherical-harmonic transforms of a named workload, for profiling.

``python -m paper_1812_03431_amd.profile_sh --workload t256_fwd_adj --reps 5``
builds the workload's plan, then runs ``reps`` analyses and syntheses of its
transform fields (3 per state) on seeded random inputs and prints the mean
HIP-event time of the Legendre kernels.  It is meant to run under rocprofv3,
so that the trace or the counters hold the transform kernels alone.
"""
import argparse

import synth

from . import rexi


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="t256_fwd_adj")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    w = synth.WORKLOADS[args.workload]
    B = 3 * w.states
    plan = rexi.plan_for(w, max_states=w.states, max_fields=B)
    dev = torch.device("cuda:0")
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
    print(f"{w.name}: {B} fields, Legendre forward {1e3 * f_ms / f_n:.1f} us, inverse {1e3 * i_ms / i_n:.1f} us "
          f"(HIP events, mean of {args.reps})", flush=True)


if __name__ == "__main__":
    main()
