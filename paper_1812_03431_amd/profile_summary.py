"""Summaries of rocprofv3 counter runs of the benchmark, for profiles/.

traffic:  two runs of ``bench.py --copy-calibration`` under ``rocprofv3 --pmc
          FETCH_SIZE`` and ``--pmc WRITE_SIZE`` -> HBM bytes of one REXI step
          (the fused solve's class launches and the reduction; mean per class
          over all steps of the run) and of one per-term step (the sum over
          its per-pole launches; the benchmark runs one).  Each counter is
          scaled by what it reads for an elementwise kernel that reads and
          writes 1 GiB (torch.mul on 2^27 doubles; the largest such
          dispatch of the run).
sh:       a kernel-trace run and one SQ counter run of ``profile_sh`` -> per
          transform kernel: duration, algorithmic TF/s of the Legendre
          kernels, MFMA work executed and MFMA-pipe busy fraction.
counters: one or more runs under ``rocprofv3 --pmc`` with SQ counters -> per
          class and per step: VALU wave-instructions, FP64 flops executed
          (SQ_INSTS_VALU_FLOPS_FP64 counts the flops of one lane per
          wave-instruction, so a step executes 64 times its sum), the other
          counters given and, where they were taken, each class's shares of
          wave lifetime (issuing, waiting at s_waitcnt, waiting for operands),
          instruction-cache misses per hit and the LDS bank-conflict share.

Writes JSON keyed by the solve kernel source's hash (bench.py reports a
summary only while the hash matches the source).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOLVE = re.compile(r"k_solve<(\d+), (true|false), (\d), (\d), (\d)>")


def source_digest():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1812_03431_amd", "csrc", "rexi_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def rows(path):
    with open(path) as f:
        yield from csv.DictReader(f)


def per_dispatch(path, counter):
    """{dispatch id: (kernel name, value summed over the counter's instances)}"""
    out = {}
    for r in rows(path):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        name, v = out.get(d, (r["Kernel_Name"], 0.0))
        out[d] = (name, v + float(r["Counter_Value"]))
    return out


def class_of(name):
    m = SOLVE.search(name)
    if m:
        se, pt, kind, w, rot = m.groups()
        return ("per_term" if pt == "true" else "batched", f"k_solve<{se}, {pt}, {kind}, {w}, {rot}>")
    if "k_reduce" in name:
        return ("batched", "k_reduce")
    return (None, None)


def calibration(path, counter):
    """The counter's reading for the 1 GiB elementwise kernel: the largest
    reading among the run's torch multiply dispatches (the others are small
    tensors)."""
    vals = [v for d, (n, v) in per_dispatch(path, counter).items() if "MulFunctor" in n]
    if not vals:
        raise SystemExit(f"{path}: no calibration dispatch (run bench.py with --copy-calibration)")
    return max(vals)


def earlier_readings(path):
    """The readings of an existing traffic summary (its own and the ones it
    carried), so that a new run keeps the history: a list of
    {source hash, schedule, MB per step, what}."""
    try:
        with open(path) as f:
            old = json.load(f)
    except (OSError, ValueError):
        return []
    runs = list(old.get("earlier_readings", {}).get("runs", []))
    if "traffic_bytes_per_launch" in old:
        runs.append({"kernel_source_sha256_16": old.get("kernel_source_sha256_16"), "schedule": old.get("schedule"),
                     "MB_per_step": round(old["traffic_bytes_per_launch"] / 1e6, 2),
                     "what": "k_solve class launches and k_reduce of one step"})
        if "k_solve_classes_bytes_per_launch" in old:
            runs.append({"kernel_source_sha256_16": old.get("kernel_source_sha256_16"), "schedule": old.get("schedule"),
                         "MB_per_step": round(old["k_solve_classes_bytes_per_launch"] / 1e6, 2),
                         "what": "k_solve class launches only (no reduction)"})
    return runs


def traffic(fetch_csv, write_csv, schedule, workload, commands, earlier=(), schedule_name=None):
    GiB_KiB = float(1 << 20)
    fcal, wcal = calibration(fetch_csv, "FETCH_SIZE"), calibration(write_csv, "WRITE_SIZE")
    fscale, wscale = GiB_KiB / fcal, GiB_KiB / wcal
    out = {}
    for kind in ("batched", "per_term"):
        cls = collections.defaultdict(lambda: {"fetch_kib": [], "write_kib": []})
        for path, counter, key in ((fetch_csv, "FETCH_SIZE", "fetch_kib"), (write_csv, "WRITE_SIZE", "write_kib")):
            for d, (name, v) in per_dispatch(path, counter).items():
                k, c = class_of(name)
                if k == kind:
                    cls[c][key].append(v)
        out[kind] = cls
    per_class = {}
    step = solve_only = 0.0
    for c, v in out["batched"].items():
        f = sum(v["fetch_kib"]) / max(1, len(v["fetch_kib"]))
        w = sum(v["write_kib"]) / max(1, len(v["write_kib"]))
        per_class[c] = {"fetch_kib_mean": f, "write_kib_mean": w, "dispatches": len(v["fetch_kib"])}
        step += (f * fscale + w * wscale) * 1024.0
        if c != "k_reduce":
            solve_only += (f * fscale + w * wscale) * 1024.0
    pt_f = sum(sum(v["fetch_kib"]) for v in out["per_term"].values())
    pt_w = sum(sum(v["write_kib"]) for v in out["per_term"].values())
    pt_n = sum(len(v["fetch_kib"]) for v in out["per_term"].values())
    digest = source_digest()
    cal = {"kernel": "torch.mul(a, 1.0, out=b) on 2^27 doubles: reads 1 GiB, writes 1 GiB",
           "fetch_kib": fcal, "write_kib": wcal, "fetch_scale": fscale, "write_scale": wscale,
           "dispatch": "the largest reading among the run's torch multiply dispatches"}
    solve = {"kernel": "k_solve (fused REXI solve) class launches and k_reduce of one step",
             "workload": workload, "schedule": schedule, "schedule_name": schedule_name,
             "kernel_source_sha256_16": digest,
             "commands": commands, "calibration": cal, "per_class": per_class,
             "traffic_bytes_per_launch": step,
             "k_solve_classes_bytes_per_launch": solve_only,
             "note": "one launch = one step; bytes = sum over the step's kernels of the mean per dispatch of "
                     "FETCH_SIZE*fetch_scale + WRITE_SIZE*write_scale (KiB -> bytes)",
             "earlier_readings": {"note": "the same two counter runs on earlier versions of the solve kernel "
                                          "(source hash, schedule); the spread of repeated runs on one kernel "
                                          "shows in the entries that share a hash",
                                  "runs": list(earlier)}}
    per_term = {"kernel": "k_solve per-term launches (one per pole and class) of one per-term step",
                "workload": workload, "kernel_source_sha256_16": digest, "commands": commands,
                "calibration": cal, "dispatches": pt_n, "fetch_kib_total": pt_f, "write_kib_total": pt_w,
                "bytes_per_step": (pt_f * fscale + pt_w * wscale) * 1024.0}
    return solve, per_term


# per-wave shares of a wave's lifetime (SQ_WAVE_CYCLES), where the counters
# were taken: issuing any instruction, issuing VALU instructions, waiting at
# s_waitcnt, waiting for an instruction's operands (dependencies)
STALL_SHARES = {"active_any": "SQ_ACTIVE_INST_ANY", "active_valu": "SQ_ACTIVE_INST_VALU",
                "wait_any": "SQ_WAIT_ANY", "wait_inst_any": "SQ_WAIT_INST_ANY"}


def counters(csv_paths, schedule, workload, commands, steps_note, clock_ghz=2.4, simds=1024, schedule_name=None):
    """Per class (mean per dispatch) and per step sums of the counters of one
    or more rocprofv3 --pmc runs (one CSV each)."""
    if isinstance(csv_paths, str):
        csv_paths = [csv_paths]
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for run, path in enumerate(csv_paths):
        for r in rows(path):
            k, c = class_of(r["Kernel_Name"])
            if k != "batched":
                continue
            per[c][(r["Counter_Name"], run, r["Dispatch_Id"])].append(float(r["Counter_Value"]))
    per_class = {}
    step = collections.Counter()
    for c, d in per.items():
        acc = collections.defaultdict(list)
        for (name, _run, _disp), v in d.items():
            acc[name].append(sum(v))
        mean = {name: sum(v) / len(v) for name, v in acc.items()}
        mean["dispatches"] = max(len(v) for v in acc.values())
        per_class[c] = mean
        for name, v in mean.items():
            if name != "dispatches":
                step[name] += v
    out = {"kernel": "k_solve class launches and k_reduce of one step", "workload": workload,
           "schedule": schedule, "schedule_name": schedule_name, "kernel_source_sha256_16": source_digest(),
           "commands": commands,
           "per_class_mean_per_dispatch": per_class, "per_step": dict(step), "note": steps_note}
    if "SQ_INSTS_VALU_FLOPS_FP64" in step:
        out["executed_fp64_flops_per_step"] = 64.0 * step["SQ_INSTS_VALU_FLOPS_FP64"]
    if "SQ_WAVE_CYCLES" in step:
        shares = {}
        for c, m in per_class.items():
            wc = m.get("SQ_WAVE_CYCLES", 0.0)
            if wc > 0:
                shares[c] = {k: m[v] / wc for k, v in STALL_SHARES.items() if v in m}
        out["stall_shares_per_class"] = shares
        # SQ_WAVE_CYCLES counts in units of four cycles
        out["wave_lifetime_over_simds_ms"] = 4.0 * step["SQ_WAVE_CYCLES"] / simds / (clock_ghz * 1e9) * 1e3
        out["wave_lifetime_note"] = (f"summed wave lifetimes of one step's solve class launches and reduction (4 x SQ_WAVE_CYCLES) "
                                     f"over {simds} SIMDs at {clock_ghz} GHz")
    if "SQC_ICACHE_MISSES" in step and step.get("SQC_ICACHE_HITS"):
        out["icache_miss_per_hit"] = step["SQC_ICACHE_MISSES"] / step["SQC_ICACHE_HITS"]
    if "SQ_LDS_BANK_CONFLICT" in step and step.get("SQ_LDS_IDX_ACTIVE"):
        out["lds_bank_conflict_share"] = step["SQ_LDS_BANK_CONFLICT"] / step["SQ_LDS_IDX_ACTIVE"]
    return out


def stats(stats_csv, trace_csv, schedule, workload, command, events_ms, schedule_name=None):
    """Text summary of a kernel-trace run: per-kernel statistics and the span
    of each REXI step (first solve class start to its reduction's end)."""
    sched = f"schedule {schedule}" + (f" ({schedule_name})" if schedule_name else "")
    lines = [f"# rocprofv3 kernel statistics: {workload} benchmark job (bench.py), {sched}",
             "# command (on one MI355X, from /tmp with TMPDIR=/tmp):", f"#   {command}",
             "# one REXI step = one captured graph: a k_solve launch per tile class "
             "(template <elements per lane, per-term, move kind, waves, states per item>) and k_reduce;",
             "# k_solve<.., true, .., 1, 1> are the per-term comparison launches (one per pole and class).",
             f"# kernel source sha256[:16] = {source_digest()}"]
    spans, start = [], None
    for r in sorted(rows(trace_csv), key=lambda r: int(r["Start_Timestamp"])):
        n = r["Kernel_Name"]
        k, c = class_of(n)
        if k == "batched" and c != "k_reduce":
            if start is None:
                start = int(r["Start_Timestamp"])
        elif c == "k_reduce" and start is not None:
            spans.append((int(r["End_Timestamp"]) - start) / 1e3)
            start = None
    if spans:
        spans.sort()
        lines.append(f"# step span (first class start to reduction end, {len(spans)} steps): mean "
                     f"{sum(spans) / len(spans):.1f} us, median {spans[len(spans) // 2]:.1f} us"
                     + (f"; HIP events around the step graphs in the bench line: {events_ms * 1e3:.1f} us"
                        if events_ms else ""))
    lines.append("# (class launches overlap on side streams, so per-class durations below do not add up to a step)")
    lines.append("")
    lines.append(" calls   total_ms     avg_us    min_us    max_us    pct  kernel")
    for r in sorted(rows(stats_csv), key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}  {r['Name'][:150]}")
    return "\n".join(lines) + "\n"


# flops of one MFMA wave-instruction of each Legendre kernel:
# v_mfma_f64_4x4x4f64 (four blocks of 4 x 4 x 4 multiply-adds) or, in the
# inverse for grids of more than 128 northern latitudes, v_mfma_f64_16x16x4f64
MFMA_FLOPS = {"k_legendre_forward": 4 * 4 * 4 * 4 * 2, "k_legendre_inverse": 4 * 4 * 4 * 4 * 2,
              "k_legendre_inverse_seq": 16 * 16 * 4 * 2}
SH_KERNELS = ("k_fft_forward", "k_legendre_forward", "k_legendre_inverse_seq", "k_legendre_inverse", "k_fft_inverse")


def sh(stats_csv, pmc_csv, title, commands, T, nlat, fields, peak=78.6):
    """Text summary of the transform kernels: durations (kernel trace) and,
    per dispatch, MFMA instructions, MFMA-pipe busy fraction, waves, VALU
    instructions per wave and LDS bank-conflict cycles (one counter run)."""
    nspec = (T + 1) * (T + 2) // 2
    alg = 2.0 * (nlat // 2) * (2 * fields) * nspec
    short = lambda n: next((k for k in SH_KERNELS if k in n), None)
    dur = {}
    for r in rows(stats_csv):
        k = short(r["Name"])
        if k:
            dur[k] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in rows(pmc_csv):
        k = short(r["Kernel_Name"])
        if k:
            per[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k].add(r["Dispatch_Id"])
    lines = [f"# {title}", "# commands (on one MI355X, from /tmp with TMPDIR=/tmp and PYTHONPATH=<repo>):"]
    lines += [f"#   {c}" for c in commands]
    lines += [f"# algorithmic Legendre flops per launch 2 (nlat/2) (2B) nspec = {alg:.4g} (folded: the kernels use the "
              f"equatorial symmetry; unfolded, 2 nlat (2B) nspec, twice that: frac x 2); FP64 matrix peak {peak} TFLOP/s",
              "# MFMA pipe busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs); executed = "
              "SQ_INSTS_MFMA x 512 flop (v_mfma_f64_4x4x4f64) or x 2048 (v_mfma_f64_16x16x4f64, k_legendre_inverse_seq)",
              "# summary: python -m paper_1812_03431_amd.profile_summary sh (this file's arguments)", "",
              f"{'kernel':24s} {'calls':>5s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'alg_TF':>7s} {'frac':>6s} "
              f"{'exec_MFLOP':>10s} {'mfma_busy':>9s} {'waves':>6s} {'valu/wave':>9s} {'lds_conf':>9s}"]
    for k in SH_KERNELS:
        if k not in dur:
            continue
        n, avg, lo, hi = dur[k]
        c = per.get(k, {})
        nd = max(1, len(disp.get(k, ())))
        leg = "legendre" in k
        tf = alg / (avg * 1e-6) / 1e12 if leg else float("nan")
        busy = (c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (1024.0 * c["GRBM_GUI_ACTIVE"] / 8.0)
                if c.get("GRBM_GUI_ACTIVE") else float("nan"))
        waves = c.get("SQ_WAVES", 0.0) / nd
        lines.append(f"{k:24s} {n:5d} {avg:8.2f} {lo:8.2f} {hi:8.2f} {tf:7.2f} {tf / peak:6.1%} "
                     f"{c.get('SQ_INSTS_MFMA', 0.0) / nd * MFMA_FLOPS.get(k, 0) / 1e6:10.1f} {busy:9.1%} {waves:6.0f} "
                     f"{c.get('SQ_INSTS_VALU', 0.0) / nd / max(1.0, waves):9.0f} {c.get('SQ_LDS_BANK_CONFLICT', 0.0) / nd:9.0f}")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("stats")
    k.add_argument("--stats", required=True)
    k.add_argument("--trace", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--events-ms", type=float, default=None, help="the bench line's HIP-event step time (ms)")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--out-solve", required=True)
    t.add_argument("--out-per-term", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True, action="append", help="one per counter run")
    c.add_argument("--out", required=True)
    for p in (t, c, k):
        p.add_argument("--schedule", type=int, required=True)
        p.add_argument("--schedule-name", default=None, help="the schedule's name (the bench matches summaries by it)")
        p.add_argument("--workload", default="t256_fwd_adj")
        p.add_argument("--command", action="append", default=[], help="the rocprofv3 command lines (recorded)")
    x = sub.add_parser("sh")
    x.add_argument("--stats", required=True)
    x.add_argument("--pmc", required=True)
    x.add_argument("--out", required=True)
    x.add_argument("--title", required=True)
    x.add_argument("--T", type=int, required=True)
    x.add_argument("--nlat", type=int, required=True)
    x.add_argument("--fields", type=int, required=True)
    x.add_argument("--command", action="append", default=[])
    a = ap.parse_args()
    if a.what == "sh":
        with open(a.out, "w") as f:
            f.write(sh(a.stats, a.pmc, a.title, a.command, a.T, a.nlat, a.fields))
        return
    if a.what == "stats":
        with open(a.out, "w") as f:
            f.write(stats(a.stats, a.trace, a.schedule, a.workload, " ".join(a.command), a.events_ms,
                          a.schedule_name))
    elif a.what == "traffic":
        solve, per_term = traffic(a.fetch, a.write, a.schedule, a.workload, a.command, earlier_readings(a.out_solve),
                                  a.schedule_name)
        with open(a.out_solve, "w") as f:
            json.dump(solve, f, indent=1)
        with open(a.out_per_term, "w") as f:
            json.dump(per_term, f, indent=1)
    else:
        out = counters(a.csv, a.schedule, a.workload, a.command,
                       "per step = sum over the step's kernels of the mean per dispatch", schedule_name=a.schedule_name)
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
