"""The measurement pipeline on the CPU: the flop counts the bench reports, and
the rocprofv3 summary tool's arithmetic on small synthetic counter files."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_flop_counts_match_the_quoted_figures():
    b = _bench()
    # the step count nspec N (40 + 156 S): 4.56e10 per forward step at T256,
    # 4 states, M = 1024 (N = 2 (M + L) + 1 = 2071 poles)
    assert b.solve_flops_per_launch(2071, 256, 4) == pytest.approx(4.559e10, rel=1e-3)
    # Thomas count N (nspec - 1) (32 + 136 S)
    nspec = 257 * 258 // 2
    assert b.solve_flops_thomas(2071, 256, 4) == 2071 * (nspec - 1) * (32 + 136 * 4)
    # Legendre, folded: 2 (nlat / 2) (2 fields) nspec = 0.204 GF per direction
    # at T256 on 256 latitudes with 12 fields; unfolded (2 nlat C nspec) is
    # twice that, the 0.41 GF quoted for the transform
    fl = b.legendre_flops(256, 256, 12)
    assert fl == pytest.approx(2.037e8, rel=1e-3)
    assert 2 * fl == pytest.approx(0.407e9, rel=1e-2)


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=header)
        w.writeheader()
        for r in rows:
            w.writerow(r)


PMC_HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    from paper_1812_03431_amd import profile_summary as ps
    solve = "void rexi::k_solve<16, false, 1, 4, 4>(SolveArgs, int, int, int*)"
    red = "rexi::k_reduce(ReduceArgs)"
    mul = "at::native::vectorized_elementwise_kernel<4, MulFunctor<double>>"
    gib_kib = float(1 << 20)
    # the counter reads half of a 1 GiB read (x2 to scale) and all of the write
    fetch = [{"Dispatch_Id": 1, "Kernel_Name": mul, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2},
             {"Dispatch_Id": 2, "Kernel_Name": mul, "Counter_Name": "FETCH_SIZE", "Counter_Value": 10.0},
             {"Dispatch_Id": 3, "Kernel_Name": solve, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0},
             {"Dispatch_Id": 4, "Kernel_Name": solve, "Counter_Name": "FETCH_SIZE", "Counter_Value": 300.0},
             {"Dispatch_Id": 5, "Kernel_Name": red, "Counter_Name": "FETCH_SIZE", "Counter_Value": 50.0}]
    write = [{"Dispatch_Id": 1, "Kernel_Name": mul, "Counter_Name": "WRITE_SIZE", "Counter_Value": gib_kib},
             {"Dispatch_Id": 3, "Kernel_Name": solve, "Counter_Name": "WRITE_SIZE", "Counter_Value": 40.0},
             {"Dispatch_Id": 4, "Kernel_Name": solve, "Counter_Name": "WRITE_SIZE", "Counter_Value": 60.0},
             {"Dispatch_Id": 5, "Kernel_Name": red, "Counter_Name": "WRITE_SIZE", "Counter_Value": 8.0}]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, PMC_HEADER, fetch)
    _write(wp, PMC_HEADER, write)
    solve_sum, per_term = ps.traffic(str(fp), str(wp), 7, "t", ["cmd"], earlier=[{"MB_per_step": 1.0}])
    assert solve_sum["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert solve_sum["calibration"]["write_scale"] == pytest.approx(1.0)
    # per class: the mean over its dispatches, then fetch x2 + write x1, KiB -> bytes
    classes = (2.0 * 200.0 + 50.0) * 1024.0
    assert solve_sum["k_solve_classes_bytes_per_launch"] == pytest.approx(classes)
    assert solve_sum["traffic_bytes_per_launch"] == pytest.approx(classes + (2.0 * 50.0 + 8.0) * 1024.0)
    assert solve_sum["earlier_readings"]["runs"] == [{"MB_per_step": 1.0}]
    assert per_term["dispatches"] == 0


def test_earlier_readings_carry_forward(tmp_path):
    from paper_1812_03431_amd import profile_summary as ps
    old = {"kernel_source_sha256_16": "abc", "schedule": 3, "traffic_bytes_per_launch": 2.5e6,
           "k_solve_classes_bytes_per_launch": 1.5e6, "earlier_readings": {"runs": [{"MB_per_step": 9.0}]}}
    path = tmp_path / "old.json"
    path.write_text(json.dumps(old))
    runs = ps.earlier_readings(str(path))
    assert [r["MB_per_step"] for r in runs] == [9.0, 2.5, 1.5]
    assert ps.earlier_readings(str(tmp_path / "missing.json")) == []


def test_sh_summary_counts_each_kernel_shape(tmp_path):
    from paper_1812_03431_amd import profile_summary as ps
    stats = tmp_path / "stats.csv"
    _write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"],
           [{"Name": "void rexi::k_legendre_forward<3>(LegRun const*)", "Calls": 2, "TotalDurationNs": 20000,
             "AverageNs": 10000, "MinNs": 9000, "MaxNs": 11000, "Percentage": 50},
            {"Name": "void rexi::k_legendre_inverse_seq<2>(LegWork const*)", "Calls": 2, "TotalDurationNs": 20000,
             "AverageNs": 10000, "MinNs": 9000, "MaxNs": 11000, "Percentage": 50}])
    pmc = tmp_path / "pmc.csv"
    rows = []
    for d, name in ((1, "k_legendre_forward<3>"), (2, "k_legendre_inverse_seq<2>")):
        rows += [{"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": "SQ_INSTS_MFMA", "Counter_Value": 1.0e6},
                 {"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": "SQ_WAVES", "Counter_Value": 10.0},
                 {"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 50.0}]
    _write(pmc, PMC_HEADER, rows)
    text = ps.sh(str(stats), str(pmc), "title", ["c1"], 256, 256, 12)
    lines = {ln.split()[0]: ln.split() for ln in text.splitlines() if ln.startswith("k_legendre")}
    # algorithmic TF/s: 2 (256/2) (24) nspec flops over 10 us
    nspec = 257 * 258 // 2
    assert float(lines["k_legendre_forward"][5]) == pytest.approx(2 * 128 * 24 * nspec / 10e-6 / 1e12, rel=1e-3)
    # executed MFMA work: 512 flops per four-block instruction, 2048 per 16x16x4 one
    assert float(lines["k_legendre_forward"][7]) == pytest.approx(1.0e6 * 512 / 1e6)
    assert float(lines["k_legendre_inverse_seq"][7]) == pytest.approx(1.0e6 * 2048 / 1e6)


def test_counter_summary_stall_shares(tmp_path):
    from paper_1812_03431_amd import profile_summary as ps
    solve = "void rexi::k_solve<12, false, 1, 4, 4>(SolveArgs, int, int, int*)"
    p1 = [{"Dispatch_Id": d, "Kernel_Name": solve, "Counter_Name": n, "Counter_Value": v}
          for d in (1, 2) for n, v in (("SQ_WAVE_CYCLES", 1000.0), ("SQ_ACTIVE_INST_VALU", 700.0),
                                       ("SQ_WAIT_ANY", 200.0), ("SQ_WAIT_INST_ANY", 10.0))]
    p2 = [{"Dispatch_Id": d, "Kernel_Name": solve, "Counter_Name": n, "Counter_Value": v}
          for d in (7, 8) for n, v in (("SQC_ICACHE_HITS", 1.0e4), ("SQC_ICACHE_MISSES", 1.0),
                                       ("SQ_LDS_BANK_CONFLICT", 6.0), ("SQ_LDS_IDX_ACTIVE", 100.0))]
    f1, f2 = tmp_path / "p1.csv", tmp_path / "p2.csv"
    _write(f1, PMC_HEADER, p1)
    _write(f2, PMC_HEADER, p2)
    out = ps.counters([str(f1), str(f2)], 70, "t", ["c1", "c2"], "note", clock_ghz=2.0, simds=4)
    sh = out["stall_shares_per_class"]["k_solve<12, false, 1, 4, 4>"]
    assert sh["active_valu"] == pytest.approx(0.7) and sh["wait_any"] == pytest.approx(0.2)
    assert sh["wait_inst_any"] == pytest.approx(0.01)
    # mean per dispatch; 4 cycles per count; over 4 SIMDs at 2 GHz
    assert out["wave_lifetime_over_simds_ms"] == pytest.approx(4.0 * 1000.0 / 4 / 2.0e9 * 1e3)
    assert out["icache_miss_per_hit"] == pytest.approx(1e-4)
    assert out["lds_bank_conflict_share"] == pytest.approx(0.06)
    assert out["per_class_mean_per_dispatch"]["k_solve<12, false, 1, 4, 4>"]["dispatches"] == 2


def test_bench_uses_a_summary_only_for_its_kernel_and_schedule(tmp_path, monkeypatch):
    b = _bench()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "profiles" / "s.json"
    path.write_text(json.dumps({"kernel_source_sha256_16": "abc", "schedule_name": "fine_items10"}))
    assert b.load_summary("s.json", "abc", "fine_items10") is not None
    assert b.load_summary("s.json", "abc", "fine_items12") is None     # another schedule
    assert b.load_summary("s.json", "abd", "fine_items10") is None     # another kernel source
    assert b.load_summary("s.json", "abc") is not None                 # schedule-independent use
    path.write_text(json.dumps({"kernel_source_sha256_16": "abc"}))    # no schedule recorded
    assert b.load_summary("s.json", "abc", "fine_items10") is None
    assert b.load_summary("missing.json", "abc") is None
