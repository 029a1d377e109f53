"""Host logic of bench.py's counter records: the source hash that keys them, the refusal of
a record taken on other sources, the scalar-issue figure and the counters-record writer."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.fixture
def sources(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    a.write_text("int f() {\n  return 1;  // one\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("a.hip",))
    return a


def test_source_hash_ignores_comments_and_blank_lines(sources):
    h0 = bench.kernel_source_hash()
    sources.write_text("// header\nint f() {\n\n  return 1;  // another comment\n}\n")
    assert bench.kernel_source_hash() == h0
    sources.write_text("int f() {\n  return 2;\n}\n")
    assert bench.kernel_source_hash() != h0


def test_records_are_refused_for_other_sources(sources, tmp_path, monkeypatch):
    traffic = tmp_path / "traffic.json"
    counters = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(traffic))
    monkeypatch.setattr(bench, "COUNTERS_RECORD", str(counters))
    assert bench.measured_traffic(10) is None  # no record
    traffic.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(),
                                   "hbm_bytes_per_frame": 100.0}))
    assert bench.measured_traffic(10) == 1000.0
    counters.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(),
                                    "per_extension": {"SQ_INSTS_SALU": 90.0,
                                                      "SQ_INSTS_VALU": 70.0}}))
    # 1000 frames x 2000 extensions in t ms: cycles per extension = t e-3 x CU_CYCLES_PER_S / 2e6
    t_ms = 2e6 * 100.0 / bench.CU_CYCLES_PER_S * 1e3  # 100 CU-cycles per extension
    per_point = {2.0: {"mean_iterations": 2000.0, "launch_ms": t_ms}}
    got = bench.issue_bound(per_point, 1000)
    assert got["cu_cycles_per_extension"] == pytest.approx(100.0)
    assert got["frac"] == pytest.approx(0.9)
    assert bench.issue_bound({3.0: per_point[2.0]}, 1000) is None  # no 2 dB point
    sources.write_text("int f() {\n  return 3;\n}\n")  # the code changed since the records
    assert bench.measured_traffic(10) is None
    assert bench.issue_bound(per_point, 1000) is None


def test_counters_record_excludes_the_statistics_launch(sources, tmp_path, monkeypatch):
    sq = tmp_path / "sq" / "run"
    sq.mkdir(parents=True)
    rows = []
    for kernel, salu in [("void scs_uniform_kernel<10, TrF32, false, 1>(x)", 9.0e6),
                         ("void scs_uniform_kernel<10, TrF32, true, 1>(x)", 5.0e9),
                         ("void other_kernel(x)", 7.0e9)]:
        rows.append({"Kernel_Name": kernel, "Counter_Name": "SQ_INSTS_SALU",
                     "Counter_Value": salu, "Dispatch_Id": len(rows)})
        rows.append({"Kernel_Name": kernel, "Counter_Name": "SQ_INSTS_VALU",
                     "Counter_Value": salu / 2, "Dispatch_Id": len(rows)})
    with open(sq / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    line = {"config": {"frames_per_point": 1000}, "per_point": {"2.0": {"mean_iterations": 100.0}}}
    bj = tmp_path / "bench.json"
    bj.write_text("log line\n" + json.dumps(line) + "\n")
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_RECORD", str(out))
    bench.write_counters_record(str(tmp_path / "sq"), str(bj))
    rec = json.loads(out.read_text())
    assert rec["kernel_source_hash"] == bench.kernel_source_hash()
    assert rec["per_extension"]["SQ_INSTS_SALU"] == pytest.approx(90.0)
    assert rec["per_extension"]["SQ_INSTS_VALU"] == pytest.approx(45.0)


def test_sweep_config_bounds_and_headline(monkeypatch):
    monkeypatch.setattr(bench, "D", bench.D)
    monkeypatch.setattr(bench, "L", bench.L)
    assert (bench.D, bench.L) == bench.HEADLINE_DL == (32, 8)
    for bad in ((0, 8), (257, 8), (32, 0), (32, 256)):
        with pytest.raises(SystemExit):
            bench.sweep_config(*bad)
    bench.sweep_config(128, 4)
    assert (bench.D, bench.L) == (128, 4)


def _write_csv(folder, rows):
    folder.mkdir(parents=True)
    with open(folder / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_util_record_and_rocprof_figures(sources, tmp_path, monkeypatch):
    """LDS bytes per extension from the 64-byte bandwidth counters of the timed launch only,
    derived metrics taken as reported, and the live figures: recorded per-extension work
    times this run's extensions per second."""
    timed, stats = "void scs_uniform_kernel<10, TrF32, false, 1>(x)", "void scs_uniform_kernel<10, TrF32, true, 1>(x)"
    lds_rows, busy_rows = [], []
    for kernel, scale in ((timed, 1.0), (stats, 7.0)):
        for c, v in (("SQ_INSTS_LDS_LOAD_BANDWIDTH", 1000.0), ("SQ_INSTS_LDS_STORE_BANDWIDTH", 500.0),
                     ("SQ_INSTS_LDS_ATOMIC_BANDWIDTH", 250.0), ("LdsUtil", 20.0)):
            lds_rows.append({"Kernel_Name": kernel, "Counter_Name": c, "Counter_Value": v * scale,
                             "Dispatch_Id": len(lds_rows)})
        for c, v in (("VALUBusy", 80.0), ("SALUBusy", 75.0), ("VALUUtilization", 50.0),
                     ("LDSBankConflict", 2.0)):
            busy_rows.append({"Kernel_Name": kernel, "Counter_Name": c, "Counter_Value": v * scale,
                              "Dispatch_Id": len(busy_rows)})
    _write_csv(tmp_path / "lds" / "run", lds_rows)
    _write_csv(tmp_path / "busy" / "run", busy_rows)
    line = {"config": {"frames_per_point": 10},
            "per_point": {"2.0": {"mean_iterations": 7.0, "launch_ms": 1.0}}}
    bj = tmp_path / "bench.json"
    bj.write_text(json.dumps(line) + "\n")
    pk = tmp_path / "peak.json"
    pk.write_text(json.dumps({"lds_peak": {"read_16B_per_lane": {"bytes_per_s": 1e12, "launch_ms": 1.0},
                                           "read_4B_per_lane": {"bytes_per_s": 5e11, "launch_ms": 1.0},
                                           "nominal_bytes_per_s": 7.8e13}}) + "\n")
    util = tmp_path / "util.json"
    counters = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "UTIL_RECORD", str(util))
    monkeypatch.setattr(bench, "COUNTERS_RECORD", str(counters))
    bench.write_util_record(str(tmp_path / "lds"), str(tmp_path / "busy"), str(bj), str(pk))
    rec = json.loads(util.read_text())
    assert rec["lds_bytes_per_extension"] == pytest.approx(1750.0 * 64 / 70.0)
    assert rec["derived_pct"] == {"VALUBusy": 80.0, "SALUBusy": 75.0, "VALUUtilization": 50.0,
                                  "LDSBankConflict": 2.0, "LdsUtil": 20.0}
    assert bench.rocprof_use({2.0: {"mean_iterations": 100.0, "launch_ms": 2.0}}, 1000) is None
    counters.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(),
                                    "per_extension": {"SQ_INSTS_SALU": 60.0, "SQ_INSTS_VALU": 40.0}}))
    got = bench.rocprof_use({2.0: {"mean_iterations": 100.0, "launch_ms": 2.0}}, 1000)
    ext_per_s = 1000 * 100.0 / 2e-3
    assert got["extensions_per_s"] == pytest.approx(ext_per_s)
    assert got["valu_lane_ops_per_s"] == pytest.approx(40.0 * 32.0 * ext_per_s)
    assert got["lds_bytes_per_s"] == pytest.approx(1600.0 * ext_per_s)
    assert got["lds_frac_measured"] == pytest.approx(1600.0 * ext_per_s / 1e12)
    sources.write_text("int f() {\n  return 4;\n}\n")
    assert bench.rocprof_use({2.0: {"mean_iterations": 100.0, "launch_ms": 2.0}}, 1000) is None


def _trace(folder, rows):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_kernel_trace.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, t0, t1 in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t1})


def test_serve_trace_summary_counts_overlap_in_the_serving_span(tmp_path):
    ms = 1_000_000
    mk = "void scs_mixed_kernel<(anonymous namespace)::TrF32>(int)"
    # one launch long before the serving span (capacity probe), then two overlapping pairs
    _trace(str(tmp_path / "t"), [(mk, 0, 10 * ms), ("fill_kernel(int)", 20 * ms, 21 * ms),
                                 (mk, 1000 * ms, 1010 * ms), (mk, 1000 * ms, 1010 * ms),
                                 (mk, 1020 * ms, 1030 * ms), (mk, 1025 * ms, 1035 * ms)])
    line = {"value": 900.0, "ms_per_step": 40.0, "config": {"workload": "serving",
            "offered_frames_per_s": 1e6}, "sustained_frames_per_s": 1e6,
            "latency_ms": {"p50": 20.0, "p99": 30.0}}
    (tmp_path / "b.json").write_text("log line\n" + json.dumps(line) + "\n")
    out = tmp_path / "s.md"
    bench.write_workload_trace_summary(str(tmp_path / "t"), str(tmp_path / "b.json"), str(out))
    text = out.read_text()
    # serving span: 4 launches, 40 ms busy over 25 ms covered
    assert "launches of the serving span: 4, mean 10.000 ms" in text
    assert "1.60 of them ran at once" in text
    assert "--workload serve" in text and "| scs_mixed_kernel<TrF32> | 5 |" in text


def test_paper_context_matches_the_decoder():
    c = bench.paper_context("scs")
    assert c["decoder"] == "SCS-RM" and c["mbps_per_thread"]["3.0"] == pytest.approx(0.23237)
    assert bench.paper_context("fsscs")["mbps_per_thread"]["3.0"] == pytest.approx(0.925226)
    assert bench.paper_context("fssc") is None
    assert all(len(v[1]) == len(bench.POINTS) for v in bench.PAPER_TP_MBPS.values())
