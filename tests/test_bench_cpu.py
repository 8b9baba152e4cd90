"""Host logic of bench.py (CPU only): the algorithmic byte count behind
roofline.achieved, the rocprofv3 summaries behind roofline.traffic and the
committed profiles, the source-hash check on stale counters, and the
one-GPU rule."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_closed_form():
    # 6 undirected pairs (4 row transfers each), 4 one-way pairs (3), 2
    # gathers with 5 sources (one read per source, one write per target),
    # rows of n = 100 nodes = 2 words; the schedule once
    st = {"pairs": 10, "directed_pairs": 4, "gathers": 2, "gather_sources": 5, "levels": 3}
    rows = 4 * 6 + 3 * 4 + 5 + 2
    sched = 8 * 10 + 4 * (2 * 2 + 1 + 5) + 8 * (3 + 1)
    assert bench.algorithmic_bytes(st, 100) == rows * 16 + sched


def _write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def test_summarize_pmc_scales_by_the_copy(tmp_path):
    # the copy of 1 GiB reads 524,288 KiB of FETCH_SIZE (factor 2) and
    # writes 1,048,576 KiB of WRITE_SIZE (factor 1); two launches of two
    # dispatches each
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    kern = "void tn::k_rowor_global<8, 10>(...)"
    _write_csv(fetch, [
        {"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": "524288"},
        {"Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": "100"},
        {"Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": "300"},
        {"Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": "200"},
        {"Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": "200"}])
    _write_csv(write, [
        {"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": "1048576"},
        {"Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": "50"},
        {"Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": "50"},
        {"Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": "50"},
        {"Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": "50"}])
    rec = bench.summarize_pmc(str(fetch), str(write), "rowor", "w", "cmd", 1024, per_launch=2)
    assert rec["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert rec["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    assert rec["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(1024 * 2.0 * 800 / 2)
    assert rec["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(1024 * 1.0 * 200 / 2)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(1024 * (800 + 100))
    # only the last dispatch (the timed launch)
    rec1 = bench.summarize_pmc(str(fetch), str(write), "rowor", "w", "cmd", 1024, last=1)
    assert rec1["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(1024 * 2.0 * 200)


def test_summarize_trace_groups_the_last_launches(tmp_path):
    stats, trace = tmp_path / "s.csv", tmp_path / "t.csv"
    _write_csv(stats, [{"Name": "k_a", "Calls": "4", "AverageNs": "1000000",
                        "TotalDurationNs": "4000000", "Percentage": "100"}])
    rows = []
    for i, dur in enumerate([5, 7, 1, 2, 3, 4]):  # ms; the last four are two launches
        rows.append({"Dispatch_Id": str(i), "Kernel_Name": "void k_a<1>(...)",
                     "Start_Timestamp": str(10**9 * i), "End_Timestamp": str(10**9 * i + dur * 10**6)})
    _write_csv(trace, rows)
    text = bench.summarize_trace(str(stats), "cmd", trace_csv=str(trace), match="k_a", last=4,
                                 per_launch=2)
    assert "last 2 launches of 2 dispatches of k_a" in text
    assert "mean 5.000 ms, each 3.000, 7.000 ms" in text


def test_traffic_only_from_counters_of_the_current_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_source_sha": "abc", "hbm_bytes_per_launch": 123.0}
    (tmp_path / "profiles" / "rowor_w_pmc.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda files: "abc")
    assert bench.load_traffic("rowor", "w") == 123.0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda files: "changed")
    assert bench.load_traffic("rowor", "w") is None
    assert bench.load_traffic("rowor", "other") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_summarize_pmc_adds_the_kernels_of_one_launch(tmp_path):
    # the saturating path of a large network is five dispatches of four
    # kernels per launch; other kernels between them are not counted
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    names = ["void tn::k_rowor_global<8, 10, true, true, false, true>(...)",
             "void tn::k_rowor_fwd<8, 7, true>(...)",
             "void tn::k_slice_full_state<4>(...)",
             "tn::k_slice_order(unsigned int const*, unsigned int, unsigned int, unsigned int*)",
             "void tn::k_rowor_global<4, 5, true, true, false, false>(...)"]
    rows_f = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE",
               "Counter_Value": "524288"}]
    rows_w = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE",
               "Counter_Value": "1048576"}]
    for name, v in zip(names, (1, 10, 100, 1000, 10000)):
        rows_f.append({"Kernel_Name": name, "Counter_Name": "FETCH_SIZE", "Counter_Value": str(v)})
        rows_w.append({"Kernel_Name": name, "Counter_Name": "WRITE_SIZE", "Counter_Value": str(v)})
        rows_f.append({"Kernel_Name": "tn::k_out_sizes(...)", "Counter_Name": "FETCH_SIZE",
                       "Counter_Value": "7"})
    _write_csv(fetch, rows_f)
    _write_csv(write, rows_w)
    rec = bench.summarize_pmc(str(fetch), str(write), "rowor", "w", "cmd", 1024, last=5,
                              per_launch=5)
    assert rec["kernel"] == bench.ROWOR_SAT_KERNELS
    assert rec["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(1024 * 2.0 * 11111)
    assert rec["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(1024 * 1.0 * 11111)


def test_counter_roofline_is_a_bandwidth():
    # counted bytes over the launch time against the HBM peak; the plain
    # recurrence's bytes only as a dense equivalent, apart
    r = bench.counter_roofline(8e9, 2.0, "k", 1e15, 5e5, "global")
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    assert r["dense_equivalent"]["bytes"] == 1e15
    empty = bench.counter_roofline(None, 2.0, "k", 1e15, 5e5, "lds")
    assert empty["achieved"] is None and empty["frac"] is None
