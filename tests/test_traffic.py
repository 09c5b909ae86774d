"""Host logic of the HBM-traffic summary (paper_2107_03958_amd/traffic.py) on
synthetic rocprofv3 counter files: the copy calibration, the per-dispatch
averages, kernel-name parsing and the source-hash gate.  CPU only."""
import csv
import json
import os

from paper_2107_03958_amd import traffic

HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEADER)
        for i, (name, value) in enumerate(rows):
            w.writerow([i + 1, name, counter, value])


def test_summarise_scales_by_the_copy(tmp_path):
    copy_kib = traffic.COPY_BYTES / 1024
    kern = "void ws::k_pass1<double, 1, 11, 2>(void const*, void*)"
    fetch_dir, write_dir = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the copy reads half its bytes in FETCH_SIZE units (scale 2) and writes all (scale 1)
    _write_counters(fetch_dir, "FETCH_SIZE", [(kern, 100.0), (kern, 200.0), ("__amd_rocclr_copyBuffer", copy_kib / 2)])
    _write_counters(write_dir, "WRITE_SIZE", [(kern, 40.0), (kern, 60.0), ("__amd_rocclr_copyBuffer", copy_kib)])
    with open(fetch_dir + ".log", "w") as fh:
        fh.write("noise\n" + json.dumps({"target": "done", "chunk": 3}) + "\n")
    res = traffic.summarise(fetch_dir, write_dir, str(tmp_path / "out"))
    assert res["densities_per_dispatch"] == 3
    assert res["fetch_scale"] == 2.0 and res["write_scale"] == 1.0
    k = res["kernels"]["ws::k_pass1<double, 1, 11, 2>"]
    assert k["read_bytes"] == 150.0 * 1024 * 2.0
    assert k["write_bytes"] == 50.0 * 1024
    assert k["traffic_bytes"] == k["read_bytes"] + k["write_bytes"]
    assert list(res["kernels"]) == ["ws::k_pass1<double, 1, 11, 2>"]     # the copy is not a kernel of the path
    assert os.path.exists(str(tmp_path / "out.md"))


def test_summary_gated_by_source_hash(tmp_path):
    path = str(tmp_path / "s.json")
    with open(path, "w") as fh:
        json.dump({"source_hash": traffic.source_hash(), "kernels": {}}, fh)
    assert traffic.load_for_current_sources(path) is not None
    with open(path, "w") as fh:
        json.dump({"source_hash": "0" * 16, "kernels": {}}, fh)
    assert traffic.load_for_current_sources(path) is None
    assert traffic.load_for_current_sources(str(tmp_path / "missing.json")) is None


def test_stats_summary_filters_and_sorts(tmp_path):
    path = str(tmp_path / "k_kernel_stats.csv")
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void ws::k_pass1<double, 1, 11, 2>(void const*)", 10, 1000, 100.0, 50.0, 90.0, 110.0, 1])
        w.writerow(["void ws::k_pass1<double, 0, 11, 2>(void const*)", 10, 600, 60.0, 30.0, 50.0, 70.0, 1])
        w.writerow(["void ws::k_pass1<float, 1, 11, 2>(void const*)", 5, 300, 60.0, 15.0, 60.0, 60.0, 1])
        w.writerow(["__amd_rocclr_copyBuffer", 4, 100, 25.0, 5.0, 25.0, 25.0, 1])
    out = str(tmp_path / "s.md")
    rows = traffic.stats_summary(path, out, "title", "rocprofv3 cmd", r"k_pass1<double")
    assert [r["name"] for r in rows] == ["ws::k_pass1<double, 1, 11, 2>", "ws::k_pass1<double, 0, 11, 2>"]
    assert rows[0]["kind"].startswith("column pass") and rows[0]["avg_us"] == 0.1
    text = open(out).read()
    assert "rocprofv3 cmd" in text and "float" not in text
    assert len(traffic.stats_summary(path, out, "t", "c")) == 3          # every ws:: kernel, not the copy
