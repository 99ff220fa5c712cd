"""CPU checks of the rocprofv3 summary generator (paper_2406_16499_amd/profiling.py)
on synthetic CSV files: the calibration copy scales the raw counters to bytes,
counters reported over several dimensions are summed per dispatch and
dispatches are averaged, and the kernel table is sorted by total time with
short kernel names."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2406_16499_amd import profiling  # noqa: E402


def _counters(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    copy_kib = bench.COPY_BYTES / 1024.0
    # the copy reads twice its bytes on the fetch counter and its bytes on the
    # write counter; the kernel has two dispatches, each split over two dimensions
    fetch = [("1", "k_copy16(float4 const*, float4*, long)", 2 * copy_kib),
             ("2", "void lsq::k_panel_final_y<float, float>(double const*)", 300.0),
             ("2", "void lsq::k_panel_final_y<float, float>(double const*)", 100.0),
             ("3", "void lsq::k_panel_final_y<float, float>(double const*)", 600.0),
             ("4", "k_other(int)", 5.0)]
    write = [("1", "k_copy16(float4 const*, float4*, long)", copy_kib),
             ("2", "void lsq::k_panel_final_y<float, float>(double const*)", 250.0),
             ("3", "void lsq::k_panel_final_y<float, float>(double const*)", 350.0)]
    fp, wp = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    _counters(fp, "FETCH_SIZE", fetch)
    _counters(wp, "WRITE_SIZE", write)
    out = str(tmp_path / "t.txt")
    text = profiling.traffic_summary(fp, wp, "panel_final_y", "k_panel_final_y<float", "cf", "cw", out)
    kv = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("#"))
    assert kv["dispatches_fetch"] == "2" and kv["dispatches_write"] == "2"
    assert float(kv["fetch_scale"]) == 0.5 and float(kv["write_scale"]) == 1.0
    # fetch: (400 + 600) / 2 = 500 KiB raw -> 250 KiB; write: 300 KiB
    assert float(kv["hbm_bytes_per_launch"]) == (250.0 + 300.0) * 1024.0
    assert kv["source_hash"] == bench.source_hash(None)
    assert open(out).read() == text


def test_stats_table_sorted_with_short_names(tmp_path):
    path = str(tmp_path / "s.csv")
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": "void lsq::k_small<float>(int)", "Calls": 2, "TotalDurationNs": 1000,
                    "AverageNs": 500, "MinNs": 400, "MaxNs": 600})
        w.writerow({"Name": "void lsq::k_big<double, (lsq::Mma)0>(double const*, int)", "Calls": 1,
                    "TotalDurationNs": 3000, "AverageNs": 3000, "MinNs": 3000, "MaxNs": 3000})
    text = profiling.stats_summary(path, "cmd", str(tmp_path / "o.txt"))
    body = [l for l in text.splitlines()[4:] if l.strip()]
    assert body[0].startswith("k_big<double, (Mma)0>") and body[1].startswith("k_small<float>")
    assert body[0].split()[-1] == "75.00" and body[1].split()[-1] == "25.00"
