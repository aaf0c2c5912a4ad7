"""Host logic of the measurement helpers (no GPU): the HBM-traffic record
built from two counter runs, and the grouping of SQ counter dispatches.

The inputs are small synthetic rocprofv3 counter CSV files in the layout
the profiler writes (one row per dispatch, counter instance and counter).
"""
import csv
import json
import os

import pytest

import counters

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_csv(directory, rows):
    os.makedirs(directory, exist_ok=True)
    with open(os.path.join(directory, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for r in rows:
            full = {k: 0 for k in FIELDS}
            full.update(r)
            w.writerow(full)


def row(disp, kernel, counter, value, vgpr=36, sgpr=48, lds=5120, t0=0, t1=1000):
    return {"Dispatch_Id": disp, "Kernel_Name": kernel, "Counter_Name": counter,
            "Counter_Value": value, "VGPR_Count": vgpr, "SGPR_Count": sgpr,
            "LDS_Block_Size": lds, "Start_Timestamp": t0, "End_Timestamp": t1}


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    # the copy moves 4 MiB each way; the fetch counter reads half of it
    fetch = [row(1, "k_trace", "FETCH_SIZE", 999.0), row(2, "k_trace", "FETCH_SIZE", 100.0),
             row(3, "k_trace", "FETCH_SIZE", 300.0), row(4, "k_probe_copy", "FETCH_SIZE", 2048.0)]
    write = [row(1, "k_trace", "WRITE_SIZE", 5.0), row(2, "k_trace", "WRITE_SIZE", 50.0),
             row(3, "k_trace", "WRITE_SIZE", 70.0), row(4, "k_probe_copy", "WRITE_SIZE", 4096.0)]
    write_csv(tmp_path / "f", fetch)
    write_csv(tmp_path / "w", write)
    rec = counters.trace_traffic(str(tmp_path / "f"), str(tmp_path / "w"), copy_mib=4)
    # the first (warm-up) dispatch is dropped: fetch 200 KiB x 2, write 60 KiB x 1
    assert rec["fetch_kib_per_launch_raw"] == 200.0 and rec["write_kib_per_launch_raw"] == 60.0
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    assert rec["hbm_bytes_per_launch"] == (400 + 60) * 1024
    assert rec["dispatches"] == {"fetch": 2, "write": 2}


def sq_rows(disp, vgpr, valu, ns, sgpr=48, instances=2):
    """One dispatch: every SQ counter split over `instances` rows."""
    out = []
    for c in counters.COUNTERS:
        v = valu if c == "SQ_INSTS_VALU" else 10.0
        for _ in range(instances):
            out.append(row(disp, "k_trace", c, v / instances, vgpr=vgpr, sgpr=sgpr, t1=ns))
    return out


def test_sq_groups_by_resources_and_by_explicit_runs(tmp_path):
    rows = []
    valu = [100, 102, 101, 300, 310, 500, 520, 100]
    vgpr = [36, 36, 36, 48, 48, 48, 48, 36]
    for i, (v, g) in enumerate(zip(valu, vgpr)):
        rows += sq_rows(i + 1, g, float(v), 1000 * (i + 1))
    rows.append(row(99, "k_build_something", "SQ_INSTS_VALU", 1e9))  # other kernels are ignored
    write_csv(tmp_path / "sq", rows)
    ds = counters.dispatches(str(tmp_path / "sq"))
    assert len(ds) == 8
    assert ds[0]["SQ_INSTS_VALU"] == 100.0          # instances summed
    by_sig = counters.groups(ds)
    # two formats with the same resources run back to back merge into one group
    assert [g["dispatches"] for g in by_sig] == [3, 4, 1]
    runs = counters.groups(ds, [3, 2, 2, 1])
    assert [g["dispatches"] for g in runs] == [3, 2, 2, 1]
    assert [g["SQ_INSTS_VALU"] for g in runs] == [101.0, 305.0, 510.0, 100.0]   # medians
    assert runs[1]["ns"] == 4500.0
    with pytest.raises(ValueError):
        counters.groups(ds, [3, 2, 2])


def test_bench_reads_records_only_for_the_current_source(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    sha = bench.kernel_source_hash()
    rec = {"workload": "w", "node_format": "f4", "kernel_source_sha1": sha,
           "hbm_bytes_per_launch": 123, "groups": [{"SQ_INSTS_VALU": 7.0, "SQ_INSTS_VMEM_RD": 3.0}]}
    for name in ("trace_traffic.json", "trace_sq_counters.json"):
        with open(tmp_path / "profiles" / name, "w") as f:
            json.dump(rec, f)
    assert bench.load_traffic("w", "f4") == 123
    assert bench.load_sq("w", "f4") == {"valu_wave_instr": 7.0, "vmem_rd_wave_instr": 3.0}
    assert bench.load_traffic("other", "f4") is None
    # a record of another node format's launch is not this launch's
    assert bench.load_sq("w", "bin2") is None and bench.load_traffic("w", "q4") is None
    rec["kernel_source_sha1"] = "0" * 12
    with open(tmp_path / "profiles" / "trace_traffic.json", "w") as f:
        json.dump(rec, f)
    assert bench.load_traffic("w", "f4") is None


def test_roofline_prices_node_visits_by_format():
    import bench
    # per segment: ray + hit 48 B; a binary visit reads 64 B and tests two
    # boxes, a 4-wide visit 128 B (float32) or 64 B (8-bit) and four boxes
    kw = dict(trace_ms=1.0, segments=10, nodes_total=100, tests_total=20, sq=None, traffic=None,
              ceilings=None)
    alg = {f: bench.roofline(**kw, node_format=f)["algorithmic"] for f in ("bin2", "f4", "q4")}
    assert alg["bin2"]["bytes_per_launch"] == 10 * 48 + 100 * 64 + 20 * 36
    assert alg["f4"]["bytes_per_launch"] == 10 * 48 + 100 * 128 + 20 * 36
    assert alg["q4"]["bytes_per_launch"] == alg["bin2"]["bytes_per_launch"]
    assert alg["bin2"]["ops_per_launch"] == 100 * 2 * 18 + 20 * 45
    assert alg["f4"]["ops_per_launch"] == alg["q4"]["ops_per_launch"] == 100 * 4 * 18 + 20 * 45


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
