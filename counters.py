#!/usr/bin/env python3
"""Hardware counters of the trace kernel, from rocprofv3 CSV output.

Two records under profiles/, each carrying the SHA-1 of the trace kernel's
source (rt_trace.hip and rt_internal.h) so that bench.py ignores them once the
kernel changes:

* HBM traffic (``traffic``): two runs of the same bench command, one with
  ``--pmc FETCH_SIZE`` and one with ``--pmc WRITE_SIZE`` (KiB per dispatch),
  each scaled by what the counter reads for a plain copy of known size
  (k_probe_copy, bench.py --copy-mib)::

    python3 counters.py traffic --fetch DIR1 --write DIR2 --copy-mib 1024 \
        --workload NAME --out profiles/trace_traffic.json

* instruction counts (``sq``): one run under ``rocprofv3 --pmc SQ_WAVES
  SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_WAVE_CYCLES
  SQ_BUSY_CYCLES SQ_INSTS_SMEM``.  Every trace-kernel dispatch is summed over
  the counter's instances; runs of consecutive dispatches with the same
  resources (vector and scalar registers, LDS: one node format, one tree)
  are grouped in dispatch order, each keeping its per-dispatch median, or
  ``--runs 14,12,12`` splits the dispatches in order into runs of those
  lengths::

    python3 counters.py sq --dir DIR --workload NAME --out profiles/trace_sq_counters.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.abspath(__file__))
TRACE_SRC = os.path.join(ROOT, "paper_2208_10008_amd", "csrc", "rt_trace.hip")


def source_sha1(path: str = TRACE_SRC) -> str:
    """SHA-1 (12 hex digits) of the trace kernel's source and of the internal
    header it compiles with."""
    h = hashlib.sha1()
    for p in (path, os.path.join(os.path.dirname(path), "rt_internal.h")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def counter_values(directory: str, counter: str) -> dict:
    """Kernel name -> list of per-dispatch counter values (dispatch order)."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    out: dict = {}
    for _, name, v in rows:
        out.setdefault(name.split("(")[0].split("<")[0].strip(), []).append(v)
    return out


def trace_traffic(fetch_dir: str, write_dir: str, copy_mib: int, kernel: str = "k_trace") -> dict:
    f = counter_values(fetch_dir, "FETCH_SIZE")
    w = counter_values(write_dir, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    f_copy, w_copy = f["k_probe_copy"][-1], w["k_probe_copy"][-1]
    f_scale, w_scale = copy_kib / f_copy, copy_kib / w_copy
    # steady-state trace launches: drop the first (warm-up) dispatch
    ft = f[kernel][1:] or f[kernel]
    wt = w[kernel][1:] or w[kernel]
    f_kib = sum(ft) / len(ft)
    w_kib = sum(wt) / len(wt)
    return {
        "fetch_kib_per_launch_raw": round(f_kib, 1),
        "write_kib_per_launch_raw": round(w_kib, 1),
        "calibration": {"copy_mib": copy_mib, "fetch_kib_raw": f_copy, "write_kib_raw": w_copy,
                        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
        "hbm_bytes_per_launch": int(round((f_kib * f_scale + w_kib * w_scale) * 1024)),
        "dispatches": {"fetch": len(ft), "write": len(wt)},
    }


COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS",
            "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_INSTS_SMEM")


def dispatches(directory: str, kernel_prefix: str = "k_trace"):
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    d = collections.OrderedDict()
    for path in files:
        with open(path) as f:
            for r in csv.DictReader(f):
                if not r["Kernel_Name"].startswith(kernel_prefix):
                    continue
                key = int(r["Dispatch_Id"])
                e = d.setdefault(key, {"vgpr_granules": int(r["VGPR_Count"]),
                                       "sig": (r["VGPR_Count"], r["SGPR_Count"], r["LDS_Block_Size"]),
                                       "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
                e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [d[k] for k in sorted(d)]


def groups(ds, runs=None):
    out = []
    if runs:
        if sum(runs) != len(ds):
            raise ValueError(f"--runs sums to {sum(runs)}, the directory holds {len(ds)} dispatches")
        k = 0
        for n in runs:
            out.append({"vgpr_granules": ds[k]["vgpr_granules"], "items": ds[k:k + n]})
            k += n
    for e in ds if not runs else ():
        if out and out[-1]["sig"] == e["sig"]:
            out[-1]["items"].append(e)
        else:
            out.append({"vgpr_granules": e["vgpr_granules"], "sig": e["sig"], "items": [e]})
    res = []
    for g in out:
        rec = {"vgpr_granules": g["vgpr_granules"], "dispatches": len(g["items"])}
        for c in COUNTERS + ("ns",):
            vals = [e[c] for e in g["items"] if c in e]
            if vals:
                rec[c] = statistics.median(vals)
        res.append(rec)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    a1 = sub.add_parser("traffic", help="HBM bytes per trace launch")
    a1.add_argument("--fetch", required=True)
    a1.add_argument("--write", required=True)
    a1.add_argument("--copy-mib", type=int, required=True)
    a2 = sub.add_parser("sq", help="instruction counts per trace launch")
    a2.add_argument("--dir", required=True)
    a2.add_argument("--runs", default="", help="comma-separated dispatch counts of the runs, in order")
    for p in (a1, a2):
        p.add_argument("--workload", required=True)
        p.add_argument("--node-format", default="bin2", choices=["bin2", "f4", "q4"],
                       help="node format of the benchmark's launch (the record's first run)")
        p.add_argument("--command", default="")
        p.add_argument("--out", required=True)
    a = ap.parse_args()
    head = {"workload": a.workload, "node_format": a.node_format, "kernel": "k_trace",
            "kernel_source_sha1": source_sha1(),
            "command": a.command}
    if a.what == "traffic":
        rec = {**head, **trace_traffic(a.fetch, a.write, a.copy_mib)}
    else:
        runs = [int(x) for x in a.runs.split(",") if x]
        rec = {**head, "groups": groups(dispatches(a.dir), runs)}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
