"""Instruction counts of the trace kernel from a rocprofv3 SQ counter run.

Usage (after one run of a bench command under ``rocprofv3 --pmc SQ_WAVES
SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_WAVE_CYCLES
SQ_BUSY_CYCLES SQ_INSTS_SMEM -T -f csv -d DIR``)::

    python -m paper_2208_10008_amd.sqcount --dir DIR --workload NAME --out profiles/trace_sq_counters.json

``--runs 14,12,12,13`` splits the dispatches in order into runs of those
lengths instead (the bench command above launches 14 binary-node traces,
then 12 of each node format after the first, then 13 for the alpha
comparison), for formats whose kernels need the same resources.

Every trace-kernel dispatch is summed over the counter's instances; runs of
consecutive dispatches with the same resources (vector and scalar register
counts and LDS size: one node format, one tree) are grouped in dispatch
order, each group keeping its per-dispatch median.  The record carries the same source hash as the traffic record, so a
change to the kernel invalidates it.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import statistics

from .traffic import source_sha1

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
    ap.add_argument("--dir", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--runs", default="", help="comma-separated dispatch counts of the runs, in order")
    a = ap.parse_args()
    runs = [int(x) for x in a.runs.split(",") if x]
    rec = {"workload": a.workload, "kernel": "k_trace", "kernel_source_sha1": source_sha1(),
           "command": a.command, "groups": groups(dispatches(a.dir), runs)}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
