"""HBM traffic of the trace kernel from two rocprofv3 counter runs.

Usage (after two runs of the same bench command, one with ``--pmc FETCH_SIZE``
and one with ``--pmc WRITE_SIZE``, each writing CSV into its own directory)::

    python -m paper_2208_10008_amd.traffic --fetch DIR1 --write DIR2 \
        --copy-mib 1024 --workload NAME --out profiles/trace_traffic.json

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  Each is scaled
by the ratio of the bytes the calibration copy (k_probe_copy, which reads and
writes ``copy_mib`` MiB) really moves to what the same counter reports for it.
The record carries the SHA-1 of the trace kernel's source so that a later
change to the kernel invalidates it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TRACE_SRC = os.path.join(HERE, "csrc", "rt_trace.hip")


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    rec = trace_traffic(a.fetch, a.write, a.copy_mib)
    rec = {"workload": a.workload, "kernel": "k_trace", "kernel_source_sha1": source_sha1(),
           "command": a.command, **rec}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
