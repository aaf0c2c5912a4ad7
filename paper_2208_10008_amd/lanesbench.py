"""Lanes per ray on the paper-size scenes: trace time for every lane count.

For the two paper-size stand-in scenes (study room, 2,778 facets; campus,
7,608 facets; Sec. IV), binary and 8-bit node trees with leaves of 16, 64
and the paper's own size (250 / 820 facets), and icosphere levels 3-9
(642 to 2,621,442 rays), times rt_trace_ex with lanes_per_ray 1, 4, 16, 64
and 0 (the library's choice) over the paper's reflection order (HIP events
over 10 launches after one untimed launch).  Prints one line per case to
stderr and a JSON document with every time, the library's choice and the
fastest lane count to stdout.

    python3 -m paper_2208_10008_amd.lanesbench > lanes.json
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--levels", default="3-9")
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args()
    import torch

    from . import BVH, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    lo, hi = (int(x) for x in a.levels.split("-"))
    levels = list(range(lo, hi + 1))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / a.reps

    dirs = torch.from_numpy(icosphere.directions(max(levels)).astype(np.float32)).cuda()
    res = {"command": "python3 -m paper_2208_10008_amd.lanesbench", "cases": []}
    for w in (workloads.paper_indoor(), workloads.paper_outdoor()):
        tris = torch.from_numpy(w.tris).cuda()
        nb = w.max_bounces
        for fmt in ("bin2", "q4"):
            for leaf in (w.max_leaf, 64, 16):
                bvh = BVH(tris, SplitParams(alpha=w.alpha, src=w.tx, max_leaf=leaf, node_format=fmt))
                for lv in levels:
                    n = icosphere.vertex_count(lv)
                    rays = rt_rays_from_directions(dirs, n, w.tx, 1e-4, w.tmax)
                    out = bvh.hits_buffer(n, nb)
                    pl = torch.empty(n, dtype=torch.float64, device="cuda")
                    nh = torch.empty(n, dtype=torch.int32, device="cuda")
                    ms = {}
                    for g in (1, 4, 16, 64, 0):
                        ms[str(g)] = round(timed(lambda: bvh.trace_bounces(
                            rays, nb, out, pl, nh, lanes_per_ray=g)), 4)
                    best = min(("1", "4", "16", "64"), key=lambda k: ms[k])
                    case = {"scene": w.name, "format": fmt, "max_leaf": leaf, "level": lv,
                            "rays": n, "ms": ms, "fastest": int(best)}
                    res["cases"].append(case)
                    print(f"[lanes] {w.name} {fmt} leaf {leaf} L{lv}: {ms} fastest G={best}",
                          file=sys.stderr, flush=True)
                bvh.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
