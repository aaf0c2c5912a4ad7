"""Paper-regime comparison (Sec. IV, Fig. 9 analogue): running time against
the number of launched rays for the traditional split (Eq. (1): alpha = 1)
and the proposed one (Eq. (2)) on the two paper-size scenes:

* indoor: study room 8 x 6 x 3.5 m, 2,778 facets, 250 facets per leaf,
  alpha 0.7, reflection orders up to 2, Tx (1.46, 2.42, 2.1), Rx (1.2, 1.2, 1.5);
* outdoor: campus, 7,608 facets, 820 facets per leaf, alpha 0.4, reflection
  order up to 3, Tx (450, 450, 10), Rx (450, 550, 25).

    python -m paper_2208_10008_amd.paperbench [--levels 3-9] [--reps 10]

Per scene, split and icosphere level: GPU time of one step (rt_rebuild of
the tree for this Tx + rt_trace_receive at the Rx) from HIP events, facet
tests and node visits per segment (instrumented launch, outside the timed
region), the paths received at the Rx (after duplicate grouping); the
CPU checker's time for the same chains (its own float64 traversal of the
same tree, all host threads) on the levels it finishes quickly; and, for
context, the GPU at its own leaf size (4).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--levels", default="3-9")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--cpu-levels", default="3-6")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    import torch

    from . import BVH, Receivers, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    def lv_range(s):
        lo, hi = (int(x) for x in s.split("-"))
        return list(range(lo, hi + 1))

    def say(*m):
        print("[paper]", *m, file=sys.stderr, flush=True)

    levels = lv_range(a.levels)
    dirs = torch.from_numpy(icosphere.directions(max(levels)).astype(np.float32)).cuda()
    res = {"command": "python3 -m paper_2208_10008_amd.paperbench", "scenes": {}}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    for w in (workloads.paper_indoor(), workloads.paper_outdoor()):
        tris = torch.from_numpy(w.tris).cuda()
        rx = torch.tensor([w.rx], dtype=torch.float64, device="cuda")
        nb = w.max_bounces
        sc = {"facets": int(w.tris.shape[0]), "tx": list(w.tx), "rx": list(w.rx),
              "max_leaf": w.max_leaf, "alpha": w.alpha, "max_order": w.max_order, "runs": {}}
        for tag, alpha, leaf in (("traditional", 1.0, w.max_leaf), ("proposed", w.alpha, w.max_leaf),
                                 ("traditional_leaf4", 1.0, 4), ("proposed_leaf4", w.alpha, 4)):
            p = SplitParams(alpha=alpha, src=w.tx, max_leaf=leaf)
            bvh = BVH(tris, p)
            info = bvh.info()
            t_build = timed(lambda: bvh.rebuild(tris, p), a.reps)
            run = {"alpha": alpha, "max_leaf": leaf, "nodes": int(info.n_nodes),
                   "depth": int(info.depth), "build_ms": round(t_build, 4), "levels": {}}
            for lv in levels:
                n = icosphere.vertex_count(lv)
                rays = rt_rays_from_directions(dirs, n, w.tx, 1e-4, w.tmax)
                delta = float(icosphere.edge_angles(lv).mean())
                recv = Receivers(rx, delta, 1 << 16)
                out = bvh.hits_buffer(n, nb)
                pl = torch.empty(n, dtype=torch.float64, device="cuda")
                nh = torch.empty(n, dtype=torch.int32, device="cuda")
                t_tr = timed(lambda: bvh.trace_receive(rays, nb, recv, out, pl, nh), a.reps)
                recv.dedup(out, nb)
                rec = recv.records()
                kept = rec[rec["keep"] == 1]
                stats = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
                bvh.trace_bounces(rays, nb, ray_stats=stats)
                segs = int(torch.clamp(nh.long() + 1, max=nb).sum().item())
                st = stats.double().sum(0).cpu().numpy() / max(segs, 1)
                run["levels"][str(lv)] = {
                    "rays": n, "segments": segs, "trace_ms": round(t_tr, 4),
                    "step_ms": round(t_build + t_tr, 4),
                    "nodes_per_segment": round(float(st[0]), 2),
                    "tests_per_segment": round(float(st[1]), 2),
                    "receptions": int(rec.size), "paths": int(kept.size),
                    "paths_by_order": np.bincount(kept["order"], minlength=nb).tolist()}
            say(w.name, tag, {k: (v["trace_ms"], v["tests_per_segment"], v["paths"])
                              for k, v in run["levels"].items()})
            sc["runs"][tag] = run
            bvh.close()
        if not a.no_cpu:
            import oracle
            threads = min(16, os.cpu_count() or 1)
            cpu = {}
            for tag, alpha in (("traditional", 1.0), ("proposed", w.alpha)):
                tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=alpha, src=w.tx,
                                                                    max_leaf=w.max_leaf))
                cpu[tag] = {}
                for lv in lv_range(a.cpu_levels):
                    r = w.rays(lv)
                    t0 = time.perf_counter()
                    oracle.bounces(w.tris, r, nb, tree=tree, nthreads=threads, segments=False)
                    cpu[tag][str(lv)] = round((time.perf_counter() - t0) * 1e3, 2)
            sc["cpu_checker_ms"] = cpu
            sc["cpu_threads"] = threads
            say(w.name, "cpu", cpu)
        res["scenes"][w.name] = sc
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
