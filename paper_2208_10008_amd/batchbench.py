"""Batched trace of the multi-scene set: 8 scenes (1k-200k facets), 64
transmitters at icosphere levels 6-9 with 1-6 bounces, all in one autotuned,
graph-captured launch; once per node format, with the hits of the formats
checked equal.

    python -m paper_2208_10008_amd.batchbench

prints one JSON line: per format the time per launch and segments per
second, and the autotuned launch shape.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--formats", default="bin2,f4,q4")
    a = ap.parse_args()
    import torch

    from . import BVH, Batch, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    def say(*m):
        print("[batch]", *m, file=sys.stderr, flush=True)

    qdefs = workloads.multiscene_queries()
    scenes = [torch.from_numpy(workloads.multiscene_scene(s)[0]).cuda() for s in range(8)]
    dirs = torch.from_numpy(icosphere.directions(9).astype(np.float32)).cuda()
    rays = [rt_rays_from_directions(dirs, icosphere.vertex_count(lv), tx, 1e-4, 2000.0)
            for _, tx, lv, _ in qdefs]
    nrays = sum(r.shape[0] for r in rays)
    say(len(qdefs), "queries,", nrays, "rays")
    result = {"workload": f"8 scenes (1k-200k facets), {len(qdefs)} transmitters, "
                          f"levels 6-9 ({nrays} rays), 1-6 bounces",
              "command": "python3 -m paper_2208_10008_amd.batchbench", "formats": {}}
    ref = None
    for fmt in a.formats.split(","):
        trees = [BVH(t, SplitParams(alpha=0.4, src=workloads.MULTI_SRC, node_format=fmt))
                 for t in scenes]
        qs = [{"bvh": trees[s], "rays": r, "max_bounces": nb}
              for (s, _, _, nb), r in zip(qdefs, rays)]
        b = Batch(len(qs))
        b.set(qs)
        b.autotune(reps=2)
        b.configure(**{**b.config(), "graph": True})
        b.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.reps):
            b.launch()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        segs = sum(int(torch.clamp(q["n_hits"] + 1, max=q["max_bounces"]).sum().item()) for q in qs)
        same = None
        if ref is None:
            ref = [q["out"].clone() for q in qs]
        else:
            same = all(torch.equal(q["out"], r) for q, r in zip(qs, ref))
        result["formats"][fmt] = {"ms_per_launch": round(ms, 3), "segments": segs,
                                  "mrays_s": round(segs / (ms * 1e-3) / 1e6, 1),
                                  "launch": b.config(), "hits_equal_to_first_format": same}
        say(fmt, result["formats"][fmt])
        b.close()
        for t in trees:
            t.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
