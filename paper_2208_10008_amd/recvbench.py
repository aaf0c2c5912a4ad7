"""Receiving-sphere reception (Sec. III-C, Eq. (4)) on the city24k launch:
2,000 buildings (about 24k facets), Tx (0, 0, 25), level-9 icosphere
(2,621,442 rays), up to 6 segments, field points outside the buildings
within 400 m of the Tx, delta = mean angle between adjacent launch
directions.

    python -m paper_2208_10008_amd.recvbench [--receivers 1,16,64,256] [--reps 10]

Times with HIP events on the launching stream:
  * the chains alone (rt_trace_bounces);
  * the chains with every segment tested as it is traced (rt_trace_receive),
    per number of field points;
  * the stored-chain kernel (rt_receive_segments) over the tracer's segment
    output, and the duplicate grouping (rt_receive_dedup).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

# float64 operations of one segment-field point test (Eq. (4) as evaluated:
# w 3, w.d 5, s 1 div, p 6, dist^2 5, |w|^2 5 + 1 sqrt, l 1, rr 1, 3 dist^2 1,
# rr^2 1, two range compares and one threshold compare not counted)
FP64_OPS_PER_TEST = 30
BYTES_PER_SEGMENT = 32 + 16  # stored segment ray + its hit record


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--receivers", default="1,16,64,256")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--dedup-receivers", type=int, default=64)
    ap.add_argument("--thresholds", default="1e-9,1e-10,1e-11,0")
    a = ap.parse_args()
    import torch

    from . import BVH, Energy, Receivers, SplitParams, rt_receive_segments
    from rtgen import icosphere, workloads

    def say(*m):
        print("[recv]", *m, file=sys.stderr, flush=True)

    w = workloads.city24k()
    nb = w.max_bounces
    delta = float(icosphere.edge_angles(w.level).mean())
    bvh = BVH(torch.from_numpy(w.tris).cuda(), SplitParams(alpha=0.4, src=w.tx))
    rays = torch.from_numpy(w.rays).cuda()
    n = w.n_rays
    out = bvh.hits_buffer(n, nb)
    pl = torch.empty(n, dtype=torch.float64, device="cuda")
    nh = torch.empty(n, dtype=torch.int32, device="cuda")

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

    t_trace = timed(lambda: bvh.trace_bounces(rays, nb, out, pl, nh))
    segs = int(torch.clamp(nh.long() + 1, max=nb).sum().item())
    say(f"chains alone {t_trace:.3f} ms, {segs} segments")
    res = {"workload": f"city24k: {w.n_tris} facets, {n} rays (level {w.level}), up to {nb} "
                       f"segments, delta {delta:.6g} rad",
           "command": "python3 -m paper_2208_10008_amd.recvbench", "segments": segs,
           "trace_ms": round(t_trace, 4), "fused": {}, "stored": {}}
    counts = [int(x) for x in a.receivers.split(",")]
    for k in sorted(set(counts + [a.dedup_receivers])):
        pts = torch.from_numpy(workloads.field_points(w.tris, 400.0, k, 100 + k)).cuda()
        recv = Receivers(pts, delta, 1 << 20)
        t = timed(lambda: bvh.trace_receive(rays, nb, recv, out, pl, nh))
        c = recv.count()
        res["fused"][str(k)] = {"ms": round(t, 4), "overhead": round(t / t_trace - 1, 4),
                                "receptions": c}
        say(f"fused, {k} field points: {t:.3f} ms ({c} receptions)")
    # stored chains: the tracer writes every segment, then the kernel reads them
    seg = torch.empty((nb, n, 8), dtype=torch.float32, device="cuda")
    t_seg = timed(lambda: bvh.trace_bounces(rays, nb, out, pl, nh, seg_rays=seg))
    res["stored"]["trace_with_segments_ms"] = round(t_seg, 4)
    for k in sorted(set(counts)):
        pts = torch.from_numpy(workloads.field_points(w.tris, 400.0, k, 100 + k)).cuda()
        recv = Receivers(pts, delta, 1 << 20)
        t = timed(lambda: rt_receive_segments(seg, out, nb, recv))
        tests = segs * k
        gbs = segs * BYTES_PER_SEGMENT / (t * 1e-3) / 1e9
        tf = tests * FP64_OPS_PER_TEST / (t * 1e-3) / 1e12
        res["stored"][str(k)] = {"ms": round(t, 4), "receptions": recv.count(),
                                 "gb_s": round(gbs, 1), "hbm_frac": round(gbs / 8000.0, 4),
                                 "fp64_tflop_s": round(tf, 2), "fp64_frac": round(tf / 78.6, 4)}
        say(f"stored-chain kernel, {k} field points: {t:.3f} ms, {gbs:.0f} GB/s, {tf:.2f} TF/s fp64")
    k = a.dedup_receivers
    pts = torch.from_numpy(workloads.field_points(w.tris, 400.0, k, 100 + k)).cuda()
    recv = Receivers(pts, delta, 1 << 20)
    rt_receive_segments(seg, out, nb, recv)
    t = timed(lambda: recv.dedup(out, nb))
    rec = recv.records()
    res["dedup"] = {"field_points": k, "ms": round(t, 4), "receptions": int(rec.size),
                    "kept": int(rec["keep"].sum())}
    say(f"dedup, {k} field points: {t:.3f} ms, {rec.size} -> {int(rec['keep'].sum())}")
    del seg
    mat = torch.from_numpy(workloads.city_materials(w.n_tris, 0)).cuda()
    refl = torch.from_numpy(workloads.REFLECTION).cuda()
    res["energy"] = {"k0": workloads.free_space_k0(), "reflection": workloads.REFLECTION.tolist(),
                     "thresholds": {}}
    for thr in (float(x) for x in a.thresholds.split(",")):
        en = Energy(mat, refl, workloads.free_space_k0(), thr,
                    power=torch.empty(n, dtype=torch.float64, device="cuda"))
        t = timed(lambda: bvh.trace_energy(rays, nb, en, out=out, path_len=pl, n_hits=nh))
        hits = nh.long()
        stopped = (en.power < thr) & (hits > 0)
        segs_e = int(torch.where(stopped, hits, torch.clamp(hits + 1, max=nb)).sum().item())
        res["energy"]["thresholds"][repr(thr)] = {
            "ms": round(t, 4), "segments": segs_e, "vs_fixed_order": round(t / t_trace, 4),
            "stopped_by_energy": round(float(stopped.double().mean().item()), 4),
            "mrays_s": round(segs_e / (t * 1e-3) / 1e6, 1)}
        say(f"energy stop at {thr:g}: {t:.3f} ms, {segs_e} segments, "
            f"{float(stopped.double().mean().item()):.3f} stopped by energy")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
