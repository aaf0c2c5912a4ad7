"""After-trace stages on the city24k launch: 2,000 buildings (about 24k
facets), Tx (0, 0, 25), level-9 icosphere (2,621,442 rays), up to 6
segments; delta = mean angle between adjacent launch directions.

    python -m paper_2208_10008_amd.recvbench [--receivers 1,16,64,256] [--reps 10]

Times with HIP events on the launching stream:
  * the chains alone (rt_trace_bounces);
  * receiving spheres (Sec. III-C, Eq. (4)), field points outside the
    buildings within 400 m of the Tx: the chains with every segment tested as
    it is traced (rt_trace_receive) per number of field points; the
    stored-chain kernel (rt_receive_segments) over the tracer's segment
    output; the duplicate grouping (rt_receive_dedup);
  * edge diffraction (Sec. III-B): wedge extraction (rt_wedges, host clock of
    the synchronising call), the diffraction pass over the stored chains
    (rt_diffract_segments, 16 cone directions) and one closest-hit segment
    for every diffracted ray;
  * the chains with the energy stop rule of Sec. III-B (rt_trace_energy) at
    several thresholds: per-facet materials (ground concrete, other facets
    concrete / glass / metal 0.8 / 0.15 / 0.05), illustrative power
    reflection coefficients, free-space constant at 2.4 GHz;
  * beside them, the CPU checker (test infrastructure, all host threads) on a
    seeded 65,536-ray sample of the launch: its chains, its chains with the
    energy rule, its reception test (64 field points) and its diffraction.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

# float64 operations of one segment-field point test (Eq. (4) as evaluated:
# w 3, w.d 5, s 1 div, p 6, dist^2 5, |w|^2 5 + 1 sqrt, l 1, rr 1, 3 dist^2 1,
# rr^2 1, two range compares and one threshold compare not counted)
FP64_OPS_PER_TEST = 30
BYTES_PER_SEGMENT = 32 + 16  # stored segment ray + its hit record


def cpu_checker(w, delta, n_sample, say):
    """The CPU checker (test infrastructure) on a seeded sample of the same
    launch, all host threads: its float64 chains with the energy rule, its
    receiving-sphere test of those chains against 64 field points, and its
    diffraction of them (16 directions).  Rates in segments per second."""
    import os
    import time as _t

    import oracle
    from oracle import diffraction, reception
    from rtgen import workloads
    threads = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(w.n_rays, size=min(n_sample, w.n_rays), replace=False))
    rays = w.rays[pick]
    tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.4, src=w.tx))
    out = {"threads": threads, "sample_rays": int(rays.shape[0])}
    t0 = _t.perf_counter()
    ch = oracle.bounces(w.tris, rays, w.max_bounces, tree=tree, nthreads=threads)
    t_ch = _t.perf_counter() - t0
    segs = int(np.sum(np.minimum(ch.n_hits + 1, w.max_bounces)))
    out["chains_msegments_s"] = round(segs / t_ch / 1e6, 3)
    mat = workloads.city_materials(w.n_tris, 0)
    t0 = _t.perf_counter()
    che, pw = oracle.bounces_energy(w.tris, rays, w.max_bounces, mat, workloads.REFLECTION,
                                    workloads.free_space_k0(), 1e-10, tree=tree, nthreads=threads,
                                    segments=False)
    t_e = _t.perf_counter() - t0
    stopped = (pw < 1e-10) & (che.n_hits > 0)
    segs_e = int(np.sum(np.where(stopped, che.n_hits, np.minimum(che.n_hits + 1, w.max_bounces))))
    out["energy_1e-10_msegments_s"] = round(segs_e / t_e / 1e6, 3)
    pts = workloads.field_points(w.tris, 400.0, 64, 164)
    t0 = _t.perf_counter()
    reception.receive(ch.seg, ch.id, ch.t, pts, delta)
    t_r = _t.perf_counter() - t0
    out["reception_64_msegments_s"] = round(segs / t_r / 1e6, 3)
    nbr = diffraction.wedges(w.tris)
    t0 = _t.perf_counter()
    nd = diffraction.diffract(w.tris, nbr, ch.seg, ch.id, ch.t, delta,
                              diffraction.cone_table(16)).size
    t_d = _t.perf_counter() - t0
    out["diffraction_msegments_s"] = round(segs / t_d / 1e6, 3)
    out["diffracted_rays"] = int(nd)
    out["segments"] = segs
    say("cpu checker:", out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--receivers", default="1,16,64,256")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--dedup-receivers", type=int, default=64)
    ap.add_argument("--thresholds", default="1e-9,1e-10,1e-11,0")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU checker's timings")
    ap.add_argument("--cpu-rays", type=int, default=65536,
                    help="seeded sample of the launch the CPU checker runs on")
    a = ap.parse_args()
    import torch

    from . import (BVH, Energy, Receivers, SplitParams, diffracted_rays, rt_diffract_segments,
                   rt_receive_segments, rt_wedges)
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

    def timed_host(fn):  # host wall clock of a synchronising call, ms
        t0 = time.perf_counter()
        fn()
        return (time.perf_counter() - t0) * 1e3

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
    # diffraction over the stored chains
    tris_d = torch.from_numpy(w.tris).cuda()
    nbr = rt_wedges(tris_d)
    t_w = min(timed_host(lambda: rt_wedges(tris_d, nbr)) for _ in range(3))
    n_cone = 16
    a_k = 2 * np.pi * (np.arange(n_cone) + 0.5) / n_cone
    cone = torch.from_numpy(np.stack([np.cos(a_k), np.sin(a_k)], 1)).cuda()
    cap = 1 << 24
    dout = torch.zeros((cap, 16), dtype=torch.int32, device="cuda")
    dcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    t_d = timed(lambda: rt_diffract_segments(tris_d, nbr, seg, out, nb, delta, cone, cap, dout, dcnt))
    nd = min(int(dcnt.item()), cap)
    drays = diffracted_rays(dout, nd)
    dhits = bvh.hits_buffer(nd, 1)[0]
    t_dt = timed(lambda: bvh.trace(drays, dhits))
    wedge_half_edges = int((nbr >= 0).sum().item())
    res["diffraction"] = {"wedges_ms": round(t_w, 3), "wedge_half_edges": wedge_half_edges,
                          "free_half_edges": int((nbr == -1).sum().item()), "cone_directions": n_cone,
                          "pass_ms": round(t_d, 4), "diffracted_rays": nd,
                          "trace_diffracted_ms": round(t_dt, 4),
                          "diffracted_mrays_s": round(nd / (t_dt * 1e-3) / 1e6, 1)}
    say(f"diffraction: wedges {t_w:.2f} ms ({wedge_half_edges} wedge half-edges), pass {t_d:.3f} ms, "
        f"{nd} diffracted rays, traced in {t_dt:.3f} ms")
    del seg, dout
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
    if not a.no_cpu:
        res["cpu_checker"] = cpu_checker(w, delta, a.cpu_rays, say)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
