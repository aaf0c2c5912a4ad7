#!/usr/bin/env python3
"""Closest-hit ray tracing benchmark on one MI355X.

A step is one pass of the whole path for one transmitter: build the BVH of
the scene with the Eq. (2) split for that transmitter (Sec. II-B, II-C), then
trace the launched rays with up to 6 specular bounces (Sec. III-B).  Scene and
rays are seeded synthetic inputs already resident in HBM.  The value is
traced segments (primary + every re-launched segment) per second of the timed
steps, in millions.  Consecutive steps alternate between two trees, output
sets and streams (--pipeline 2, the default), so one transmitter's build runs
while the previous transmitter's rays are traced; every step still builds its
whole tree and traces all its rays.  The serial rate (--pipeline 1: each step
waits for the previous one) is reported beside it.

Prints one JSON line.  Extra fields: the trace kernel's roofline (algorithmic
bytes from the instrumented kernel's node and facet counts), the CPU checker's
rate on the same workload, the traditional (alpha = 1) vs improved split
comparison, facet tests and nodes per ray, per-step latency percentiles
(device time from a step's first kernel to its last).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "closest-hit Mrays/s (24k-tri scene, ≤6 bounces); tri tests/ray; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
TRACE_SRC = os.path.join(ROOT, "paper_2208_10008_amd", "csrc", "rt_trace.hip")
NODE_BYTES = 64      # binary node: both child boxes + references
FACET_BYTES = 36     # three float32 vertices
RAY_BYTES = 32
HIT_BYTES = 16


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="city24k", choices=["city24k", "microcell", "dense200k"])
    ap.add_argument("--alpha", type=float, default=0.4)
    ap.add_argument("--max-leaf", type=int, default=4)
    ap.add_argument("--node-format", default="bin2", choices=["bin2", "f4", "q4"])
    ap.add_argument("--pipeline", type=int, default=2, choices=[1, 2],
                    help="trees / streams that consecutive steps alternate between")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-serial", action="store_true",
                    help="skip the serial reference steps (profiling runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the streaming-read probes (measured L2 / MALL / HBM ceilings)")
    ap.add_argument("--no-stats", action="store_true",
                    help="skip the instrumented launch (node and facet counts)")
    return ap.parse_args()


def kernel_source_hash():
    from paper_2208_10008_amd.traffic import source_sha1
    return source_sha1(TRACE_SRC)


def load_traffic(workload_name):
    """HBM bytes per trace launch from committed counter runs, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "trace_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha1") != kernel_source_hash() or rec.get("workload") != workload_name:
        return None
    return rec.get("hbm_bytes_per_launch")


# Vector instruction issue of the chip: 256 CUs x 4 SIMDs, one wave64
# instruction every 4 cycles per SIMD (16 lanes a cycle, no packed FP32), 2.4 GHz.
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def load_sq(workload_name):
    """Vector instructions per trace launch (binary nodes, the benchmark's
    tree) from a committed SQ counter run on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "trace_sq_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha1") != kernel_source_hash() or rec.get("workload") != workload_name:
        return None
    g = rec["groups"][0]
    return {"valu_wave_instr": g["SQ_INSTS_VALU"], "vmem_rd_wave_instr": g["SQ_INSTS_VMEM_RD"]}


def probe_ceilings(R, torch):
    """Streaming-read bandwidth (GB/s) from working sets that stay in each
    XCD's L2 (2 MiB read whole by every work-group), in the Infinity Cache
    (64 MiB: every work-group cycles over its own 64 KiB slice, 8 MiB per XCD,
    more than its L2) and in HBM (4 GiB in disjoint slices)."""
    groups = 1024
    sink = torch.empty(groups, dtype=torch.int32, device="cuda")
    big = torch.ones(4 << 28, dtype=torch.int32, device="cuda")  # 4 GiB
    out = {}
    for name, mib, span, passes in (("l2", 2, 2 << 20, 4), ("mall", 64, 64 << 10, 128),
                                    ("hbm", 4096, 4 << 20, 1)):
        buf = big[: mib << 18]
        best = None
        for _ in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            moved = R.rt_probe_read(buf, span, passes, groups, sink)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[name] = round(moved / (best * 1e-3) / 1e9, 1)
    del big
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU mode (rays are "
              "independent, so each GPU would trace its own slice of the rays with the whole "
              "tree; no collective is needed)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2208_10008_amd as R
    from rtgen import workloads

    torch.cuda.set_device(0)
    w = {"city24k": workloads.city24k, "microcell": workloads.microcell,
         "dense200k": workloads.dense200k}[args.workload]()
    params = R.SplitParams(alpha=args.alpha, src=w.tx, max_leaf=args.max_leaf,
                           node_format=args.node_format)
    nb = w.max_bounces
    tris = torch.from_numpy(w.tris).cuda()
    rays = torch.from_numpy(w.rays).cuda()
    n = w.n_rays
    depth = args.pipeline
    outs = [(torch.empty((nb, n, 4), dtype=torch.int32, device="cuda"),
             torch.empty(n, dtype=torch.float64, device="cuda"),
             torch.empty(n, dtype=torch.int32, device="cuda")) for _ in range(depth)]
    out, path_len, n_hits = outs[0]
    trees = [R.BVH(tris, params) for _ in range(depth)]
    bvh = trees[0]
    streams = [torch.cuda.Stream() for _ in range(depth)]  # default priority

    def step(k, p, d, ev=None):
        """Step k on tree, outputs and stream k mod d: rebuild, then trace."""
        i = k % d
        s = streams[i]
        if ev is not None:
            ev[0].record(s)
        R.rt_rebuild(trees[i].handle, tris, p, stream=s)
        if ev is not None:
            ev[1].record(s)
        R.rt_trace_bounces(trees[i].handle, rays, nb, *outs[i], stream=s)
        if ev is not None:
            ev[2].record(s)

    def timed(p, steps, warmup, d=1):
        for k in range(warmup):
            step(k, p, d)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(k, p, d, evs[k])
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        build_ms = [e[0].elapsed_time(e[1]) for e in evs]
        trace_ms = [e[1].elapsed_time(e[2]) for e in evs]
        step_ms = [e[0].elapsed_time(e[2]) for e in evs]  # one step's latency on the device
        return total, step_ms, build_ms, trace_ms

    total, step_lat, build_ms, trace_ms = timed(params, args.steps, args.warmup, depth)
    serial = depth > 1 and not args.no_serial
    if serial:
        s_steps = max(5, args.steps // 3)
        s_tot, _, s_build, s_trace = timed(params, s_steps, 1, 1)
    nh = n_hits.cpu().numpy()
    segments = int(np.minimum(nh + 1, nb).sum())
    ms_per_step = 1e3 * total / args.steps
    value = segments / (total / args.steps) / 1e6
    trace_mean_ms = float(np.mean(trace_ms))

    # instrumented launch (outside the timed region): nodes and facet tests
    if args.no_stats:
        st = np.zeros((n, 2), np.int64)
    else:
        stats = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        R.rt_trace_ex(bvh.handle, rays, nb, out, path_len, n_hits, ray_stats=stats)
        st = stats.cpu().numpy().astype(np.int64)
    nodes_total, tests_total = int(st[:, 0].sum()), int(st[:, 1].sum())
    alg_bytes = segments * (RAY_BYTES + HIT_BYTES) + nodes_total * NODE_BYTES + tests_total * FACET_BYTES
    achieved = alg_bytes / (trace_mean_ms * 1e-3) / 1e9
    traffic = load_traffic(w.name)
    sq = load_sq(w.name)
    info = bvh.info()

    if args.copy_mib:
        # one plain copy kernel (k_probe_copy): reads and writes copy_mib MiB each
        a = torch.ones(args.copy_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        R.rt_probe_copy(a, b)
        torch.cuda.synchronize()
        del a, b
    ceilings = None if args.no_probe else probe_ceilings(R, torch)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name, "tris": w.n_tris, "rays": n, "max_bounces": nb,
            "tx": list(w.tx), "alpha": args.alpha, "max_leaf": args.max_leaf,
            "node_format": args.node_format,
            "step": "rt_rebuild (Eq. 2 BVH for this Tx) + rt_trace_bounces",
            "pipeline": depth,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_trace<bounce>", "kernel_ms": round(trace_mean_ms, 4),
            "alg_bytes_per_launch": alg_bytes,
            "measured_ceilings_gbs": ceilings,
            "frac_of_measured_l2": (round(achieved / ceilings["l2"], 4) if ceilings else None),
            "frac_of_measured_mall": (round(achieved / ceilings["mall"], 4) if ceilings else None),
            "valu_wave_instr_per_launch": (sq["valu_wave_instr"] if sq else None),
            "valu_issue_frac": (round(sq["valu_wave_instr"] / (trace_mean_ms * 1e-3 * VALU_ISSUE_PER_S), 4)
                                if sq else None),
        },
        "segments_per_step": segments,
        "trace_only_mrays_s": round(segments / (trace_mean_ms * 1e-3) / 1e6, 2),
        "primary_mrays_s": round(n / (total / args.steps) / 1e6, 2),
        "build_ms": round(float(np.mean(build_ms)), 4),
        "trace_ms": round(trace_mean_ms, 4),
        "latency_ms_p50": round(float(np.percentile(step_lat, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(step_lat, 99)), 4),
        "tri_tests_per_ray": round(tests_total / segments, 3),
        "nodes_per_ray": round(nodes_total / segments, 3),
        "tri_tests_per_primary_p50_p99": [int(np.percentile(st[:, 1], 50)), int(np.percentile(st[:, 1], 99))],
        "bvh": {"nodes": info.n_nodes, "depth": info.depth, "trace_bytes": info.trace_bytes},
    }
    if serial:
        result["serial"] = {
            "steps": s_steps, "ms_per_step": round(1e3 * s_tot / s_steps, 4),
            "mrays_s": round(segments / (s_tot / s_steps) / 1e6, 2),
            "build_ms": round(float(np.mean(s_build)), 4),
            "trace_ms": round(float(np.mean(s_trace)), 4),
        }

    if not args.no_compare:
        fmts = {}
        for fmt in ("bin2", "f4", "q4"):
            pf = R.SplitParams(alpha=args.alpha, src=w.tx, max_leaf=args.max_leaf, node_format=fmt)
            _, _, _, f_trace = timed(pf, 10, 2)
            fmts[fmt] = round(float(np.mean(f_trace)), 4)
        result["trace_ms_by_node_format"] = fmts
        trad = R.SplitParams(alpha=1.0, src=w.tx, max_leaf=args.max_leaf, node_format=args.node_format)
        t_tot, _, t_build, t_trace = timed(trad, max(5, args.steps // 3), 1)
        i_tot, _, i_build, i_trace = timed(params, max(5, args.steps // 3), 1)
        result["improved_vs_traditional"] = {
            "alpha_improved": args.alpha, "alpha_traditional": 1.0,
            "trace_ms_improved": round(float(np.mean(i_trace)), 4),
            "trace_ms_traditional": round(float(np.mean(t_trace)), 4),
            "trace_time_ratio": round(float(np.mean(i_trace) / np.mean(t_trace)), 4),
            "step_ms_improved": round(1e3 * i_tot / max(5, args.steps // 3), 4),
            "step_ms_traditional": round(1e3 * t_tot / max(5, args.steps // 3), 4),
            "paper_claim": "20-35% less computation time than the traditional BVH "
                           "(hardware not stated in the paper)",
        }
        step(0, params, 1)  # leave the improved tree in place
        torch.cuda.synchronize()

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.alpha, args.max_leaf)

    print(json.dumps(result), flush=True)


def cpu_baseline(w, alpha, max_leaf):
    """The CPU checker (float64 C++, all of its threads) running the same
    step: the paper's build for the transmitter, then every ray's chain with
    the Sec. III-B traversal (with its margin bookkeeping)."""
    import numpy as np

    import oracle

    threads = min(16, os.cpu_count() or 1)
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=alpha, src=w.tx, max_leaf=max_leaf))
        t1 = time.perf_counter()
        ch = oracle.bounces(w.tris, w.rays, w.max_bounces, tree=tree, nthreads=threads, segments=False)
        t2 = time.perf_counter()
        segs = int(np.minimum(ch.n_hits + 1, w.max_bounces).sum())
        runs.append((t2 - t0, t1 - t0, segs))
        if t2 - t0 > 10:
            break
    runs.sort()
    tot, build, segs = runs[len(runs) // 2]
    # brute force (every ray against every facet, the definition of the hit):
    # the 242-facet scene whole and a seeded subsample of this workload's rays
    from rtgen import workloads
    mc = workloads.microcell()
    t0 = time.perf_counter()
    oracle.brute(mc.tris, mc.rays, nthreads=threads)
    t_mc = time.perf_counter() - t0
    sub = np.random.default_rng(0).choice(w.n_rays, size=min(w.n_rays, 65536), replace=False)
    t0 = time.perf_counter()
    oracle.brute(w.tris, w.rays[np.sort(sub)], nthreads=threads)
    t_sub = time.perf_counter() - t0
    return {"value": round(segs / tot / 1e6, 3), "unit": "Mrays/s", "cores": threads,
            "kind": "oracle", "seconds_per_step": round(tot, 3), "build_s": round(build, 3),
            "sample": f"whole workload: {w.n_rays} rays, <= {w.max_bounces} segments each, "
                      f"float64 build + traversal, median of {len(runs)} runs",
            "brute_force_mrays_s": {
                mc.name: round(mc.n_rays / t_mc / 1e6, 4),
                f"{w.name} (65536 primary rays)": round(len(sub) / t_sub / 1e6, 4)}}


if __name__ == "__main__":
    main()
