#!/usr/bin/env python3
"""Closest-hit ray tracing benchmark on one MI355X.

A step is one pass of the whole path for one transmitter: build the BVH of
the scene with the Eq. (2) split for that transmitter (Sec. II-B, II-C), then
trace the launched rays with up to 6 specular bounces (Sec. III-B).  Scene and
rays are seeded synthetic inputs already resident in HBM.  The value is
traced segments (primary + every re-launched segment) per second of the timed
steps, in millions.  Consecutive steps alternate between two trees and output
sets (--pipeline 2, the default), so one transmitter's build runs while the
previous transmitter's rays are traced; builds run on a stream holding some
of the 256 compute units (32 on city24k, 64 on the dense city) and traces on
one holding the rest (rt_streams_split_cus).  Each step orders its ray
batches most horizontal first (rt_rays_batch_order) before tracing them;
every step still builds its whole tree, orders and traces all its rays.  The
pipelined builds are queued with rt_rebuild_async, the next one before the host
waits (rt_bvh_wait) for the current one, so the build stream does not wait for
the host between builds.  The value comes from a pass of the timed steps that records no events among them;
a second pass of the same steps with HIP events around each stage gives the
kernel, build and batch-order times and the step latency.  The
trees' traversal nodes are 4-wide float32 on city24k and binary float32 on the
dense city (NODE_FORMAT); the rate of the same step with each node format is
reported beside it, and so is the serial rate (--pipeline 1: each step waits
for the previous one, on all compute units).

Prints one JSON line.  Extra fields: the trace kernel's roofline (vector
instruction issue, from the committed SQ counters of the current kernel
source, over the kernel time measured here; the algorithmic node and facet
bytes against the measured L2 ceiling beside it), the CPU checker's rate on
the same workload, the traditional (alpha = 1) vs improved split comparison
and an alpha sweep in both distance normalisations, facet tests and nodes per
ray, per-step latency percentiles (device time from a step's first kernel to
its last).

Other suites (--suite), each printing one JSON line of its own:
  paper   Sec. IV regime: the study room and campus stand-ins at the paper's
          leaf sizes, traditional vs proposed split, time against ray count
  recv    after-trace stages on the city launch: receiving spheres (Eq. (4)),
          duplicate grouping, diffraction, energy stop rule
  batch   the multi-scene batched launch (8 scenes, 64 transmitters) per node
          format, autotuned and graph-captured
  lanes   lanes per ray on the paper-size scenes: every lane count per case
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
TRACE_SRC = os.path.join(ROOT, "paper_2208_10008_amd", "csrc", "rt_trace.hip")
# bytes of one node visit: binary nodes hold both child boxes and references,
# 4-wide float32 nodes four boxes, 8-bit nodes four quantised boxes
NODE_BYTES = {"bin2": 64, "f4": 128, "q4": 64}
CHILDREN = {"bin2": 2, "f4": 4, "q4": 4}  # child boxes tested per node visit
FACET_BYTES = 36     # three float32 vertices
RAY_BYTES = 32
HIT_BYTES = 16
# Algorithmic vector operations: one child-box slab test ~18 operations, one
# facet test ~45.
OPS_PER_CHILD_TEST = 18
OPS_PER_FACET_TEST = 45
# Vector issue of the chip: 256 CUs x 4 SIMDs, one wave64 instruction every 4
# cycles per SIMD (16 lanes a cycle, packed FP32 off), 2.4 GHz.  In lane
# operations: 256 x 4 x 16 x 2.4e9 = 39.32e12 per second.
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
ALU_PEAK_TOPS = VALU_ISSUE_PER_S * 64 / 1e12
# the GPU machine's host share for one GPU: worker pools stay within it
CPU_SHARE = 16


# Compute units the pipelined steps give the builds (the traces get the rest),
# measured per workload: the 24k-facet build fits beside the trace on 32 of
# 256, the 200k-facet build on 64.
BUILD_CUS = {"city24k": 32, "microcell": 0, "dense200k": 64}
# Traversal nodes of the benchmark's trees, measured per workload in the
# pipelined step: on the 24k-facet city the 4-wide nodes' shorter traversal
# pays for their longer build; the 200k-facet tree exceeds an XCD's L2, where
# binary nodes trace fastest.
NODE_FORMAT = {"city24k": "f4", "microcell": "bin2", "dense200k": "bin2"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--suite", default="step", choices=["step", "paper", "recv", "batch", "lanes"])
    ap.add_argument("--workload", default="city24k", choices=["city24k", "microcell", "dense200k"])
    ap.add_argument("--alpha", type=float, default=0.4)
    ap.add_argument("--max-leaf", type=int, default=4)
    ap.add_argument("--node-format", default=None, choices=["bin2", "f4", "q4"],
                    help="traversal nodes of the benchmark's trees: binary float32, 4-wide float32 "
                         "or 4-wide 8-bit; default per workload (NODE_FORMAT); every format is "
                         "also timed beside it")
    ap.add_argument("--pipeline", type=int, default=2, choices=[1, 2],
                    help="trees / streams that consecutive steps alternate between")
    ap.add_argument("--cut", type=int, default=0,
                    help="two-launch trace: chains alive after this many segments are traced by a "
                         "second launch in full waves (rt_trace_opts.cut; 0: one launch)")
    ap.add_argument("--build-cus", type=int, default=None, choices=[0] + list(range(8, 129, 8)),
                    help="pipelined steps: builds on this many compute units, traces on the rest "
                         "(rt_streams_split_cus); 0: one stream per tree on all of them; default "
                         "per workload (BUILD_CUS)")
    ap.add_argument("--order", default="elevation", choices=["elevation", "given"],
                    help="trace batch order: most horizontal batches first (rt_rays_batch_order, "
                         "computed in every step) or the rays' own order")
    ap.add_argument("--pad", action="store_true",
                    help="write the rows after each chain's miss as misses too (the library default; "
                         "the step leaves them, since n_hits says where every chain ends)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the alpha / d_norm sweep")
    ap.add_argument("--no-serial", action="store_true",
                    help="skip the serial reference steps (profiling runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the streaming-read probes (measured L2 / MALL / HBM ceilings)")
    ap.add_argument("--no-stats", action="store_true",
                    help="skip the instrumented launch (node and facet counts)")
    # suites
    ap.add_argument("--reps", type=int, default=10, help="suites: launches timed per case")
    ap.add_argument("--levels", default="3-9", help="paper / lanes suites: icosphere levels")
    ap.add_argument("--cpu-levels", default="3-6", help="paper suite: levels the checker runs")
    ap.add_argument("--receivers", default="1,16,64,256", help="recv suite: field point counts")
    ap.add_argument("--dedup-receivers", type=int, default=64)
    ap.add_argument("--thresholds", default="1e-9,1e-10,1e-11,0", help="recv suite: energy stops")
    ap.add_argument("--cpu-rays", type=int, default=65536,
                    help="recv suite: seeded sample of the launch the checker runs on")
    ap.add_argument("--formats", default="bin2,f4,q4", help="batch suite: node formats")
    return ap.parse_args()


def kernel_source_hash():
    from counters import source_sha1
    return source_sha1(TRACE_SRC)


def _profile_record(name, workload_name, node_format):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel_source_sha1") != kernel_source_hash() or rec.get("workload") != workload_name
            or rec.get("node_format", "bin2") != node_format):
        return None
    return rec


def load_traffic(workload_name, node_format):
    """HBM bytes per trace launch from committed counter runs, if they were
    taken on the current kernel source with this node format."""
    rec = _profile_record("trace_traffic.json", workload_name, node_format)
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def load_sq(workload_name, node_format):
    """Vector instructions per trace launch (the benchmark's launch: its tree
    and node format) from a committed SQ counter run on the current kernel
    source."""
    rec = _profile_record("trace_sq_counters.json", workload_name, node_format)
    if rec is None:
        return None
    g = rec["groups"][0]
    return {"valu_wave_instr": g["SQ_INSTS_VALU"], "vmem_rd_wave_instr": g["SQ_INSTS_VMEM_RD"]}


def roofline(trace_ms, segments, nodes_total, tests_total, sq, traffic, ceilings, node_format):
    """The trace kernel's roofline.  The bound is vector instruction issue: the
    kernel's VALU wave-instructions per launch (SQ counters) over its measured
    time against the chip's non-packed issue rate, in lane operations.  The
    algorithmic operations and bytes (per segment: ray and hit record, the
    node bytes per node visited, 36 B per facet tested) are reported beside
    it."""
    sec = trace_ms * 1e-3
    alg_bytes = (segments * (RAY_BYTES + HIT_BYTES) + nodes_total * NODE_BYTES[node_format]
                 + tests_total * FACET_BYTES)
    alg_ops = nodes_total * CHILDREN[node_format] * OPS_PER_CHILD_TEST + tests_total * OPS_PER_FACET_TEST
    alg_gbs = alg_bytes / sec / 1e9
    r = {"bound": "alu", "achieved": None, "peak": round(ALU_PEAK_TOPS, 2),
         "unit": "TOP/s (VALU lane operations, packed FP32 off)", "frac": None,
         "traffic": traffic, "kernel": "k_trace<bounce>", "kernel_ms": round(trace_ms, 4),
         "valu_wave_instr_per_launch": sq["valu_wave_instr"] if sq else None,
         "counters": "profiles/trace_sq_counters.json" if sq else None,
         "algorithmic": {
             "ops_per_launch": alg_ops,
             "tops": round(alg_ops / sec / 1e12, 3),
             "frac_of_alu_peak": round(alg_ops / sec / 1e12 / ALU_PEAK_TOPS, 4),
             "bytes_per_launch": alg_bytes, "gbs": round(alg_gbs, 1),
             "measured_ceilings_gbs": ceilings,
             "frac_of_measured_l2": round(alg_gbs / ceilings["l2"], 4) if ceilings else None}}
    if sq:
        tops = sq["valu_wave_instr"] * 64 / sec / 1e12
        r["achieved"] = round(tops, 3)
        r["frac"] = round(tops / ALU_PEAK_TOPS, 4)
    if traffic:
        r["hbm_gbs"] = round(traffic / sec / 1e9, 1)
    return r


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


def cpu_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(CPU_SHARE, avail))


def say(tag, *m):
    print(f"[{tag}]", *m, file=sys.stderr, flush=True)


def event_timer(torch, reps):
    """Average device time (ms) of fn over reps launches after one untimed one."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    return timed


# ----------------------------------------------------------------- the step
def main_step(args):
    import numpy as np
    import torch

    import paper_2208_10008_amd as R
    from rtgen import workloads

    torch.cuda.set_device(0)
    w = {"city24k": workloads.city24k, "microcell": workloads.microcell,
         "dense200k": workloads.dense200k}[args.workload]()
    if args.node_format is None:
        args.node_format = NODE_FORMAT.get(args.workload, "bin2")
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
    plain = torch.cuda.Stream()  # default priority, all compute units (serial steps)
    if args.build_cus is None:
        args.build_cus = BUILD_CUS.get(args.workload, 0)
    split = R.SplitStreams(args.build_cus) if depth > 1 and args.build_cus > 0 else None
    if split is not None:  # builds on build_cus compute units, traces on the rest
        bstreams, tstreams = [split.small] * depth, [split.large] * depth
    else:  # one stream per tree, build and trace of a step on it
        bstreams = tstreams = [torch.cuda.Stream() for _ in range(depth)]
    done = [torch.cuda.Event() for _ in range(depth)]  # tree i's last trace has ended
    wss = [R.chain_workspace(n) for _ in range(depth)] if args.cut > 0 else [None] * depth
    nbat = (n + 63) // 64
    orders = [torch.empty(nbat, dtype=torch.int32, device="cuda") for _ in range(depth)]
    okeys = [torch.empty(R.rt_rays_batch_order_ws_bytes(n) // 4, dtype=torch.int32, device="cuda")
             for _ in range(depth)]

    flags = 0 if args.pad else R.RT_TRACE_NO_PAD

    built = [torch.cuda.Event() for _ in range(depth)]  # tree i's last queued build has ended

    def queue_build(k, p, d, ev=None):
        """Step k's build, tree k mod d, queued without waiting for it (the
        host reads its record in finish_step)."""
        i = k % d
        sb = bstreams[i]
        sb.wait_event(done[i])  # the tree's previous trace has finished
        if ev is not None:
            ev[0].record(sb)
        R.rt_rebuild_async(trees[i].handle, tris, p, stream=sb)
        if ev is not None:
            ev[1].record(sb)
        built[i].record(sb)

    def finish_step(k, p, d, ev=None, flags=flags):
        """Step k after its build: order the ray batches (they need the rays
        only), wait for the build's record, trace once the build has ended.
        With one tree (d = 1) the build is synchronous, on the same stream."""
        i = k % d
        sb, st = (plain, plain) if d == 1 else (bstreams[i], tstreams[i])
        if d == 1:
            if ev is not None:
                ev[0].record(sb)
            R.rt_rebuild(trees[i].handle, tris, p, stream=sb)
            if ev is not None:
                ev[1].record(sb)
        if ev is not None:
            ev[3].record(st)
        order = None
        if args.order == "elevation":
            order = R.rt_rays_batch_order(rays, axis=2, order=orders[i], keys=okeys[i], stream=st)
        if ev is not None:
            ev[4].record(st)
        if d > 1:
            R.rt_bvh_wait(trees[i].handle)
            st.wait_event(built[i])
        if ev is not None:
            ev[5].record(st)
        if args.cut > 0 or flags or order is not None:
            R.rt_trace_ex(trees[i].handle, rays, nb, *outs[i], cut=args.cut, chain_ws=wss[i],
                          stream=st, flags=flags, batch_order=order)
        else:
            R.rt_trace_bounces(trees[i].handle, rays, nb, *outs[i], stream=st)
        done[i].record(st)
        if ev is not None:
            ev[2].record(st)

    def run_steps(steps, p, d, evs=None, flags=flags):
        """Steps 0 .. steps - 1.  Pipelined (d > 1): step k + 1's build is
        queued before the host waits for step k's, so the build stream goes
        from one build to the next without waiting for the host."""
        if d > 1 and steps > 0:
            queue_build(0, p, d, evs[0] if evs else None)
        for k in range(steps):
            if d > 1 and k + 1 < steps:
                queue_build(k + 1, p, d, evs[k + 1] if evs else None)
            finish_step(k, p, d, evs[k] if evs else None, flags=flags)

    order_ms = []  # the last timed() call's batch-order times

    def timed(p, steps, warmup, d=1, flags=flags, events=True):
        """Wall time of `steps` steps after `warmup` untimed ones; with
        events, HIP events around each step's build, batch order and trace
        give their times and the step's latency.  events=False records none
        inside the timed region (each event is a barrier packet on its
        stream, about 1-3 % of a step): the rates come from such passes."""
        run_steps(warmup, p, d, flags=flags)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)] \
            if events else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(steps, p, d, evs, flags=flags)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        if not events:
            return total, None, None, None
        build_ms = [e[0].elapsed_time(e[1]) for e in evs]
        # the trace launch on its own stream, from the end of its wait for the build
        trace_ms = [e[5].elapsed_time(e[2]) for e in evs]
        order_ms[:] = [e[3].elapsed_time(e[4]) for e in evs]
        step_ms = [e[0].elapsed_time(e[2]) for e in evs]  # one step's latency on the device
        return total, step_ms, build_ms, trace_ms

    def launch_counts(p=None):
        """Nodes visited and facets tested per traced segment (instrumented
        launch on tree 0, outside any timed region)."""
        if p is not None:
            R.rt_rebuild(bvh.handle, tris, p)
        stats = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        R.rt_trace_ex(bvh.handle, rays, nb, out, path_len, n_hits, ray_stats=stats)
        st = stats.cpu().numpy().astype(np.int64)
        segs = int(np.minimum(n_hits.cpu().numpy() + 1, nb).sum())
        return st, segs

    # the value: the timed steps with no events among them; then the same
    # steps with events (kernel, build and order times, step latency)
    total, _, _, _ = timed(params, args.steps, args.warmup, depth, events=False)
    _, step_lat, build_ms, trace_ms = timed(params, args.steps, args.warmup, depth)
    main_order_ms = list(order_ms)
    serial = depth > 1 and not args.no_serial
    if serial:
        s_steps = max(5, args.steps // 3)
        s_tot, _, _, _ = timed(params, s_steps, 1, 1, events=False)
        _, _, s_build, s_trace = timed(params, s_steps, 1, 1)
        if flags:
            p_tot, _, _, _ = timed(params, args.steps, 1, depth, flags=0, events=False)
            _, _, p_build, p_trace = timed(params, args.steps, 1, depth, flags=0)
    nh = n_hits.cpu().numpy()
    segments = int(np.minimum(nh + 1, nb).sum())
    ms_per_step = 1e3 * total / args.steps
    value = segments / (total / args.steps) / 1e6
    trace_mean_ms = float(np.mean(trace_ms))

    if args.no_stats:
        st = np.zeros((n, 2), np.int64)
    else:
        st, _ = launch_counts()
    nodes_total, tests_total = int(st[:, 0].sum()), int(st[:, 1].sum())
    info = bvh.info()
    tree_stats = bvh.stats()

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
            "step": ("rt_rebuild_async + rt_bvh_wait" if depth > 1 else "rt_rebuild")
                    + " (Eq. 2 BVH for this Tx) + " + (
                "rt_rays_batch_order + " if args.order == "elevation" else "") + (
                f"rt_trace_ex (two launches, cut {args.cut})" if args.cut > 0 else
                "rt_trace_ex (one launch)" if flags or args.order == "elevation" else "rt_trace_bounces"),
            "pipeline": depth,
            "streams": (f"builds on {args.build_cus} compute units, traces on {256 - args.build_cus}"
                        if split is not None else "one stream per tree, all compute units"),
            "miss_rows": "padded" if args.pad else "left (RT_TRACE_NO_PAD; n_hits ends each chain)",
        },
        "roofline": roofline(trace_mean_ms, segments, nodes_total, tests_total,
                             load_sq(w.name, args.node_format), load_traffic(w.name, args.node_format),
                             ceilings, args.node_format),
        "segments_per_step": segments,
        "trace_only_mrays_s": round(segments / (trace_mean_ms * 1e-3) / 1e6, 2),
        "primary_mrays_s": round(n / (total / args.steps) / 1e6, 2),
        "build_ms": round(float(np.mean(build_ms)), 4),
        "trace_ms": round(trace_mean_ms, 4),
        "batch_order_ms": round(float(np.mean(main_order_ms)), 4),
        "latency_ms_p50": round(float(np.percentile(step_lat, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(step_lat, 99)), 4),
        "tri_tests_per_ray": round(tests_total / segments, 3),
        "nodes_per_ray": round(nodes_total / segments, 3),
        "tri_tests_per_primary_p50_p99": [int(np.percentile(st[:, 1], 50)), int(np.percentile(st[:, 1], 99))],
        "nodes_per_primary_p50_p99": [int(np.percentile(st[:, 0], 50)), int(np.percentile(st[:, 0], 99))],
        "bvh": {"nodes": info.n_nodes, "depth": info.depth, "trace_bytes": info.trace_bytes,
                "tree_cost": round(tree_stats.tree_cost, 4),
                "leaf_hist": list(tree_stats.leaf_hist)[:8]},
    }
    if serial:
        result["serial"] = {
            "steps": s_steps, "ms_per_step": round(1e3 * s_tot / s_steps, 4),
            "mrays_s": round(segments / (s_tot / s_steps) / 1e6, 2),
            "build_ms": round(float(np.mean(s_build)), 4),
            "trace_ms": round(float(np.mean(s_trace)), 4),
        }
        if flags:
            result["padded"] = {
                "steps": args.steps, "ms_per_step": round(1e3 * p_tot / args.steps, 4),
                "mrays_s": round(segments / (p_tot / args.steps) / 1e6, 2),
                "build_ms": round(float(np.mean(p_build)), 4),
                "trace_ms": round(float(np.mean(p_trace)), 4),
            }

    if not args.no_compare:
        fmts, piped = {}, {}
        for fmt in ("bin2", "f4", "q4"):
            pf = R.SplitParams(alpha=args.alpha, src=w.tx, max_leaf=args.max_leaf, node_format=fmt)
            _, _, _, f_trace = timed(pf, 10, 2)
            fmts[fmt] = round(float(np.mean(f_trace)), 4)
            # the benchmark's step (pipelined, same streams) with this format's trees
            f_tot, _, _, _ = timed(pf, args.steps, args.warmup, depth, events=False)
            piped[fmt] = round(segments / (f_tot / args.steps) / 1e6, 2)
        result["trace_ms_by_node_format"] = fmts
        result["mrays_s_by_node_format"] = piped
        reps = max(5, args.steps // 3)
        trad = R.SplitParams(alpha=1.0, src=w.tx, max_leaf=args.max_leaf, node_format=args.node_format)
        t_tot, _, t_build, t_trace = timed(trad, reps, 1)
        i_tot, _, i_build, i_trace = timed(params, reps, 1)
        result["improved_vs_traditional"] = {
            "alpha_improved": args.alpha, "alpha_traditional": 1.0,
            "trace_ms_improved": round(float(np.mean(i_trace)), 4),
            "trace_ms_traditional": round(float(np.mean(t_trace)), 4),
            "trace_time_ratio": round(float(np.mean(i_trace) / np.mean(t_trace)), 4),
            "step_ms_improved": round(1e3 * i_tot / reps, 4),
            "step_ms_traditional": round(1e3 * t_tot / reps, 4),
            "paper_claim": "20-35% less computation time than the traditional BVH "
                           "(hardware not stated in the paper)",
        }
        if not args.no_sweep:
            result["split_sweep"] = split_sweep(R, w, args, timed, launch_counts, bvh)
        finish_step(0, params, 1)  # leave the improved tree in place
        torch.cuda.synchronize()

    if split is not None:
        split.close()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.alpha, args.max_leaf)

    print(json.dumps(result), flush=True)


def split_sweep(R, w, args, timed, launch_counts, bvh):
    """Eq. (2) weight alpha swept in both distance normalisations (unit:
    both terms scaled to O(1); raw: the printed units), each tree timed on
    serial steps (rebuild + trace) against alpha = 1 (Eq. (1), the same tree
    in both normalisations), with its Eq. (1) tree cost and node / facet
    counts per segment."""
    import numpy as np
    alphas = (0.0, 0.2, 0.4, 0.6, 0.7, 0.8, 0.9, 1.0)
    res = {"alphas": list(alphas), "steps": 6, "unit": {}, "raw": {}}
    for norm in ("unit", "raw"):
        rows = {}
        for a in alphas:
            p = R.SplitParams(alpha=a, src=w.tx, max_leaf=args.max_leaf, d_norm=norm,
                              node_format=args.node_format)
            _, _, b_ms, t_ms = timed(p, 6, 1)
            st, segs = launch_counts(p)
            info = bvh.stats()
            rows[repr(a)] = {"trace_ms": round(float(np.median(t_ms)), 4),
                             "build_ms": round(float(np.median(b_ms)), 4),
                             "depth": int(info.depth), "tree_cost": round(info.tree_cost, 3),
                             "nodes_per_ray": round(float(st[:, 0].sum()) / segs, 3),
                             "tests_per_ray": round(float(st[:, 1].sum()) / segs, 3)}
        base = rows[repr(1.0)]["trace_ms"]
        for r in rows.values():
            r["trace_vs_alpha1"] = round(r["trace_ms"] / base, 4)
        res[norm] = rows
        say("sweep", norm, {k: (v["trace_ms"], v["trace_vs_alpha1"]) for k, v in rows.items()})
    return res


def cpu_baseline(w, alpha, max_leaf):
    """The CPU checker (float64 C++, the machine's host threads for one GPU)
    running the same step: the paper's build for the transmitter, then every
    ray's chain with the Sec. III-B traversal (with its margin bookkeeping)."""
    import numpy as np

    import oracle

    threads = cpu_threads()
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
            "host_cpus": os.cpu_count(),
            "threads_note": f"worker threads = min({CPU_SHARE}, CPUs this process may run on): "
                            f"the host share of one GPU on the GPU box",
            "kind": "oracle", "seconds_per_step": round(tot, 3), "build_s": round(build, 3),
            "sample": f"whole workload: {w.n_rays} rays, <= {w.max_bounces} segments each, "
                      f"float64 build + traversal, median of {len(runs)} runs",
            "brute_force_mrays_s": {
                mc.name: round(mc.n_rays / t_mc / 1e6, 4),
                f"{w.name} (65536 primary rays)": round(len(sub) / t_sub / 1e6, 4)}}


# ----------------------------------------------------------------- suites
def _levels(s):
    lo, hi = (int(x) for x in s.split("-"))
    return list(range(lo, hi + 1))


def suite_paper(args):
    """Sec. IV regime (Fig. 9 analogue): running time against the number of
    launched rays, traditional split (Eq. (1): alpha = 1) against the proposed
    one (Eq. (2)), on the two paper-size stand-in scenes:
      indoor: study room 8 x 6 x 3.5 m, 2,778 facets, 250 facets per leaf,
        alpha 0.7, reflection orders up to 2, Tx (1.46, 2.42, 2.1), Rx (1.2, 1.2, 1.5);
      outdoor: campus, 7,608 facets, 820 facets per leaf, alpha 0.4,
        reflection order up to 3, Tx (450, 450, 10), Rx (450, 550, 25).
    Per scene, split and level: GPU time of one step (rt_rebuild for this Tx +
    rt_trace_receive at the Rx, HIP events), facet tests and node visits per
    segment, the paths received at the Rx after duplicate grouping; the CPU
    checker's time on the same chains (its float64 traversal of the same
    tree) for the levels it finishes quickly; the GPU at leaf size 4."""
    import numpy as np
    import torch

    from paper_2208_10008_amd import BVH, Receivers, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    levels = _levels(args.levels)
    timed = event_timer(torch, args.reps)
    dirs = torch.from_numpy(icosphere.directions(max(levels)).astype(np.float32)).cuda()
    res = {"suite": "paper", "command": "python3 bench.py --suite paper", "scenes": {}}
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
            info = bvh.stats()
            t_build = timed(lambda: bvh.rebuild(tris, p))
            run = {"alpha": alpha, "max_leaf": leaf, "nodes": int(info.n_nodes),
                   "depth": int(info.depth), "tree_cost": round(info.tree_cost, 3),
                   "build_ms": round(t_build, 4), "levels": {}}
            for lv in levels:
                n = icosphere.vertex_count(lv)
                rays = rt_rays_from_directions(dirs, n, w.tx, 1e-4, w.tmax)
                delta = float(icosphere.edge_angles(lv).mean())
                recv = Receivers(rx, delta, 1 << 16)
                out = bvh.hits_buffer(n, nb)
                pl = torch.empty(n, dtype=torch.float64, device="cuda")
                nh = torch.empty(n, dtype=torch.int32, device="cuda")
                t_tr = timed(lambda: bvh.trace_receive(rays, nb, recv, out, pl, nh))
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
            say("paper", w.name, tag, {k: (v["trace_ms"], v["tests_per_segment"], v["paths"])
                                       for k, v in run["levels"].items()})
            sc["runs"][tag] = run
            bvh.close()
        if not args.no_cpu_baseline:
            sc["cpu_checker_ms"], sc["cpu_threads"] = paper_cpu_baseline(w, _levels(args.cpu_levels))
            say("paper", w.name, "cpu", sc["cpu_checker_ms"])
        res["scenes"][w.name] = sc
    print(json.dumps(res), flush=True)


def paper_cpu_baseline(w, levels):
    """The CPU checker's chains on the paper scene's own trees (traditional and
    proposed split), per icosphere level, in ms."""
    import oracle
    threads = cpu_threads()
    cpu = {}
    for tag, alpha in (("traditional", 1.0), ("proposed", w.alpha)):
        tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=alpha, src=w.tx,
                                                            max_leaf=w.max_leaf))
        cpu[tag] = {}
        for lv in levels:
            r = w.rays(lv)
            t0 = time.perf_counter()
            oracle.bounces(w.tris, r, w.max_bounces, tree=tree, nthreads=threads, segments=False)
            cpu[tag][str(lv)] = round((time.perf_counter() - t0) * 1e3, 2)
    return cpu, threads


# float64 operations of one segment-field point test (Eq. (4) as evaluated:
# w 3, w.d 5, s 1 div, p 6, dist^2 5, |w|^2 5 + 1 sqrt, l 1, rr 1, 3 dist^2 1,
# rr^2 1, two range compares and one threshold compare not counted)
FP64_OPS_PER_TEST = 30
BYTES_PER_SEGMENT = 32 + 16  # stored segment ray + its hit record


def suite_recv(args):
    """After-trace stages on the city launch (2,000 buildings, 23,971 facets,
    Tx (0, 0, 25), level-9 icosphere, up to 6 segments; delta = mean angle
    between adjacent launch directions), HIP events on the launching stream:
    the chains alone; receiving spheres (Sec. III-C, Eq. (4)) at field points
    outside the buildings within 400 m of the Tx, tested as the segments are
    traced (rt_trace_receive) per number of field points, and over the stored
    segments (rt_receive_segments); duplicate grouping (rt_receive_dedup);
    edge diffraction (Sec. III-B: rt_wedges, host clock of the synchronising
    call; rt_diffract_segments with 16 cone directions; one closest-hit
    segment per diffracted ray); the energy stop rule (rt_trace_energy) at
    several thresholds; beside them the CPU checker on a seeded 65,536-ray
    sample of the launch."""
    import numpy as np
    import torch

    from paper_2208_10008_amd import (BVH, Energy, Receivers, SplitParams, diffracted_rays,
                                      rt_diffract_segments, rt_receive_segments, rt_wedges)
    from rtgen import icosphere, workloads

    w = workloads.city24k()
    nb = w.max_bounces
    delta = float(icosphere.edge_angles(w.level).mean())
    bvh = BVH(torch.from_numpy(w.tris).cuda(), SplitParams(alpha=0.4, src=w.tx))
    rays = torch.from_numpy(w.rays).cuda()
    n = w.n_rays
    out = bvh.hits_buffer(n, nb)
    pl = torch.empty(n, dtype=torch.float64, device="cuda")
    nh = torch.empty(n, dtype=torch.int32, device="cuda")
    timed = event_timer(torch, args.reps)

    def timed_host(fn):  # host wall clock of a synchronising call, ms
        t0 = time.perf_counter()
        fn()
        return (time.perf_counter() - t0) * 1e3

    t_trace = timed(lambda: bvh.trace_bounces(rays, nb, out, pl, nh))
    segs = int(torch.clamp(nh.long() + 1, max=nb).sum().item())
    say("recv", f"chains alone {t_trace:.3f} ms, {segs} segments")
    res = {"suite": "recv",
           "workload": f"city24k: {w.n_tris} facets, {n} rays (level {w.level}), up to {nb} "
                       f"segments, delta {delta:.6g} rad",
           "command": "python3 bench.py --suite recv", "segments": segs,
           "trace_ms": round(t_trace, 4), "fused": {}, "stored": {}}
    counts = [int(x) for x in args.receivers.split(",")]
    for k in sorted(set(counts + [args.dedup_receivers])):
        pts = torch.from_numpy(workloads.field_points(w.tris, 400.0, k, 100 + k)).cuda()
        recv = Receivers(pts, delta, 1 << 20)
        t = timed(lambda: bvh.trace_receive(rays, nb, recv, out, pl, nh))
        c = recv.count()
        res["fused"][str(k)] = {"ms": round(t, 4), "overhead": round(t / t_trace - 1, 4),
                                "receptions": c}
        say("recv", f"fused, {k} field points: {t:.3f} ms ({c} receptions)")
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
        say("recv", f"stored-chain kernel, {k} field points: {t:.3f} ms, {gbs:.0f} GB/s")
    k = args.dedup_receivers
    pts = torch.from_numpy(workloads.field_points(w.tris, 400.0, k, 100 + k)).cuda()
    recv = Receivers(pts, delta, 1 << 20)
    rt_receive_segments(seg, out, nb, recv)
    t = timed(lambda: recv.dedup(out, nb))
    rec = recv.records()
    res["dedup"] = {"field_points": k, "ms": round(t, 4), "receptions": int(rec.size),
                    "kept": int(rec["keep"].sum())}
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
    say("recv", "diffraction", res["diffraction"])
    del seg, dout
    mat = torch.from_numpy(workloads.city_materials(w.n_tris, 0)).cuda()
    refl = torch.from_numpy(workloads.REFLECTION).cuda()
    res["energy"] = {"k0": workloads.free_space_k0(), "reflection": workloads.REFLECTION.tolist(),
                     "thresholds": {}}
    for thr in (float(x) for x in args.thresholds.split(",")):
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
        say("recv", f"energy stop at {thr:g}: {t:.3f} ms, {segs_e} segments")
    if not args.no_cpu_baseline:
        res["cpu_checker"] = recv_cpu_baseline(w, delta, args.cpu_rays)
    print(json.dumps(res), flush=True)


def recv_cpu_baseline(w, delta, n_sample):
    """The CPU checker on a seeded sample of the same launch: its float64
    chains, the chains with the energy rule, its receiving-sphere test of
    those chains against 64 field points and its diffraction of them (16
    directions).  Rates in segments per second."""
    import numpy as np

    import oracle
    from oracle import diffraction, reception
    from rtgen import workloads
    threads = cpu_threads()
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(w.n_rays, size=min(n_sample, w.n_rays), replace=False))
    rays = w.rays[pick]
    tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.4, src=w.tx))
    out = {"threads": threads, "sample_rays": int(rays.shape[0])}
    t0 = time.perf_counter()
    ch = oracle.bounces(w.tris, rays, w.max_bounces, tree=tree, nthreads=threads)
    t_ch = time.perf_counter() - t0
    segs = int(np.sum(np.minimum(ch.n_hits + 1, w.max_bounces)))
    out["chains_msegments_s"] = round(segs / t_ch / 1e6, 3)
    mat = workloads.city_materials(w.n_tris, 0)
    t0 = time.perf_counter()
    che, pw = oracle.bounces_energy(w.tris, rays, w.max_bounces, mat, workloads.REFLECTION,
                                    workloads.free_space_k0(), 1e-10, tree=tree, nthreads=threads,
                                    segments=False)
    t_e = time.perf_counter() - t0
    stopped = (pw < 1e-10) & (che.n_hits > 0)
    segs_e = int(np.sum(np.where(stopped, che.n_hits, np.minimum(che.n_hits + 1, w.max_bounces))))
    out["energy_1e-10_msegments_s"] = round(segs_e / t_e / 1e6, 3)
    pts = workloads.field_points(w.tris, 400.0, 64, 164)
    t0 = time.perf_counter()
    reception.receive(ch.seg, ch.id, ch.t, pts, delta)
    t_r = time.perf_counter() - t0
    out["reception_64_msegments_s"] = round(segs / t_r / 1e6, 3)
    nbr = diffraction.wedges(w.tris)
    t0 = time.perf_counter()
    nd = diffraction.diffract(w.tris, nbr, ch.seg, ch.id, ch.t, delta,
                              diffraction.cone_table(16)).size
    t_d = time.perf_counter() - t0
    out["diffraction_msegments_s"] = round(segs / t_d / 1e6, 3)
    out["diffracted_rays"] = int(nd)
    out["segments"] = segs
    say("recv", "cpu checker:", out)
    return out


def suite_batch(args):
    """Batched trace of the multi-scene set: 8 scenes (1k-200k facets), 64
    transmitters at icosphere levels 6-9 with 1-6 bounces, all in one
    autotuned, graph-captured launch; once per node format, with the hits of
    the formats checked equal."""
    import numpy as np
    import torch

    from paper_2208_10008_amd import BVH, Batch, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    qdefs = workloads.multiscene_queries()
    scenes = [torch.from_numpy(workloads.multiscene_scene(s)[0]).cuda() for s in range(8)]
    dirs = torch.from_numpy(icosphere.directions(9).astype(np.float32)).cuda()
    rays = [rt_rays_from_directions(dirs, icosphere.vertex_count(lv), tx, 1e-4, 2000.0)
            for _, tx, lv, _ in qdefs]
    nrays = sum(r.shape[0] for r in rays)
    say("batch", len(qdefs), "queries,", nrays, "rays")
    result = {"suite": "batch",
              "workload": f"8 scenes (1k-200k facets), {len(qdefs)} transmitters, "
                          f"levels 6-9 ({nrays} rays), 1-6 bounces",
              "command": "python3 bench.py --suite batch", "formats": {}}
    ref = None
    for fmt in args.formats.split(","):
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
        for _ in range(args.reps):
            b.launch()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.reps
        segs = sum(int(torch.clamp(q["n_hits"] + 1, max=q["max_bounces"]).sum().item()) for q in qs)
        same = None
        if ref is None:
            ref = [q["out"].clone() for q in qs]
        else:
            same = all(torch.equal(q["out"], r) for q, r in zip(qs, ref))
        result["formats"][fmt] = {"ms_per_launch": round(ms, 3), "segments": segs,
                                  "mrays_s": round(segs / (ms * 1e-3) / 1e6, 1),
                                  "launch": b.config(), "hits_equal_to_first_format": same}
        say("batch", fmt, result["formats"][fmt])
        b.close()
        for t in trees:
            t.close()
    print(json.dumps(result), flush=True)


def suite_lanes(args):
    """Lanes per ray on the paper-size scenes: for the study room (2,778
    facets) and the campus (7,608 facets), binary and 8-bit node trees with
    leaves of the paper's size (250 / 820), 64 and 16 facets, per icosphere
    level: rt_trace_ex with lanes_per_ray 1, 4, 16, 64 and 0 (the library's
    choice) over the paper's reflection order."""
    import numpy as np
    import torch

    from paper_2208_10008_amd import BVH, SplitParams, rt_rays_from_directions
    from rtgen import icosphere, workloads

    levels = _levels(args.levels)
    timed = event_timer(torch, args.reps)
    dirs = torch.from_numpy(icosphere.directions(max(levels)).astype(np.float32)).cuda()
    res = {"suite": "lanes", "command": "python3 bench.py --suite lanes", "cases": []}
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
                    res["cases"].append({"scene": w.name, "format": fmt, "max_leaf": leaf,
                                         "level": lv, "rays": n, "ms": ms, "fastest": int(best)})
                    say("lanes", f"{w.name} {fmt} leaf {leaf} L{lv}: {ms} fastest G={best}")
                bvh.close()
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU mode (rays are "
              "independent, so each GPU would trace its own slice of the rays with the whole "
              "tree; no collective is needed)", file=sys.stderr)
        sys.exit(2)
    {"step": main_step, "paper": suite_paper, "recv": suite_recv, "batch": suite_batch,
     "lanes": suite_lanes}[args.suite](args)


if __name__ == "__main__":
    main()
