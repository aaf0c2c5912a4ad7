"""Batched trace (rt_batch) on the GPU: every query's results equal the same
query traced alone, bit for bit, whatever the launch shape, order, graph
capture or the other queries in the batch; the full multi-scene set (8
scenes of 1k-200k facets, 64 transmitters) is checked against single-query
runs and, on samples, against the CPU checker."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import workloads

from _parity import compare_hits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NTHREADS = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def small_set():
    """Scenes 0-3 of the multi-scene set (1k-24k facets), scene 1 with 8-bit
    nodes, two queries per scene at icosphere levels 4-6 with 1-6 bounces."""
    rng = np.random.default_rng(7)
    trees, queries = [], []
    for s in range(4):
        tris, half = workloads.multiscene_scene(s)
        fmt = "q4" if s == 1 else "bin2"
        bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=workloads.MULTI_SRC, node_format=fmt))
        trees.append(bvh)
        for _ in range(2):
            tx = (float(rng.uniform(-0.5, 0.5) * half), float(rng.uniform(-0.5, 0.5) * half),
                  float(rng.uniform(5, 40)))
            lv, nb = int(rng.integers(4, 7)), int(rng.integers(1, 7))
            queries.append({"bvh": bvh, "rays": dev(workloads.multiscene_rays(tx, lv)),
                            "max_bounces": nb})
    return trees, queries


def alone(q):
    out, pl, nh = q["bvh"].trace_bounces(q["rays"], q["max_bounces"])
    return out, pl, nh


def fresh(queries):
    return [{k: q[k] for k in ("bvh", "rays", "max_bounces")} for q in queries]


def assert_same(batch_queries, ref):
    for k, (q, (out, pl, nh)) in enumerate(zip(batch_queries, ref)):
        assert torch.equal(q["out"], out), f"query {k}: hits differ"
        assert torch.equal(q["path_len"], pl), f"query {k}: path lengths differ"
        assert torch.equal(q["n_hits"], nh), f"query {k}: hit counts differ"


@pytest.mark.parametrize("mode,order", [("direct", "cost"), ("direct", "given"),
                                        ("queue", "cost"), ("queue", "given")])
def test_batch_equals_each_query_alone(small_set, mode, order):
    _, queries = small_set
    ref = [alone(q) for q in queries]
    b = R.Batch(16)
    qs = fresh(queries)
    assert b.set(qs) == [0] * len(qs)
    b.configure(mode=mode, order=order)
    b.launch()
    torch.cuda.synchronize()
    assert_same(qs, ref)
    b.close()


def test_batch_graph_replays(small_set):
    """Captured graph replayed with eager work between replays; new rays of
    the same shape go through the same graph, a new shape recaptures."""
    _, queries = small_set
    b = R.Batch(16)
    qs = fresh(queries)
    b.set(qs)
    b.configure(graph=True)
    ref = [alone(q) for q in queries]
    for rep in range(3):
        for q in qs:
            q["out"].fill_(-7)
        b.launch()
        torch.cuda.synchronize()
        assert_same(qs, ref)
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        alone(queries[rep])
        torch.cuda.synchronize()
    # same shapes, other rays: the table upload in the graph carries them
    qs2 = fresh(queries)
    for q in qs2:
        q["rays"] = q["rays"].flip(0).contiguous()
    b.set(qs2)
    b.launch()
    torch.cuda.synchronize()
    assert_same(qs2, [alone(q) for q in qs2])
    # a different shape (fewer queries) is captured again
    qs3 = fresh(queries[:3])
    b.set(qs3)
    b.launch()
    torch.cuda.synchronize()
    assert_same(qs3, [alone(q) for q in qs3])
    b.close()


def field_points(bvh_tris_half, rng, m):
    tris, half = bvh_tris_half
    from rtgen import scenes
    return dev(scenes.free_points(rng, half, tris, 1.5, m))


@pytest.mark.parametrize("mode,graph", [("direct", False), ("queue", False), ("direct", True)])
def test_batch_receptions_equal_each_query_alone(small_set, mode, graph):
    """Queries with field points (every other query, both node formats) in
    one batch with plain queries: each gets the reception count and records
    of rt_trace_receive on the same rays alone, and the same chains; the
    counts are cleared by every launch (graph replays included)."""
    from rtgen import icosphere
    trees, queries = small_set
    rng = np.random.default_rng(17)
    delta = float(icosphere.edge_angles(6).mean())
    qs = fresh(queries)
    for k, q in enumerate(qs):
        if k % 2 == 0:
            pos = field_points(workloads.multiscene_scene(k // 2), rng, 12)
            q["receivers"] = R.Receivers(pos, delta, 1 << 16)
    ref = []
    for q in qs:
        if "receivers" in q:
            rcv = R.Receivers(q["receivers"].pos, delta, 1 << 16)
            out, pl, nh = q["bvh"].trace_receive(q["rays"], q["max_bounces"], rcv)
            ref.append((out, pl, nh, rcv))
        else:
            ref.append(alone(q) + (None,))
    b = R.Batch(16)
    assert b.set(qs) == [0] * len(qs)
    b.configure(mode=mode, graph=graph)
    total = 0
    for rep in range(2 if graph else 1):
        b.launch()
        torch.cuda.synchronize()
        for k, (q, (out, pl, nh, rcv)) in enumerate(zip(qs, ref)):
            assert torch.equal(q["out"], out) and torch.equal(q["path_len"], pl), k
            assert torch.equal(q["n_hits"], nh), k
            if rcv is None:
                continue
            got = q["receivers"]
            assert got.count() == rcv.count() <= got.cap, k
            assert np.array_equal(np.sort(got.records(), order=("rx", "ray", "order")),
                                  np.sort(rcv.records(), order=("rx", "ray", "order"))), k
            total += got.count()
    log(f"{mode} graph={graph}: {total} receptions")
    assert total > 0
    b.close()


def test_batch_receivers_are_checked(small_set):
    _, queries = small_set
    qs = fresh(queries[:3])
    pos = dev(np.zeros((4, 3)))
    qs[0]["receivers"] = R.Receivers(pos, float("nan"), 16)    # bad delta
    qs[1]["receivers"] = R.Receivers(pos, 0.01, 16)
    b = R.Batch(4)
    st = b.set(qs)
    assert st[0] != 0 and st[1] == 0 and st[2] == 0
    b.launch()
    torch.cuda.synchronize()
    ref = alone(qs[2])
    assert torch.equal(qs[2]["out"], ref[0])
    b.close()


def test_batch_autotune_keeps_results(small_set):
    _, queries = small_set
    ref = [alone(q) for q in queries]
    b = R.Batch(16)
    qs = fresh(queries)
    b.set(qs)
    ms = b.autotune(reps=2)
    log("autotune", b.config(), "%.3f ms" % ms)
    assert ms > 0
    for q in qs:
        q["out"].fill_(-7)
    b.launch()
    torch.cuda.synchronize()
    assert_same(qs, ref)
    b.close()


def test_batch_invalid_queries_are_left_out(small_set):
    import ctypes
    _, queries = small_set
    good = fresh(queries[:2])
    ref = [alone(q) for q in good]
    b = R.Batch(8)
    statuses = b.set(good)
    assert statuses == [0, 0]
    # raw table with a NULL tree and a bad bounce count between good queries
    arr = (R.rt_query * 4)()
    for k, q in zip((0, 3), good):
        arr[k].bvh = q["bvh"].handle
        arr[k].rays = q["rays"].data_ptr()
        arr[k].n = q["rays"].shape[0]
        arr[k].max_bounces = q["max_bounces"]
        arr[k].out = q["out"].data_ptr()
        arr[k].path_len = q["path_len"].data_ptr()
        arr[k].n_hits = q["n_hits"].data_ptr()
    arr[1].bvh = None
    arr[1].n = 10
    arr[2] = arr[0]
    arr[2].max_bounces = 0
    for q in good:
        q["out"].fill_(-7)
    assert R.load().rt_batch_set(b.handle, arr, 4) == 0
    assert [arr[k].status for k in range(4)] == [0, R.RT_EINVAL, R.RT_EINVAL, 0]
    b.launch()
    torch.cuda.synchronize()
    assert_same(good, ref)
    with pytest.raises(R.RtError):  # more queries than the batch holds
        R.Batch(1).set(fresh(queries[:2]))
    b.close()


@pytest.mark.slow
def test_multiscene_batch_full_size():
    """Config 4 at full size: 8 scenes (1k-200k facets), 64 transmitters at
    levels 6-9 (40,962-2,621,442 rays) with 1-6 bounces, one autotuned,
    graph-captured launch; every query equals its single-query run bit for
    bit, and 2,000 sampled primary rays per query match the CPU checker."""
    t0 = time.time()
    qdefs = workloads.multiscene_queries()
    scenes = [workloads.multiscene_scene(s)[0] for s in range(8)]
    trees = [R.BVH(dev(t), R.SplitParams(alpha=0.4, src=workloads.MULTI_SRC)) for t in scenes]
    qs = []
    host_rays = []
    for s, tx, lv, nb in qdefs:
        r = workloads.multiscene_rays(tx, lv)
        host_rays.append(r)
        qs.append({"bvh": trees[s], "rays": dev(r), "max_bounces": nb})
    nrays = sum(r.shape[0] for r in host_rays)
    log("config 4:", len(qs), "queries,", nrays, "rays, setup %.1fs" % (time.time() - t0))
    b = R.Batch(len(qs))
    b.set(qs)
    ms = b.autotune(reps=1)
    b.configure(**{**b.config(), "graph": True})
    for q in qs:
        q["out"].fill_(-7)
    b.launch()
    torch.cuda.synchronize()
    log("config 4 batch: %.2f ms per launch (autotuned %s)" % (ms, b.config()))
    for k, q in enumerate(qs):
        out, pl, nh = alone(q)
        assert torch.equal(q["out"], out), f"query {k}: hits differ from the single-query run"
        assert torch.equal(q["path_len"], pl) and torch.equal(q["n_hits"], nh), f"query {k}"
        del out, pl, nh
    rng = np.random.default_rng(3)
    otrees = {}
    for k, ((s, tx, lv, nb), q, r) in enumerate(zip(qdefs, qs, host_rays)):
        if s not in otrees:
            otrees[s] = oracle.build_tree(scenes[s], oracle.SplitParams(alpha=0.4,
                                                                        src=workloads.MULTI_SRC))
        pick = np.sort(rng.choice(r.shape[0], size=min(2000, r.shape[0]), replace=False))
        o = q["out"][0].cpu().numpy()[pick]
        ids, t = o[:, 0], o[:, 1].view(np.float32).astype(np.float64)
        ref = oracle.trace_bvh(otrees[s], r[pick], nthreads=NTHREADS)
        compare_hits(scenes[s], r[pick], ids, t, ref)
    log("config 4 checked in %.1fs" % (time.time() - t0))
    b.close()
