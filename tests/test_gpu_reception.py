"""Receiving-sphere reception (Sec. III-C, Eq. (4)) on the GPU, through the
C ABI, against the CPU checker (oracle.reception).

* Stored chains (synthetic, seeded): the GPU kernel and the checker evaluate
  the same float64 expression in the same order on the same float32 inputs,
  so the sets of (field point, ray, order) must be equal and l, dist
  bit-identical; duplicate grouping must keep the same records.
* Traced chains: the fused trace+reception kernel must give exactly what the
  stored-chain kernel gives on the segments the tracer wrote, and leave the
  chains themselves unchanged.
* Against the checker's own float64 chains (reflections in float64): on rays
  whose chains agree with the checker's (same facets, hit distances within
  1e-5, clean margins), receptions must agree except where the checker's own
  test lies within 5e-3 of its threshold (sqrt(3) dist / (l delta) = 1) or
  the foot of the perpendicular within 5e-3 of the segment's length of an end
  -- a float32 segment differs from the float64 one by about 1e-5 of the path
  length, which moves sqrt(3) dist / (l delta) by about 1e-5 sqrt(3) / delta.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from oracle import reception as rc
from rtgen import icosphere, scenes, workloads

from _parity import BAND, agree_with_checker, keyed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def hits_tensor(hid, ht):
    """[max_b, m] ids and float32 t -> rt_hit int32 [max_b, m, 4] on the device."""
    h = np.zeros(hid.shape + (4,), np.int32)
    h[..., 0] = hid
    h[..., 1] = np.asarray(ht, np.float32).view(np.int32)
    return dev(h)


def gpu_segments(seg, hid, ht, rx, delta, cap=1 << 16):
    recv = R.Receivers(dev(rx), delta, cap)
    hits = hits_tensor(hid, ht)
    R.rt_receive_segments(dev(seg), hits, seg.shape[0], recv)
    return recv, hits


@pytest.mark.parametrize("seed,groups,n_rx", [(0, 600, 256), (1, 37, 5), (2, 1, 1)])
def test_stored_chains_equal_the_checker_bit_for_bit(seed, groups, n_rx):
    seg, hid, ht, rx = workloads.reception_chains(seed, groups=groups, n_rx=n_rx)
    delta = 0.02
    recv, hits = gpu_segments(seg, hid, ht, rx, delta)
    got = recv.records()
    ref = rc.receive(seg, hid, ht, rx, delta)
    assert recv.count() == ref.size
    g, gk = keyed(got)
    r, rk = keyed(ref)
    assert gk == rk
    assert np.array_equal(g["l"].view(np.int64), r["l"].view(np.int64))
    assert np.array_equal(g["dist"].view(np.int64), r["dist"].view(np.int64))
    log(f"seed {seed}: {ref.size} receptions, {seg.shape[1]} rays")
    # duplicate grouping: same records kept
    recv.dedup(hits, seg.shape[0])
    kept = recv.records()
    kg, kk = keyed(kept)
    kr, _ = keyed(rc.dedup(ref, hid))
    assert kk == rk and np.array_equal(kg["keep"], kr["keep"])
    log(f"  kept {int(kr['keep'].sum())}")


def test_stored_chains_edge_cases():
    seg, hid, ht, rx = workloads.reception_chains(3, groups=50, n_rx=40)
    full = rc.receive(seg, hid, ht, rx, 0.02)
    assert full.size > 20
    # capacity smaller than the count: count is complete, records are a subset
    recv, _ = gpu_segments(seg, hid, ht, rx, 0.02, cap=7)
    assert recv.count() == full.size
    sub = recv.records()
    assert sub.size == 7
    _, fk = keyed(full)
    assert set(keyed(sub)[1]) <= set(fk)
    # cap 0 and no field points: nothing stored, count set
    recv, _ = gpu_segments(seg, hid, ht, rx, 0.02, cap=0)
    assert recv.count() == full.size and recv.records().size == 0
    recv, _ = gpu_segments(seg, hid, ht, rx[:0], 0.02)
    assert recv.count() == 0
    # delta 0: only field points exactly on a segment
    recv, _ = gpu_segments(seg, hid, ht, rx, 0.0)
    assert recv.count() == rc.receive(seg, hid, ht, rx, 0.0).size
    # an empty ray set resets the count
    recv, _ = gpu_segments(seg[:, :0], hid[:, :0], ht[:, :0], rx, 0.02)
    assert recv.count() == 0
    # NaN field point: never received
    bad = rx.copy()
    bad[0] = np.nan
    recv, _ = gpu_segments(seg, hid, ht, bad, 0.02)
    assert not np.any(recv.records()["rx"] == 0)


@pytest.fixture(scope="module")
def micro_city():
    """Multi-scene scene 1 (about 4k facets on an 816 m square) and a Tx at
    25 m outside the buildings near the centre."""
    tris, half = workloads.multiscene_scene(1)
    src = scenes.free_point(np.random.default_rng(3), half * 0.3, tris, 25.0)
    return tris, half, src


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_fused_equals_stored_chain_kernel(micro_city, fmt):
    tris, half, src = micro_city
    level, nb = 6, 4
    rays = workloads.multiscene_rays(src, level)
    rx = workloads.field_points(tris, half * 0.5, 32, 5)
    delta = float(icosphere.edge_angles(level).mean())
    bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=src, node_format=fmt))
    d_rays = dev(rays)
    recv = R.Receivers(dev(rx), delta, 1 << 16)
    out, pl, nh = bvh.trace_receive(d_rays, nb, recv)
    seg = torch.full((nb, rays.shape[0], 8), float("nan"), dtype=torch.float32, device="cuda")
    out2, pl2, nh2 = bvh.trace_bounces(d_rays, nb, seg_rays=seg)
    torch.cuda.synchronize()
    assert torch.equal(out, out2) and torch.equal(pl, pl2) and torch.equal(nh, nh2)
    recv2 = R.Receivers(dev(rx), delta, 1 << 16)
    R.rt_receive_segments(seg, out2, nb, recv2)
    a, ak = keyed(recv.records())
    b, bk = keyed(recv2.records())
    assert recv.count() == recv2.count() and ak == bk
    assert np.array_equal(a["l"], b["l"]) and np.array_equal(a["dist"], b["dist"])
    log(f"{fmt}: {len(ak)} receptions at {rx.shape[0]} field points")
    assert len(ak) > 100


def test_traced_receptions_against_float64_chains(micro_city):
    tris, half, src = micro_city
    level, nb = 6, 4
    rays = workloads.multiscene_rays(src, level)
    rx = workloads.field_points(tris, half * 0.5, 24, 6)
    delta = float(icosphere.edge_angles(level).mean())
    p = R.SplitParams(alpha=0.4, src=src)
    bvh = R.BVH(dev(tris), p)
    recv = R.Receivers(dev(rx), delta, 1 << 16)
    out, _, _ = bvh.trace_receive(dev(rays), nb, recv)
    o = out.cpu().numpy()
    ids_g, t_g = o[..., 0], o[..., 1].view(np.float32).astype(np.float64)
    st = agree_with_checker(tris, rays, rx, delta, nb, oracle.SplitParams(alpha=0.4, src=src),
                            recv.records(), ids_g, t_g)
    log("traced receptions vs float64 chains:", st)
    assert st["compared"] > 0.95 * st["checker"]


@pytest.mark.slow
def test_city24k_full_size_receptions():
    """The benchmark's scene and launch (city24k, level 9, 6 bounces) with 64
    field points: the fused kernel equals the stored-chain kernel on all
    2.6M chains; on 20,000 random rays plus every ray with a reception the
    receptions agree with those on the checker's chains."""
    w = workloads.city24k()
    nb = w.max_bounces
    rx = workloads.field_points(w.tris, 1000.0 * 0.4, 64, 9)
    delta = float(icosphere.edge_angles(w.level).mean())
    p = R.SplitParams(alpha=0.4, src=w.tx)
    bvh = R.BVH(dev(w.tris), p)
    d_rays = dev(w.rays)
    recv = R.Receivers(dev(rx), delta, 1 << 20)
    out, _, _ = bvh.trace_receive(d_rays, nb, recv)
    seg = torch.empty((nb, w.n_rays, 8), dtype=torch.float32, device="cuda")
    out2, _, _ = bvh.trace_bounces(d_rays, nb, seg_rays=seg)
    assert torch.equal(out, out2)
    recv2 = R.Receivers(dev(rx), delta, 1 << 20)
    R.rt_receive_segments(seg, out2, nb, recv2)
    del seg
    a, ak = keyed(recv.records())
    b, bk = keyed(recv2.records())
    assert recv.count() <= recv.cap and ak == bk
    assert np.array_equal(a["l"], b["l"]) and np.array_equal(a["dist"], b["dist"])
    log(f"city24k: {len(ak)} receptions at 64 field points")
    # sample: 20,000 random rays (a missed reception shows there) plus every
    # ray the GPU reports (so that each reported reception is checked)
    rng = np.random.default_rng(11)
    pick = np.union1d(rng.choice(w.n_rays, 20_000, replace=False), a["ray"])
    o = out.cpu().numpy()[:, pick]
    ids_g, t_g = o[..., 0], o[..., 1].view(np.float32).astype(np.float64)
    sub = a[np.isin(a["ray"], pick)].copy()
    sub["ray"] = np.searchsorted(pick, sub["ray"])
    st = agree_with_checker(w.tris, w.rays[pick], rx, delta, nb,
                            oracle.SplitParams(alpha=0.4, src=w.tx), sub, ids_g, t_g)
    log("city24k sampled receptions vs float64 chains:", st)
    assert st["compared"] > 0.9 * st["checker"]
