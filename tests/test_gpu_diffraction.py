"""Edge diffraction (Sec. III-B) on the GPU through the C ABI, against the CPU
checker (oracle.diffraction).

* Wedges: the neighbour of every half-edge equals the checker's exactly.
* Diffraction of stored chains: on chains the checker traced (rounded to
  float32 as the tracer stores them), the GPU and the checker evaluate the
  same float64 expressions in the same order, so the diffracted rays must be
  the same records bit for bit.
* The diffracted rays are ordinary rays: traced on the GPU they follow the
  closest-hit rule against the checker (tests/_parity.py).
* The whole GPU pipeline on the benchmark launch (trace with stored
  segments, wedges, diffraction): every diffracted ray starts on its edge and
  keeps the incident angle with it (Keller's law).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from oracle import diffraction as df
from rtgen import icosphere, scenes, workloads

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


def scene(name):
    if name == "room":
        return workloads.paper_indoor().tris
    if name == "campus":
        return workloads.paper_outdoor().tris
    if name == "city1":
        return workloads.multiscene_scene(1)[0]
    return workloads.city24k().tris


@pytest.mark.parametrize("name", ["room", "campus", "city1", "city24k"])
def test_wedges_equal_the_checker(name):
    tris = scene(name)
    gpu = R.rt_wedges(dev(tris)).cpu().numpy()
    ref = df.wedges(tris)
    assert np.array_equal(gpu, ref)
    log(f"{name}: {tris.shape[0]} facets, wedge half-edges {(ref >= 0).sum()}, free {(ref == -1).sum()}")


def test_wedges_negative_zero_and_duplicates():
    t = scenes._pack(scenes._box(0.0, 0.0, 0.0, 2.0, 2.0, 2.0)).copy()
    t[t == 0.0] = -0.0                       # -0 and +0 are the same point
    t = np.concatenate([t, t[:1]])           # a duplicated facet: its edges have 3 facets
    assert np.array_equal(R.rt_wedges(dev(t)).cpu().numpy(), df.wedges(t))
    with pytest.raises(R.RtError):
        bad = t.copy()
        bad[3, 4] = np.nan
        R.rt_wedges(dev(bad))


def stored_checker_chains(tris, src, level, nb, max_leaf=4, alpha=0.4):
    rays = icosphere.make_rays(src, icosphere.directions(level), 1e-4, 2000.0)
    tree = oracle.build_tree(tris, oracle.SplitParams(alpha=alpha, src=src, max_leaf=max_leaf))
    ch = oracle.bounces(tris, rays, nb, tree=tree, nthreads=NTHREADS)
    seg32 = ch.seg.astype(np.float32)
    t32 = ch.t.astype(np.float32)
    return rays, ch, seg32, t32


def hits_tensor(hid, ht):
    h = np.zeros(hid.shape + (4,), np.int32)
    h[..., 0] = hid
    h[..., 1] = np.asarray(ht, np.float32).view(np.int32)
    return dev(h)


def sort_records(r):
    return np.sort(r, order=("ray", "order", "cone"))


CASES = {"room": lambda: (workloads.paper_indoor().tris, workloads.paper_indoor().tx, 5, 3, 0.3),
         "city1": lambda: (workloads.multiscene_scene(1)[0],
                           scenes.free_point(np.random.default_rng(3),
                                             workloads.multiscene_scene(1)[1] * 0.3,
                                             workloads.multiscene_scene(1)[0], 25.0), 6, 3, 0.05)}


@pytest.mark.parametrize("name", sorted(CASES))
def test_diffraction_of_checker_chains_bit_for_bit(name):
    tris, src, level, nb, delta = CASES[name]()
    rays, ch, seg32, t32 = stored_checker_chains(tris, src, level, nb)
    cone = df.cone_table(16)
    ref = sort_records(df.diffract(tris, df.wedges(tris), seg32, ch.id, t32, delta, cone))
    d_tris = dev(tris)
    nbr = R.rt_wedges(d_tris)
    cap = 1 << 20
    out, count = R.rt_diffract_segments(d_tris, nbr, dev(seg32), hits_tensor(ch.id, t32), nb, delta,
                                        dev(cone), cap)
    got = sort_records(R.diffracted_records(out, count, cap))
    assert int(count.item()) == ref.size and ref.size > 50
    for f in ("ray", "order", "facet", "edge", "cone"):
        assert np.array_equal(got[f], ref[f]), f
    assert np.array_equal(got["path"].view(np.int64), ref["path"].view(np.int64))
    ray8 = np.concatenate([ref["o"], ref["tmin"][:, None], ref["d"], ref["tmax"][:, None]], 1)
    assert np.array_equal(got["ray8"].view(np.int32), ray8.astype(np.float32).view(np.int32))
    log(f"{name}: {ref.size} diffracted rays from {len(np.unique(ref['ray']))} rays")
    # the checker's diffracted rays traced on the GPU follow the closest-hit rule
    bvh = R.BVH(d_tris, R.SplitParams(alpha=0.4, src=src))
    out_h = bvh.trace(dev(ray8.astype(np.float32)))
    o = out_h.cpu().numpy()
    tree = oracle.build_tree(tris, oracle.SplitParams(alpha=0.4, src=src))
    hr = oracle.trace_bvh(tree, ray8.astype(np.float32), nthreads=NTHREADS)
    st = compare_hits(tris, ray8.astype(np.float32), o[:, 0], o[:, 1].view(np.float32), hr)
    log(f"  traced: {st}")


def test_diffraction_edge_cases():
    tris, src, level, nb, delta = CASES["room"]()
    rays, ch, seg32, t32 = stored_checker_chains(tris, src, 4, nb)
    d_tris = dev(tris)
    nbr = R.rt_wedges(d_tris)
    cone = dev(df.cone_table(8))
    full = df.diffract(tris, df.wedges(tris), seg32, ch.id, t32, delta, df.cone_table(8))
    assert full.size > 20
    out, count = R.rt_diffract_segments(d_tris, nbr, dev(seg32), hits_tensor(ch.id, t32), nb, delta,
                                        cone, 5)
    assert int(count.item()) == full.size and R.diffracted_records(out, count, 5).size == 5
    out, count = R.rt_diffract_segments(d_tris, nbr, dev(seg32), hits_tensor(ch.id, t32), nb, delta,
                                        cone[:0], 16)
    assert int(count.item()) == 0
    out, count = R.rt_diffract_segments(d_tris, nbr, dev(seg32), hits_tensor(ch.id, t32), nb, 0.0,
                                        cone, 1 << 16)
    assert int(count.item()) == df.diffract(tris, df.wedges(tris), seg32, ch.id, t32, 0.0,
                                            df.cone_table(8)).size


@pytest.mark.slow
def test_city24k_pipeline_keller_law():
    w = workloads.city24k()
    nb = w.max_bounces
    d_tris = dev(w.tris)
    bvh = R.BVH(d_tris, R.SplitParams(alpha=0.4, src=w.tx))
    seg = torch.empty((nb, w.n_rays, 8), dtype=torch.float32, device="cuda")
    out, _, _ = bvh.trace_bounces(dev(w.rays), nb, seg_rays=seg)
    nbr = R.rt_wedges(d_tris)
    delta = float(icosphere.edge_angles(w.level).mean())
    cone = df.cone_table(16)
    cap = 1 << 22
    rec_t, count = R.rt_diffract_segments(d_tris, nbr, seg, out, nb, delta, dev(cone), cap)
    rec = R.diffracted_records(rec_t, count, cap)
    log(f"city24k: {int(count.item())} diffracted rays")
    assert 0 < rec.size <= cap
    t3 = w.tris.reshape(-1, 3, 3).astype(np.float64)
    a = t3[rec["facet"], rec["edge"]]
    b = t3[rec["facet"], (rec["edge"] + 1) % 3]
    e = b - a
    ehat = e / np.linalg.norm(e, axis=1, keepdims=True)
    q = rec["ray8"][:, 0:3].astype(np.float64)
    # q on the edge segment (float32 rounding of a point on it)
    s = ((q - a) * e).sum(1) / (e * e).sum(1)
    off = np.linalg.norm(q - (a + s[:, None] * e), axis=1)
    scale = np.abs(a).max(1) + np.abs(b).max(1) + 1.0
    assert np.all((s > -1e-6) & (s < 1 + 1e-6)) and np.all(off <= 1e-6 * scale)
    # Keller's law against the parent segment's direction
    sg = seg.cpu().numpy()
    dpar = sg[rec["order"], rec["ray"], 4:7].astype(np.float64)
    ihat = dpar / np.linalg.norm(dpar, axis=1, keepdims=True)
    dk = rec["ray8"][:, 4:7].astype(np.float64)
    assert np.all(np.abs((dk * ehat).sum(1) - (ihat * ehat).sum(1)) <= 1e-6)
    assert np.all(np.abs(np.linalg.norm(dk, axis=1) - 1) <= 1e-6)
    # the diffracted rays trace (as ordinary rays) without error
    traced = bvh.trace(R.diffracted_rays(rec_t, rec.size))
    assert traced.shape[0] == rec.size
