"""Several lanes per ray (GPU, through the C ABI).

With lanes_per_ray G > 1 the G lanes of a group trace one reflection chain
together and split every leaf's facets; the closest hit is merged by the same
rule (smaller t, then smaller facet id).  The chains must be bit-identical to
the one-lane kernel's (hits, t, u, v, path lengths, hit counts) for every node
format, on the paper's large-leaf trees (Sec. IV: 250 and 820 facets per
leaf) and on small leaves, with ray counts that leave a wave partly empty;
and the first segments must follow the closest-hit rule against brute force
(tests/_parity.py).  The library's own choice of G (rt_trace_receive, the
plain trace calls) is checked through the receptions, which must equal the
two-pass form computed from one-lane segments.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import icosphere, workloads

from _parity import compare_hits, keyed

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
def indoor():
    return workloads.paper_indoor()


@pytest.fixture(scope="module")
def outdoor():
    return workloads.paper_outdoor()


def chains(bvh, rays, nb, lanes):
    out, pl, nh = bvh.trace_bounces(rays, nb, lanes_per_ray=lanes)
    return out.cpu().numpy(), pl.cpu().numpy(), nh.cpu().numpy()


def assert_same_chains(a, b, what):
    assert np.array_equal(a[0], b[0]), what + ": hit records differ"
    assert np.array_equal(a[1].view(np.uint64), b[1].view(np.uint64)), what + ": path lengths differ"
    assert np.array_equal(a[2], b[2]), what + ": hit counts differ"


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
@pytest.mark.parametrize("which", ["indoor", "outdoor"])
def test_lanes_equal_one_lane_on_the_paper_trees(request, which, fmt):
    w = request.getfixturevalue(which)
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf,
                                           node_format=fmt))
    rays_np = w.rays(5)[:9000 + 37]               # ragged: not a multiple of 64
    rays = dev(rays_np)
    nb = w.max_bounces + 1
    ref = chains(bvh, rays, nb, 1)
    for g in (4, 16, 64):
        assert_same_chains(chains(bvh, rays, nb, g), ref, f"{w.name} {fmt} G={g}")
    # first segments against brute force
    ids, t = ref[0][0, :, 0], ref[0][0, :, 1].view(np.float32)
    compare_hits(w.tris, rays_np, ids, t, oracle.brute(w.tris, rays_np, nthreads=NTHREADS))
    log(f"{w.name} {fmt}: {rays_np.shape[0]} chains equal for G = 1, 4, 16, 64; "
        f"{int((ref[0][..., 0] >= 0).sum())} hits")
    bvh.close()


@pytest.mark.parametrize("max_leaf", [4, 16, 100])
def test_lanes_equal_one_lane_on_the_city(max_leaf):
    w = workloads.city24k(level=5, max_bounces=4)
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=0.4, src=w.tx, max_leaf=max_leaf))
    rays = dev(w.rays[:5000 + 5])
    ref = chains(bvh, rays, 4, 1)
    for g in (4, 16, 64):
        assert_same_chains(chains(bvh, rays, 4, g), ref, f"city max_leaf {max_leaf} G={g}")
    bvh.close()


@pytest.mark.parametrize("n_rays", [1, 3, 17, 63, 65])
@pytest.mark.parametrize("n_tris", [1, 5, 16])
def test_lanes_on_one_leaf_scenes(n_rays, n_tris):
    """The root is a leaf and the facet array ends inside the lanes' first
    round: lanes past the last facet must neither test nor read it."""
    rng = np.random.default_rng(n_tris * 100 + n_rays)
    tris = (rng.random((n_tris, 9)) * 4.0 - 2.0).astype(np.float32)
    tris[:, 2::3] += 5.0                          # in front of the origin along +z
    d = icosphere.directions(3)[:n_rays].copy()
    d[:, 2] = np.abs(d[:, 2]) + 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays_np = icosphere.make_rays((0.0, 0.0, 0.0), d, 0.0, 100.0)
    bvh = R.BVH(dev(tris), R.SplitParams(src=(0.0, 0.0, 0.0), max_leaf=16))
    rays = dev(rays_np)
    ref = chains(bvh, rays, 3, 1)
    for g in (4, 16, 64):
        assert_same_chains(chains(bvh, rays, 3, g), ref, f"{n_tris} facets, {n_rays} rays, G={g}")
    compare_hits(tris, rays_np, ref[0][0, :, 0], ref[0][0, :, 1].view(np.float32),
                 oracle.brute(tris, rays_np, nthreads=1))
    bvh.close()


def test_library_choice_in_the_reception_path(indoor):
    """rt_trace_receive picks several lanes per ray for this small launch on a
    250-facet-leaf tree; its receptions must equal those of the one-lane
    chains' segments tested afterwards (rt_receive_segments)."""
    w = indoor
    lv = 4
    rays = dev(w.rays(lv))
    n, nb = rays.shape[0], w.max_bounces
    delta = float(icosphere.edge_angles(lv).mean())
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf))
    rx = torch.tensor([w.rx, (2.0, 3.0, 1.2), (6.5, 4.0, 2.5)], dtype=torch.float64, device="cuda")
    fused = R.Receivers(rx, delta, 1 << 14)
    out, pl, nh = bvh.trace_receive(rays, nb, fused)
    seg = torch.empty((nb, n, 8), dtype=torch.float32, device="cuda")
    out1, pl1, nh1 = bvh.trace_bounces(rays, nb, seg_rays=seg)
    assert torch.equal(out, out1) and torch.equal(nh, nh1)
    assert np.array_equal(pl.cpu().numpy().view(np.uint64), pl1.cpu().numpy().view(np.uint64))
    two = R.Receivers(rx, delta, 1 << 14)
    R.rt_receive_segments(seg, out1, nb, two)
    ka, kb = keyed(fused.records()), keyed(two.records())
    assert ka[1] == kb[1] and ka[0].size > 0
    assert np.array_equal(ka[0]["l"], kb[0]["l"]) and np.array_equal(ka[0]["dist"], kb[0]["dist"])
    log(f"indoor L{lv}: {n} rays, {ka[0].size} receptions equal")
    bvh.close()


def test_lanes_argument_checks(indoor):
    w = indoor
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf))
    rays = dev(w.rays(2))
    n = rays.shape[0]
    out = bvh.hits_buffer(n, 2)
    seg = torch.empty((2, n, 8), dtype=torch.float32, device="cuda")
    stats = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    lib = R.load()

    def call(**kw):
        o = R.rt_trace_opts()
        o.seg_rays = kw.get("seg", None)
        o.ray_stats = kw.get("stats", None)
        o.grid, o.lanes_per_ray = kw.get("grid", 0), kw["lanes"]
        return lib.rt_trace_ex(bvh.handle, rays.data_ptr(), n, 2, out.data_ptr(), None, None,
                               ctypes.byref(o), None)

    for bad in (2, 3, 8, 32, 128, -1):
        assert call(lanes=bad) == R.RT_EINVAL
        assert b"lanes_per_ray" in lib.rt_last_error()
    assert call(lanes=4, seg=seg.data_ptr()) == R.RT_EINVAL
    assert call(lanes=16, stats=stats.data_ptr()) == R.RT_EINVAL
    assert call(lanes=64, grid=8) == R.RT_EINVAL
    for ok in (0, 1, 4, 16, 64):
        assert call(lanes=ok) == R.RT_OK
    torch.cuda.synchronize()
    bvh.close()


@pytest.mark.parametrize("level", [3, 5, 6])
def test_library_choice_in_the_energy_path(indoor, level):
    """rt_trace_energy on a 250-facet-leaf tree picks 64 (levels 3, 5) or 16
    (level 6) lanes per ray; with a zero threshold no chain stops by energy,
    so its chains must equal the one-lane fixed-order chains bit for bit, and
    every chain with a hit reports a positive power."""
    w = indoor
    rays = dev(w.rays(level))
    n, nb = rays.shape[0], 4
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf))
    e = R.Energy(dev(w.material), dev(workloads.REFLECTION), workloads.free_space_k0(), 0.0,
                 power=torch.full((n,), -1.0, dtype=torch.float64, device="cuda"))
    out, pl, nh = bvh.trace_energy(rays, nb, e)
    ref = chains(bvh, rays, nb, 1)
    assert_same_chains((out.cpu().numpy(), pl.cpu().numpy(), nh.cpu().numpy()), ref,
                       f"energy, level {level}")
    pw, hn = e.power.cpu().numpy(), ref[2]
    assert np.all(pw[hn == 0] == 0) and np.all(pw[hn > 0] > 0)
    bvh.close()


@pytest.mark.parametrize("which", ["indoor", "outdoor"])
def test_lanes_at_full_size(request, which):
    """Level 9 (2,621,442 rays, the paper regime's largest launch): 4 and 16
    lanes per ray and the library's own choice equal one lane per ray bit for
    bit on every chain."""
    w = request.getfixturevalue(which)
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf))
    rays = dev(w.rays(9))
    nb = w.max_bounces
    ref = chains(bvh, rays, nb, 1)
    for g in (4, 16, 0):
        assert_same_chains(chains(bvh, rays, nb, g), ref, f"{w.name} level 9 G={g}")
    log(f"{w.name} level 9: {rays.shape[0]} chains equal for G = 4, 16 and the library's choice")
    bvh.close()
