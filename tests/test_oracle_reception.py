"""Pins of the CPU checker's receiving-sphere reception (Sec. III-C, Eq. (4))
against what is fixed independently of it: hand-worked segments, the exact
mean number of receptions of a point source in free space, hole-free
coverage of an icosphere launch, and image-source path lengths."""
import math

import numpy as np
import pytest

import oracle
from oracle import reception as rc
from rtgen import icosphere

from _scenes import ground_and_wall


def keys(rec, *fields):
    return [tuple(int(x) for x in row) for row in zip(*(rec[f] for f in fields))]


def one_chain(segs, hits):
    """segs: list of (o, tmin, d, tmax); hits: list of (id, t) per segment."""
    nb = len(segs)
    seg = np.full((nb, 1, 8), np.nan)
    hid = np.full((nb, 1), -1, np.int32)
    ht = np.full((nb, 1), np.inf)
    for b, ((o, t0, d, t1), (i, t)) in enumerate(zip(segs, hits)):
        seg[b, 0] = [*o, t0, *d, t1]
        hid[b, 0], ht[b, 0] = i, t
    return seg, hid, ht


def test_worked_segments():
    # segment 0: o = 0, d = (2, 0, 0) (not unit), hits facet 7 at t = 5 (x = 10),
    # path length 5 * |d| = 10; segment 1 leaves (10, 0, 0) along (0, 3, 0)
    # (|d| = 3) and misses, tmax = 100.
    seg, hid, ht = one_chain([((0, 0, 0), 0.0, (2, 0, 0), 1000.0),
                              ((10, 0, 0), 0.0, (0, 3, 0), 100.0)],
                             [(7, 5.0), (-1, np.inf)])
    # R1 = (4, 0.3, 0.4): foot at s = 2 (x = 4), dist 0.5, l = sqrt(16.25)
    # R2 = (12, -1, 0): beyond the hit point x = 10 on segment 0 (s = 6 > 5),
    #      behind the start of segment 1 (s = -1/3): never received
    # R3 = (10.6, 30, -0.8): segment 1, foot s = 10, dist 1, l = 10 + sqrt(900 + 1)
    R = np.array([[4, 0.3, 0.4], [12, -1, 0], [10.6, 30, -0.8]], np.float64)
    l1 = math.sqrt(16.25)
    l3 = 10 + math.sqrt(901.0)
    # delta just above / below the threshold sqrt(3) dist / l of R1 and R3
    d1, d3 = math.sqrt(3) * 0.5 / l1, math.sqrt(3) * 1.0 / l3
    got = rc.receive(seg, hid, ht, R, d1 * 1.001)
    assert keys(got, "rx", "ray", "order") == [(0, 0, 0), (2, 0, 1)]   # d3 < d1
    assert abs(got["l"][0] - l1) < 1e-14 and abs(got["dist"][0] - 0.5) < 1e-14
    assert abs(got["l"][1] - l3) < 1e-12 and abs(got["dist"][1] - 1.0) < 1e-12
    got = rc.receive(seg, hid, ht, R, d3 * 1.001)
    assert keys(got, "rx", "order") == [(2, 1)]
    got = rc.receive(seg, hid, ht, R, d3 * 0.999)
    assert got.size == 0
    # R2 beyond the hit point stays unreceived even with a huge sphere
    got = rc.receive(seg, hid, ht, R[1:2], 10.0)
    assert got.size == 0
    # the end of a segment that missed is its tmax: R on segment 1 at s = 200
    got = rc.receive(seg, hid, ht, np.array([[10, 600, 0.0]]), 1.0)
    assert got.size == 0
    got = rc.receive(seg, hid, ht, np.array([[10, 299, 0.0]]), 1e-9)
    assert keys(got, "order") == [(1,)] and got["dist"][0] == 0.0


def test_segments_after_a_miss_are_not_tested():
    seg, hid, ht = one_chain([((0, 0, 0), 0.0, (1, 0, 0), 10.0),
                              ((5, 5, 5), 0.0, (1, 0, 0), 10.0)],
                             [(-1, np.inf), (3, 1.0)])
    got = rc.receive(seg, hid, ht, np.array([[6, 5, 5.0]]), 1.0)
    assert got.size == 0
    assert rc.receive(seg, hid, ht, np.zeros((0, 3)), 1.0).size == 0


def free_space(level, receivers, delta):
    dirs = icosphere.directions(level)
    rays = icosphere.make_rays((0.0, 0.0, 0.0), dirs, 0.0, 1e6)
    m = rays.shape[0]
    seg = rays.reshape(1, m, 8)
    return rc.receive(seg, np.full((1, m), -1, np.int32), np.full((1, m), np.inf), receivers, delta)


def random_points(n, seed, rmin=10.0, rmax=1000.0):
    g = np.random.default_rng(seed)
    u = g.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * g.uniform(rmin, rmax, size=(n, 1))


def test_free_space_mean_reception_count():
    # a ray at angle theta to the direction of the field point is received
    # iff sin(theta) <= delta / sqrt(3) (theta <= 90 deg); for a direction
    # uniform on the sphere that has probability (1 - cos theta_c) / 2, so the
    # mean count over field points is n_rays times that.
    level = 4
    delta = float(icosphere.edge_angles(level).mean())
    n_rays = icosphere.vertex_count(level)
    R = random_points(6000, 1)
    got = free_space(level, R, delta)
    counts = np.bincount(got["rx"], minlength=R.shape[0])
    theta_c = math.asin(delta / math.sqrt(3))
    expect = n_rays * (1 - math.cos(theta_c)) / 2
    assert abs(counts.mean() - expect) < 0.03 * expect, (counts.mean(), expect)
    # order 0: l is the distance from the source
    np.testing.assert_allclose(got["l"], np.linalg.norm(R[got["rx"]], axis=1), rtol=1e-15)


def test_free_space_coverage_with_the_largest_spacing():
    # with delta the largest angle between adjacent rays, every direction is
    # within delta / sqrt(3) of a ray (the circumradius of the worst facet of
    # the launch triangulation), so no field point is missed
    level = 4
    delta = float(icosphere.edge_angles(level).max())
    R = random_points(6000, 2)
    got = free_space(level, R, delta)
    counts = np.bincount(got["rx"], minlength=R.shape[0])
    assert counts.min() >= 1
    kept = rc.dedup(got, np.full((1, icosphere.vertex_count(level)), -1, np.int32))
    assert np.array_equal(np.bincount(kept["rx"][kept["keep"] == 1], minlength=R.shape[0]),
                          np.ones(R.shape[0], np.int64))
    # the representative is the nearest ray to each field point
    for r in range(0, 6000, 250):
        mine = got[got["rx"] == r]
        assert mine["dist"][kept[kept["rx"] == r]["keep"] == 1][0] == mine["dist"].min()


def chains_from(tris, src, level, max_b, delta_kind="max"):
    dirs = icosphere.directions(level)
    rays = icosphere.make_rays(src, dirs, 1e-4, 1e5)
    ch = oracle.bounces(tris, rays, max_b)
    a = icosphere.edge_angles(level)
    return ch, float(a.max() if delta_kind == "max" else a.mean())


def assert_image_bounds(rec, image):
    """Unfolded, the received ray is a straight line from the image source;
    with F the foot of the perpendicular from the field point R (distance
    dist) and a >= 0 the distance of the last reflection point before F,
    l = |S'F| - a + sqrt(a^2 + dist^2): by the triangle inequality
    l >= |S'R| = image, and l - image <= sqrt(a^2 + dist^2) - a <= dist."""
    tol = 1e-12 * image
    assert np.all(rec["l"] >= image - tol), (rec["l"], image)
    assert np.all(rec["l"] <= image + rec["dist"] + tol), (rec["l"] - image, rec["dist"])


def test_ground_image_source_path_lengths():
    tris = ground_and_wall(half=5000.0, wall_x=4000.0)[:2]     # ground only
    src = (0.0, 0.0, 10.0)
    ch, delta = chains_from(tris, src, 6, 2)
    R = np.array([[50, -30, 1.5], [120, -200, 3.0], [-80, 10, 20.0]])
    got = rc.receive(ch.seg, ch.id, ch.t, R, delta)
    kept = rc.dedup(got, ch.id)
    for r in range(R.shape[0]):
        direct = np.linalg.norm(R[r] - np.array(src))
        image = np.linalg.norm(R[r] - np.array([0.0, 0.0, -10.0]))
        o0 = got[(got["rx"] == r) & (got["order"] == 0)]
        o1 = got[(got["rx"] == r) & (got["order"] == 1)]
        assert o0.size >= 1 and o1.size >= 1
        np.testing.assert_allclose(o0["l"], direct, rtol=1e-12)
        assert_image_bounds(o1, image)
        k = kept[(kept["rx"] == r) & (kept["keep"] == 1)]
        assert sorted(k["order"]) == [0, 1]


def test_ground_then_wall_second_order():
    # ground z = 0 and wall x = 20; source (0, 0, 10), field point
    # (18, -25, 2): the path ground -> wall unfolds to the double image
    # (40, 0, -10) and has length sqrt(22^2 + 25^2 + 12^2); the other order
    # (wall -> ground) would cross the ground plane behind the wall
    tris = ground_and_wall(half=100.0, wall_x=20.0)
    src = (0.0, 0.0, 10.0)
    ch, delta = chains_from(tris, src, 6, 3)
    R = np.array([[18.0, -25.0, 2.0]])
    got = rc.receive(ch.seg, ch.id, ch.t, R, delta)
    o2 = got[got["order"] == 2]
    assert o2.size >= 1
    seqs = {(int(ch.id[0, k]) // 2, int(ch.id[1, k]) // 2) for k in o2["ray"]}
    assert seqs == {(0, 1)}                                  # ground first, then wall
    image = math.sqrt(22 ** 2 + 25 ** 2 + 12 ** 2)
    assert_image_bounds(o2, image)
    kept = rc.dedup(got, ch.id)
    k2 = kept[(kept["order"] == 2) & (kept["keep"] == 1)]
    assert k2.size == len({tuple(ch.id[:2, k]) for k in o2["ray"]})


def test_dedup_tie_goes_to_smaller_ray():
    rec = np.zeros(3, rc.RECEPTION)
    rec["rx"] = 0
    rec["order"] = 1
    rec["ray"] = [5, 2, 9]
    rec["dist"] = [0.25, 0.25, 0.5]
    hid = np.zeros((2, 10), np.int32)
    hid[0, 9] = 1                     # ray 9 hit another facet first: its own path
    out = rc.dedup(rec, hid)
    assert list(out["keep"]) == [0, 1, 1]
