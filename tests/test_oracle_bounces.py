"""Pins of the CPU checker's reflection chains (Sec. III-B: reflected rays
until the set order) against image-source closed forms."""
import numpy as np

import oracle

from _scenes import corridor, ground_and_wall


def test_ground_then_wall_image_source():
    tris = ground_and_wall(wall_x=20.0)
    d = (np.float32([1, 0, -1]) / np.float32(np.sqrt(2))).astype(np.float32)
    rays = np.array([[0, 0, 10, 1e-4, d[0], d[1], d[2], 1e3]], dtype=np.float32)
    for tree in (None, oracle.build_tree(tris, oracle.SplitParams(max_leaf=1))):
        c = oracle.bounces(tris, rays, 4, tree=tree)
        assert c.n_hits[0] == 2
        assert c.id[0, 0] in (0, 1) and c.id[1, 0] in (2, 3) and c.id[2, 0] == -1
        dx, dz = float(d[0]), float(d[2])
        norm = np.sqrt(dx * dx + dz * dz)
        # ground at t = 10/|dz|, wall at t = 10/dx; the reflected direction
        # keeps |d|; the image of the source in the ground is (0, 0, -10)
        assert abs(c.t[0, 0] - 10 / abs(dz)) < 1e-13 and abs(c.t[1, 0] - 10 / dx) < 1e-12
        expect = (10 / abs(dz) + 10 / dx) * norm
        assert abs(c.path_len[0] - expect) < 1e-12 * expect
        assert abs(c.path_len[0] - np.hypot(20, 20)) < 1e-5
        np.testing.assert_allclose(c.seg[1, 0, 0:3], [10, 0, 0], atol=1e-12)
        np.testing.assert_allclose(c.seg[2, 0, 0:3], [20, 0, 10], atol=1e-12)
        np.testing.assert_allclose(c.seg[2, 0, 4:7], [-dx, 0, -dz], atol=1e-15)


def test_corridor_zigzag():
    w = 10.0
    tris = corridor(width=w)
    rays = np.array([[5, 0, 0, 1e-4, 1, 0.5, 0, 1e3]], dtype=np.float32)
    nb = 6
    c = oracle.bounces(tris, rays, nb)
    assert c.n_hits[0] == nb
    # horizontal run w/2 then w per hit, |d| / |dx| = sqrt(1.25)
    expect = (w / 2 + (nb - 1) * w) * np.sqrt(1.25)
    assert abs(c.path_len[0] - expect) < 1e-12 * expect
    ys = c.seg[1:, 0, 1]
    np.testing.assert_allclose(ys, [2.5 + 5 * k for k in range(nb - 1)], atol=1e-12)
    walls = c.id[:, 0] // 2
    assert list(walls) == [1, 0, 1, 0, 1, 0]


def test_miss_stops_chain():
    tris = corridor()
    rays = np.array([[5, 0, 0, 1e-4, 0, 1, 0, 1e3]], dtype=np.float32)   # parallel to both walls
    c = oracle.bounces(tris, rays, 3)
    assert c.n_hits[0] == 0 and c.path_len[0] == 0.0 and np.all(c.id[:, 0] == -1)
    assert np.all(np.isnan(c.seg[1:, 0]))


def test_tmax_per_segment():
    tris = corridor(width=10.0)
    # tmax bounds the ray parameter t of every segment: the first needs t = 5,
    # every later one t = 10, so tmax = 9 ends the chain after one hit
    rays = np.array([[5, 0, 0, 1e-4, 1, 0.5, 0, 9.0]], dtype=np.float32)
    c = oracle.bounces(tris, rays, 4)
    assert c.n_hits[0] == 1
