"""Pins of the CPU checker's edge diffraction (Sec. III-B: rays meeting
facets give diffracted rays) against geometry fixed independently of it:
edge counts of closed solids, the coplanarity threshold, the Keller cone law
(every diffracted direction makes the incident angle with the edge), the
exterior angle of a right-angled wedge, the diffraction point and the path
length to it."""
import math

import numpy as np
import pytest

from oracle import diffraction as df
from rtgen.scenes import _box, _pack, _quad


def box(x0=0.0, y0=0.0, z0=0.0, x1=10.0, y1=10.0, z1=10.0):
    return _pack(_box(x0, y0, z0, x1, y1, z1))


def test_wedges_of_closed_solids():
    nbr = df.wedges(box())
    # 12 box edges (90 degrees) are wedges, the 6 face diagonals are coplanar
    assert (nbr >= 0).sum() == 24 and (nbr == -2).sum() == 12 and (nbr == -1).sum() == 0
    for f in range(12):
        for k in range(3):
            g = nbr[f, k]
            if g >= 0:
                assert f in nbr[g]                           # symmetric
    tet = _pack([((0, 0, 0), (1, 0, 0), (0, 1, 0)), ((0, 0, 0), (0, 1, 0), (0, 0, 1)),
                 ((0, 0, 0), (0, 0, 1), (1, 0, 0)), ((1, 0, 0), (0, 0, 1), (0, 1, 0))])
    assert (df.wedges(tet) >= 0).sum() == 12
    quad = _pack(_quad((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)))
    nq = df.wedges(quad)
    assert (nq == -1).sum() == 4 and (nq == -2).sum() == 2


@pytest.mark.parametrize("deg,wedge", [(0.5, False), (0.9, False), (1.5, True), (30.0, True)])
def test_coplanarity_threshold(deg, wedge):
    a = math.radians(deg)
    # the second facet folds about the diagonal (1,0,0)-(0,1,0); its free vertex
    # lies sqrt(2)/2 from the fold line, so a height tan(deg) sqrt(2)/2 tilts it by deg
    tris = _pack([((0, 0, 0), (1, 0, 0), (0, 1, 0)),
                  ((1, 0, 0), (0, 1, 0), (1, 1, math.tan(a) * math.sqrt(2) / 2))])
    n1 = np.array([0.0, 0.0, 1.0])
    v = tris[1].reshape(3, 3).astype(np.float64)
    n2 = np.cross(v[1] - v[0], v[2] - v[0])
    ang = math.degrees(math.acos(abs(n2 @ n1) / np.linalg.norm(n2)))
    nbr = df.wedges(tris)
    assert ((nbr[0] >= 0).any()) == (ang > 1.0) == wedge, ang


def hit_on_face_x0(y, z, d=(1.0, 0.0, 0.0), delta=0.1, n_cone=36, L=0.0):
    tris = box()
    nbr = df.wedges(tris)
    # find the facet of the face x = 0 that contains (0, y, z)
    t3 = tris.reshape(-1, 3, 3).astype(np.float64)
    for f in range(12):
        if np.all(t3[f, :, 0] == 0):
            v = t3[f]
            m = np.array([[v[1, 1] - v[0, 1], v[2, 1] - v[0, 1]], [v[1, 2] - v[0, 2], v[2, 2] - v[0, 2]]])
            uv = np.linalg.solve(m, [y - v[0, 1], z - v[0, 2]])
            if uv.min() >= 0 and uv.sum() <= 1:
                break
    d = np.asarray(d, np.float64)
    o = np.array([0.0, y, z]) - 5.0 * d
    return tris, nbr, f, o, d, df.diffract_one(tris.reshape(-1, 3, 3), nbr, f, o, d, 5.0, L, 1e-4,
                                               1e3, delta, df.cone_table(n_cone))


def test_perpendicular_incidence_on_a_right_wedge():
    # hit 0.05 from the vertical edge x = y = 0; tube radius 5 * 0.1 / sqrt(3) = 0.289
    _, _, _, o, d, rays = hit_on_face_x0(0.05, 5.0)
    # 36 directions at 5, 15, ..., 355 degrees from the incident direction
    # around the edge; the 9 inside the box's right angle are dropped
    assert len(rays) == 27
    for k, j, path, q, dk in rays:
        assert np.array_equal(q, np.float32([0, 0, 5]))
        assert abs(dk[2]) < 1e-7                # beta = 90 deg: the cone is the plane z = 5
        assert abs(np.linalg.norm(dk.astype(np.float64)) - 1) < 1e-6
        assert not (dk[0] > 1e-6 and dk[1] > 1e-6)   # never into the box (x > 0, y > 0)
        assert abs(path - np.linalg.norm(np.array([0, 0, 5.0]) - o)) < 1e-12
    assert len({j for _, j, _, _, _ in rays}) == 27


def test_keller_cone_law_oblique():
    d = np.array([1.0, 0.2, -0.6])
    _, _, _, o, d, rays = hit_on_face_x0(0.03, 6.0, d=d)
    ihat = d / np.linalg.norm(d)
    assert rays
    for k, j, path, q, dk in rays:
        e = np.array([0.0, 0.0, 1.0])
        cb = ihat @ e
        # the same signed angle with the edge as the incident ray: the cone opens forward
        assert abs(dk.astype(np.float64) @ e - cb) < 1e-6
        assert q[0] == 0 and q[1] == 0 and abs(q[2] - 6.0) < 1e-5


def test_tube_radius_has_the_sqrt3():
    # hit 0.05 from the edge after l = 5: rho = 5 delta / sqrt(3) reaches it
    # for delta > 0.01732, while 5 delta alone would reach it from delta > 0.01
    _, _, _, _, _, rays = hit_on_face_x0(0.05, 5.0, delta=0.015)
    assert rays == []
    _, _, _, _, _, rays = hit_on_face_x0(0.05, 5.0, delta=0.0175)
    assert rays


def test_no_diffraction_outside_the_tube_and_free_edges_keep_all():
    _, _, _, _, _, rays = hit_on_face_x0(3.0, 5.0, delta=0.1)     # 3 m from every edge, rho 0.29
    assert rays == []
    _, _, _, _, _, rays = hit_on_face_x0(3.0, 5.0, delta=1.1)     # rho 3.18 > 3
    assert rays
    # a free panel: every cone direction is kept
    panel = _pack(_quad((0, 0, 0), (0, 10, 0), (0, 10, 10), (0, 0, 10)))
    nbr = df.wedges(panel)
    t3 = panel.reshape(-1, 3, 3)
    f = next(f for f in range(2) if nbr[f].max() == -1 and (t3[f, :, 1] == 0).sum() == 2)
    out = df.diffract_one(t3, nbr, f, np.array([-5.0, 0.05, 5.0]), np.array([1.0, 0, 0]), 5.0, 0.0,
                          1e-4, 1e3, 0.1, df.cone_table(12))
    assert len(out) == 12


def test_path_prefix_and_stored_chains():
    tris = box()
    nbr = df.wedges(tris)
    # two-segment stored chain: the second segment hits the face x = 0 near the edge
    seg = np.full((2, 1, 8), np.nan)
    seg[0, 0] = [-20, 0.05, 5, 0, 0, 0, 1, 1000]     # goes up, misses... but marked as a hit below
    seg[1, 0] = [-5, 0.05, 5, 0, 1, 0, 0, 1000]
    t3 = tris.reshape(-1, 3, 3).astype(np.float64)
    f = next(f for f in range(12) if np.all(t3[f, :, 0] == 0) and
             df.diffract_one(tris.reshape(-1, 3, 3), nbr, f, seg[1, 0, :3], seg[1, 0, 4:7], 5.0, 0.0,
                             1e-4, 1e3, 0.1, df.cone_table(8)))
    hid = np.array([[7], [f]], np.int32)
    ht = np.array([[2.5], [5.0]], np.float32)
    out = df.diffract(tris, nbr, seg, hid, ht, 0.1, df.cone_table(8))
    assert out.size > 0 and np.all(out["order"] == 1) and np.all(out["ray"] == 0)
    # L_1 = 2.5 * |(0, 0, 1)| = 2.5; path = 2.5 + |q - o| = 2.5 + sqrt(5^2 + 0.05^2)
    assert np.allclose(out["path"], 2.5 + math.hypot(5, 0.05), rtol=1e-14)


def test_distance_is_to_the_edge_segment_not_its_line():
    # triangle A B C with an obtuse angle at A; its edges AC and BC have
    # coplanar neighbours (they do not diffract), AB is free.  The hit
    # (-4, 0.6, 0) is 0.6 from AB's line but its foot (-4, 0, 0) lies outside
    # AB, so its distance to the edge is |p - A| = 4.04 > rho = 1
    A, B, C = (0, 0, 0), (10, 0, 0), (-8, 1, 0)
    tris = _pack([(A, B, C), (A, C, (-10, 0, 0)), (B, C, (0, 5, 0))])
    nbr = df.wedges(tris)
    assert nbr[0].tolist() == [-1, -2, -2]
    l = 5.0
    delta = 1.0 * math.sqrt(3) / l
    out = df.diffract_one(tris.reshape(-1, 3, 3), nbr, 0, np.array([-4.0, 0.6, 5.0]),
                          np.array([0.0, 0.0, -1.0]), l, 0.0, 1e-4, 1e3, delta, df.cone_table(8))
    assert out == []
    out = df.diffract_one(tris.reshape(-1, 3, 3), nbr, 0, np.array([0.5, 0.6, 5.0]),
                          np.array([0.0, 0.0, -1.0]), l, 0.0, 1e-4, 1e3, delta, df.cone_table(8))
    assert out and all(k == 0 for k, *_ in out)    # 0.6 from AB inside the segment: diffracts
