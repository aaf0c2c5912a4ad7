"""Pins of the CPU checker's closest hit (Sec. III-B: nearest facet hit)."""
import numpy as np
import pytest

import oracle
from oracle import npref
from rtgen import workloads

from _scenes import box_scene, ground_and_wall


def test_box_worked_cases():
    tris, cases = box_scene()
    rays = np.array([c["ray"] for c in cases], dtype=np.float32)
    h = oracle.brute(tris, rays)
    for k, c in enumerate(cases):
        assert h.id[k] == c["id"], c["name"]
        if c["id"] < 0:
            assert h.t[k] == np.inf
        else:
            assert h.t[k] == c["t"], c["name"]
            if c.get("edge"):
                assert h.margin[k] == 0.0
            else:
                assert h.margin[k] > 1e-4, c["name"]


def test_box_numpy_solver_agrees():
    tris, cases = box_scene()
    rays = np.array([c["ray"] for c in cases], dtype=np.float32)
    ids, ts = npref.brute_solve(tris, rays)
    assert [int(i) for i in ids] == [c["id"] for c in cases]


def test_barycentrics_of_worked_case():
    # point (0,3,6) on facet (0,0,0),(0,10,10),(0,0,10): p = (1-u-v) a + u b + v c
    # gives u = 0.3 (weight of b), v = 0.3 (weight of c)
    tris, cases = box_scene()
    h = oracle.brute(tris, np.array([cases[0]["ray"]], dtype=np.float32))
    assert abs(h.u[0] - 0.3) < 1e-15 and abs(h.v[0] - 0.3) < 1e-15
    assert abs(h.margin[0] - oracle.MARGIN_CAP) < 1e-18     # far from every edge


def test_ground_closed_form():
    # from height h downwards at 45 degrees: t = h / |dz| (|d| = 1 up to rounding)
    tris = ground_and_wall(wall_x=1e4)
    for h in (1.0, 10.0, 37.5):
        d = np.float32([1, 0, -1]) / np.float32(np.sqrt(2))
        d = d.astype(np.float32)
        ray = np.array([[3, 4, h, 1e-4, d[0], d[1], d[2], 1e3]], dtype=np.float32)
        r = oracle.brute(tris, ray)
        assert r.id[0] in (0, 1)
        assert abs(r.t[0] - h / abs(float(d[2]))) <= 1e-14 * r.t[0]
        assert abs(r.t[0] - h * np.sqrt(2)) < 1e-6 * h


def test_skip_id():
    tris, cases = box_scene()
    ray = np.array([cases[0]["ray"]], dtype=np.float32)
    r = oracle.brute(tris, ray, skip=np.array([1], np.int32))
    assert r.id[0] == 2 and r.t[0] == 15.0        # x0 facet skipped: far face


def test_tie_goes_to_lower_id():
    # two coincident copies of one facet: equal t, lower id wins, zero gap margin
    tris = np.array([[0, 0, 0, 0, 10, 0, 0, 0, 10]] * 2, dtype=np.float32)
    ray = np.array([[-1, 2, 3, 1e-4, 1, 0, 0, 10]], dtype=np.float32)
    r = oracle.brute(tris, ray)
    assert r.id[0] == 0 and r.t[0] == 1.0 and r.margin[0] == 0.0 and r.t2[0] == 1.0


def test_degenerate_facet_never_hit():
    tris = np.array([[0, 0, 0, 0, 5, 5, 0, 10, 10],       # zero area (collinear)
                     [5, -10, -10, 5, 10, -10, 5, 0, 10]], dtype=np.float32)
    # the ray crosses the collinear facet's segment at t = 1, then the real one
    ray = np.array([[-1, 2, 2, 1e-4, 1, 0, 0, 100]], dtype=np.float32)
    r = oracle.brute(tris, ray)
    assert r.id[0] == 1 and r.t[0] == 6.0


def test_near_miss_margin():
    # the ray passes 0.5 % of an edge outside a facet in front of the real hit
    tris = np.array([[0, 0, 0, 0, 10, 0, 0, 0, 10],        # near facet, x = 0
                     [5, -50, -50, 5, 50, -50, 5, 0, 50]], dtype=np.float32)
    ray = np.array([[-1, 5.025, 5.0, 1e-4, 1, 0, 0, 100]], dtype=np.float32)
    r = oracle.brute(tris, ray)
    assert r.id[0] == 1
    # outside by u + v - 1 = (5.025 + 5.0) / 10 - 1 = 0.0025 (float32 input)
    y = float(np.float32(5.025))
    assert abs(r.margin[0] - min(oracle.MARGIN_CAP, (y + 5.0) / 10 - 1)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_numpy_solver_agrees_on_microcell(seed):
    w = workloads.microcell(seed)
    idx = np.random.default_rng(seed).choice(w.n_rays, 600, replace=False)
    rays = w.rays[idx]
    h = oracle.brute(w.tris, rays)
    ids, ts = npref.brute_solve(w.tris, rays)
    clean = h.margin > 1e-6
    assert clean.mean() > 0.95
    assert np.array_equal(ids[clean], h.id[clean])
    hit = clean & (h.id >= 0)
    assert np.allclose(ts[hit], h.t[hit], rtol=1e-11, atol=0)


def test_bvh_traversal_equals_brute_force_microcell():
    w = workloads.microcell()
    for alpha in (1.0, 0.7, 0.0):
        tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=alpha, src=w.tx))
        a = oracle.brute(w.tris, w.rays)
        b = oracle.trace_bvh(tree, w.rays)
        assert np.array_equal(a.id, b.id)
        assert np.array_equal(a.t, b.t)
        assert np.array_equal(a.margin, b.margin)
        assert np.array_equal(a.t2, b.t2)


def test_bvh_traversal_equals_brute_force_city_sample():
    w = workloads.city24k(level=7)
    idx = np.random.default_rng(3).choice(w.n_rays, 1500, replace=False)
    rays = w.rays[idx]
    tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.4, src=w.tx))
    a = oracle.brute(w.tris, rays)
    b = oracle.trace_bvh(tree, rays, stats=True)
    assert np.array_equal(a.id, b.id) and np.array_equal(a.t, b.t)
    assert np.array_equal(a.margin, b.margin)
    # the tree really prunes: far fewer facet tests than brute force
    assert b.tris_tested.mean() < 0.01 * w.n_tris
