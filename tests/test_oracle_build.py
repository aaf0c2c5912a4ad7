"""Pins of the CPU checker's tree build (Sec. II-B Eq. (2), Sec. II-C flow)."""
import numpy as np
import pytest

import oracle
from rtgen import workloads

from _scenes import check_tree, split_case_tris


def _check(tris, tree, p):
    check_tree(tris, tree.lo, tree.hi, tree.left, tree.right, tree.first, tree.count,
               tree.depth, tree.perm, p.max_leaf, p.depth_limit)


@pytest.mark.parametrize("case", range(10))
def test_hand_worked_split(case):
    tris, g = split_case_tris()
    c = g["cases"][case]
    p = oracle.SplitParams(alpha=c["alpha"], src=tuple(g["src"]), nbins=g["nbins"],
                           max_leaf=g["max_leaf"], d_norm=c["d_norm"])
    tree = oracle.build_tree(tris, p)
    assert tree.axis[0] == 0 and tree.plane[0] == c["plane"]
    l = tree.left[0]
    assert sorted(tree.perm[tree.first[l]: tree.first[l] + tree.count[l]].tolist()) == c["left"]
    if "cost" in c:
        assert abs(tree.cost[0] - c["cost"]) <= 1e-12 * abs(c["cost"])


def test_leaf_threshold_and_single_leaf():
    tris, g = split_case_tris()
    tree = oracle.build_tree(tris, oracle.SplitParams(max_leaf=4))
    assert tree.n_nodes == 1 and tree.count[0] == 4 and tree.left[0] == -1
    tree = oracle.build_tree(tris, oracle.SplitParams(max_leaf=3))
    assert tree.n_nodes == 3


def test_identical_centroids_split_by_position():
    tri = [0, 0, 0, 1, 0, 0, 0, 1, 0]
    tris = np.array([tri] * 5, dtype=np.float32)
    tree = oracle.build_tree(tris, oracle.SplitParams(max_leaf=1))
    assert tree.flags[0] & 2
    assert tree.count[tree.left[0]] == 2 and tree.count[tree.right[0]] == 3
    _check(tris, tree, oracle.SplitParams(max_leaf=1))


def test_depth_limit_forces_halving():
    # exponentially spaced facets make SAH peel one facet per level
    xs = [2.0 ** k for k in range(40)]
    tris = np.array([[x, 0, 0, x * 1.01, 0, 0, x, x * 0.01, 0] for x in xs], dtype=np.float32)
    p = oracle.SplitParams(max_leaf=1, depth_limit=8, nbins=4)
    tree = oracle.build_tree(tris, p)
    assert tree.depth.max() <= 8
    assert np.any(tree.flags & 1)
    _check(tris, tree, p)


@pytest.mark.parametrize("alpha,d_norm", [(1.0, "unit"), (0.4, "unit"), (0.7, "raw"), (0.0, "unit")])
def test_invariants_city(alpha, d_norm):
    w = workloads.city24k(level=0)
    p = oracle.SplitParams(alpha=alpha, src=w.tx, d_norm=d_norm)
    tree = oracle.build_tree(w.tris, p)
    _check(w.tris, tree, p)


def test_alpha_one_is_eq1_whatever_the_distance_settings():
    # alpha = 1 leaves only the surface-area terms of Eq. (2), i.e. Eq. (1):
    # the source point, the distance mode and the normalisation cannot matter
    w = workloads.microcell()
    ref = oracle.build_tree(w.tris, oracle.SplitParams(alpha=1.0, src=(0, 0, 0)))
    for kw in (dict(src=(500, -30, 2)), dict(d_norm="raw"), dict(d_mode="kweighted"),
               dict(d_mode="sum", src=(-9, 9, 99))):
        t = oracle.build_tree(w.tris, oracle.SplitParams(alpha=1.0, **kw))
        assert np.array_equal(t.perm, ref.perm) and np.array_equal(t.left, ref.left)
        assert np.array_equal(t.axis, ref.axis) and np.array_equal(t.plane, ref.plane)


def test_parent_distance_mode_reduces_to_eq1():
    # with d taken from the parent volume, d^2 is the same for every candidate,
    # so the argmin is that of Eq. (1) (the reading the default mode avoids)
    w = workloads.microcell()
    ref = oracle.build_tree(w.tris, oracle.SplitParams(alpha=1.0))
    t = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.3, d_mode="parent", src=w.tx))
    assert np.array_equal(t.perm, ref.perm) and np.array_equal(t.plane, ref.plane)


def test_distance_term_changes_the_tree():
    w = workloads.microcell()
    a = oracle.build_tree(w.tris, oracle.SplitParams(alpha=1.0, src=w.tx))
    b = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.0, src=w.tx))
    assert not np.array_equal(a.perm, b.perm)


def test_rejects_bad_params():
    tris, _ = split_case_tris()
    for kw in (dict(alpha=1.5), dict(alpha=-0.1), dict(max_leaf=0), dict(nbins=1)):
        with pytest.raises(ValueError):
            oracle.build_tree(tris, oracle.SplitParams(**kw))
