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


# ---------------------------------------------------------------- tree cost
def _strip(x0, x1):
    """A right triangle covering the box [x0, x1] x [0, 1] x {0}."""
    return [x0, 0, 0, x1, 0, 0, x0, 1, 0]


def test_tree_cost_hand_worked():
    # two unit squares' triangles at x in [0, 1] and [9, 10]: leaf boxes of
    # area 2 * 1 * 1 = 2, root box [0, 10] x [0, 1] of area 2 * 10 = 20
    two = np.array([_strip(0, 1), _strip(9, 10)], np.float32)
    t = oracle.build_tree(two, oracle.SplitParams(max_leaf=1))
    assert t.n_nodes == 3
    assert oracle.tree_cost(t) == pytest.approx(20 / 20 + 2 / 20 + 2 / 20, rel=1e-15)   # 1.2
    assert oracle.tree_cost(t, t_isect=2.0, t_trav=0.5) == pytest.approx(0.5 + 0.4, rel=1e-15)
    t = oracle.build_tree(two, oracle.SplitParams(max_leaf=2))      # root leaf of 2 facets
    assert t.n_nodes == 1 and oracle.tree_cost(t) == pytest.approx(2.0, rel=1e-15)
    # three: x in [0, 1], [2, 3], [9, 10].  Eq. (1) prefers {A, B} | {C}
    # ((6 * 2 + 2 * 1) / 20 against (2 * 1 + 16 * 2) / 20), then A | B:
    # internal areas 20 and 6, leaf areas 2, 2, 2
    three = np.array([_strip(0, 1), _strip(2, 3), _strip(9, 10)], np.float32)
    t = oracle.build_tree(three, oracle.SplitParams(max_leaf=1))
    assert t.n_nodes == 5 and sorted(t.count[t.left < 0].tolist()) == [1, 1, 1]
    assert oracle.tree_cost(t) == pytest.approx((20 + 6) / 20 + 6 / 20, rel=1e-15)      # 1.6
    assert oracle.tree_cost(t, t_isect=2.0, t_trav=0.5) == pytest.approx(0.65 + 0.6, rel=1e-15)


def _recursive_cost(tree, node, t_isect, t_trav):
    """Eq. (1) per node: a leaf costs k t_i; an internal node t_trav plus each
    child's cost weighted by the child's share of its surface area."""
    w = tree.hi[node] - tree.lo[node]
    s = 2.0 * (w[0] * w[1] + w[1] * w[2] + w[2] * w[0])
    if tree.left[node] < 0:
        return tree.count[node] * t_isect
    c = t_trav
    for ch in (tree.left[node], tree.right[node]):
        wc = tree.hi[ch] - tree.lo[ch]
        sc = 2.0 * (wc[0] * wc[1] + wc[1] * wc[2] + wc[2] * wc[0])
        c += sc / s * _recursive_cost(tree, ch, t_isect, t_trav)
    return c


@pytest.mark.parametrize("alpha,max_leaf", [(1.0, 4), (0.4, 1), (0.7, 8)])
def test_tree_cost_equals_recursive_form(alpha, max_leaf):
    # summed node by node with root-relative areas, or recursively with
    # parent-relative areas: the area ratios telescope to the same value
    w = workloads.microcell()
    t = oracle.build_tree(w.tris, oracle.SplitParams(alpha=alpha, src=w.tx, max_leaf=max_leaf))
    for ti, tt in ((1.0, 1.0), (3.0, 0.25)):
        assert oracle.tree_cost(t, ti, tt) == pytest.approx(_recursive_cost(t, 0, ti, tt),
                                                            rel=1e-12)
