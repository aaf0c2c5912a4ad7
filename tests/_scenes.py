"""Small hand-made scenes with closed-form answers, shared by the tests."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def box_scene():
    """The 12-facet box of closest_hit_box.json, facets in the fixture's order."""
    g = load_golden("closest_hit_box.json")
    tris = []
    for face in g["face_order"]:
        p0, p1, p2, p3 = g["faces"][face]
        tris.append(p0 + p1 + p2)
        tris.append(p0 + p2 + p3)
    return np.array(tris, dtype=np.float32), g["cases"]


def quad(p0, p1, p2, p3):
    return [list(p0) + list(p1) + list(p2), list(p0) + list(p2) + list(p3)]


def ground_and_wall(half=100.0, wall_x=20.0, height=100.0):
    """Ground z = 0 over [-half, half]^2 and a wall in the plane x = wall_x."""
    t = quad((-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0))
    t += quad((wall_x, -half, 0), (wall_x, half, 0), (wall_x, half, height), (wall_x, -half, height))
    return np.array(t, dtype=np.float32)


def corridor(width=10.0, ext=1000.0):
    """Two parallel walls x = 0 and x = width, large in y and z."""
    t = quad((0, -ext, -ext), (0, ext, -ext), (0, ext, ext), (0, -ext, ext))
    t += quad((width, -ext, -ext), (width, -ext, ext), (width, ext, ext), (width, ext, -ext))
    return np.array(t, dtype=np.float32)


def split_case_tris():
    g = load_golden("split_cases.json")
    tris = [[x0, 0, 0, x0 + 1, 0, 0, x0, 1, 0] for x0 in g["x0"]]
    return np.array(tris, dtype=np.float32), g


def check_tree(tris, lo, hi, left, right, first, count, depth, perm, max_leaf, depth_limit,
               exact_boxes=True):
    """Tree invariants of a binary BVH in node-array form (any node order):
    the leaf ranges partition perm, perm is a bijection, every node box holds
    its facets' boxes (equals their union when exact_boxes), parents hold
    children, leaves hold 1..max_leaf facets, depth <= depth_limit."""
    n = tris.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n)), "perm is not a bijection"
    v = tris.reshape(-1, 3, 3).astype(np.float64)
    flo, fhi = v.min(1), v.max(1)
    # find the root: the node that is nobody's child
    nn = left.shape[0]
    is_child = np.zeros(nn, bool)
    internal = left >= 0
    is_child[left[internal]] = True
    is_child[right[internal]] = True
    roots = np.nonzero(~is_child)[0]
    assert roots.size == 1, "tree must have one root"
    root = roots[0]
    assert first[root] == 0 and count[root] == n and depth[root] == 0
    seen = np.zeros(n, np.int32)
    stack = [root]
    visited = 0
    while stack:
        i = stack.pop()
        visited += 1
        a, k = first[i], count[i]
        ids = perm[a:a + k]
        blo, bhi = flo[ids].min(0), fhi[ids].max(0)
        if exact_boxes:
            assert np.array_equal(lo[i], blo) and np.array_equal(hi[i], bhi), f"node {i} box != union"
        else:
            assert np.all(lo[i] <= blo) and np.all(hi[i] >= bhi), f"node {i} box misses a facet"
        assert depth[i] <= depth_limit
        if left[i] < 0:
            assert 1 <= k <= max_leaf, f"leaf {i} holds {k}"
            seen[a:a + k] += 1
        else:
            l, r = left[i], right[i]
            assert first[l] == a and first[r] == a + count[l] and count[l] + count[r] == k
            assert count[l] > 0 and count[r] > 0
            assert depth[l] == depth[i] + 1 and depth[r] == depth[i] + 1
            for c in (l, r):
                assert np.all(lo[c] >= lo[i]) and np.all(hi[c] <= hi[i]), "child outside parent"
            stack += [l, r]
    assert visited == nn, "unreachable nodes"
    assert np.all(seen == 1), "leaf ranges must partition the facets"
