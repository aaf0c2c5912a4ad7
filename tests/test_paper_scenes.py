"""The paper-size stand-in scenes (Sec. IV-A): exact facet counts, extents,
the paper's Tx and Rx in free space with a direct path between them, and
checker trees at the paper's leaf sizes."""
import numpy as np
import pytest

import oracle
from rtgen import workloads

from _scenes import check_tree


@pytest.fixture(scope="module", params=["indoor", "outdoor"])
def scene(request):
    return workloads.paper_indoor() if request.param == "indoor" else workloads.paper_outdoor()


def test_counts_and_extent(scene):
    v = scene.tris.reshape(-1, 3).astype(np.float64)
    if scene.name.startswith("indoor"):
        assert scene.tris.shape == (2778, 9)
        assert np.allclose(v.min(0), 0) and np.allclose(v.max(0), [8, 6, 3.5])
    else:
        assert scene.tris.shape == (7608, 9)
        assert np.allclose(v.min(0)[:2], 0) and np.allclose(v.max(0)[:2], 1000)
    t = scene.tris.astype(np.float64).reshape(-1, 3, 3)
    area = np.linalg.norm(np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]), axis=1)
    assert area.min() > 0
    assert np.array_equal(scene.tris, (workloads.paper_indoor() if scene.name.startswith("indoor")
                                       else workloads.paper_outdoor()).tris)   # seeded


def test_direct_path_and_free_endpoints(scene):
    tx, rx = np.array(scene.tx), np.array(scene.rx)
    d = rx - tx
    ray = np.array([[*tx, 0.0, *d, 1.0]], np.float32)
    h = oracle.brute(scene.tris, ray)
    assert h.id[0] < 0, "the direct Tx-Rx path is blocked"
    # both points lie strictly inside the scene's extent
    v = scene.tris.reshape(-1, 3)
    for p in (tx, rx):
        assert np.all(p > v.min(0)) and np.all(p[:2] < v.max(0)[:2])


def test_checker_trees_at_paper_leaf_sizes(scene):
    for alpha in (1.0, scene.alpha):
        tree = oracle.build_tree(scene.tris, oracle.SplitParams(alpha=alpha, src=scene.tx,
                                                                max_leaf=scene.max_leaf))
        check_tree(scene.tris, tree.lo, tree.hi, tree.left, tree.right, tree.first, tree.count,
                   tree.depth, tree.perm, scene.max_leaf, 64)
        assert tree.count[tree.left < 0].max() <= scene.max_leaf
