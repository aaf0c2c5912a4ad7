"""Comparison of GPU results with the CPU checker (oracle) on the same inputs.

Rule (closest hit): a ray is clean when the checker's margin exceeds 1e-4;
clean rays must give the checker's facet id exactly and t within relative
1e-5.  Every ray, clean or not, must give an answer in the acceptable set:
the checker's winner, a facet crossed within 1e-4 of its edges no later than
the winner's t (relative 1e-4), or a miss when the winner itself lies within
1e-4 of an edge or of either end of the range.
"""
import numpy as np

import oracle

CLEAN = 1e-4
T_REL = 1e-5


def _rel(a, s):
    return a / np.maximum(np.abs(s), 1e-3)


def compare_hits(tris, rays, gid, gt, ref: "oracle.Hits", skip=None):
    """Returns a dict of counts; raises AssertionError on a violation."""
    gid = np.asarray(gid, np.int32)
    gt = np.asarray(gt, np.float64)
    clean = ref.margin > CLEAN
    m = rays.shape[0]
    bad_id = clean & (gid != ref.id)
    hit = clean & (ref.id >= 0)
    with np.errstate(invalid="ignore"):
        bad_t = hit & ~(np.abs(gt - ref.t) <= T_REL * ref.t)
    miss_ok = clean & (ref.id < 0) & (gt == np.inf)
    assert not bad_id.any(), f"{bad_id.sum()} clean rays with the wrong facet, e.g. ray {np.nonzero(bad_id)[0][:5]}"
    assert not bad_t.any(), f"{bad_t.sum()} clean rays with t off by > 1e-5, e.g. {np.nonzero(bad_t)[0][:5]}"
    assert np.all(miss_ok == (clean & (ref.id < 0))), "clean misses must report t = +inf"
    # acceptable set for the rest
    low = np.nonzero(~clean & (gid != ref.id))[0]
    if low.size:
        r = rays[low]
        tmin, tmax = r[:, 3].astype(np.float64), r[:, 7].astype(np.float64)
        g = gid[low]
        w = ref.id[low]
        ok = np.zeros(low.size, bool)
        has_g = g >= 0
        if has_g.any():
            valid, tg, ug, vg = oracle.evaluate(tris, r, np.where(has_g, g, -1))
            out = np.maximum(np.maximum(-ug, -vg), ug + vg - 1)
            limit = np.where(w >= 0, ref.t[low] + CLEAN * np.maximum(ref.t[low], 1e-3),
                             tmax + CLEAN * np.maximum(tmax, 1e-3))
            lo = tmin - CLEAN * np.maximum(np.abs(tmin), 1e-3)
            ok |= has_g & valid.astype(bool) & (out <= CLEAN) & (tg >= lo) & (tg <= limit)
            if skip is not None:
                ok &= ~(has_g & (g == np.asarray(skip)[low]))
        no_g = (g < 0) & (w >= 0)
        if no_g.any():
            u, v, t1 = ref.u[low], ref.v[low], ref.t[low]
            edge = np.minimum(np.minimum(u, v), 1 - u - v) <= CLEAN
            rng = np.minimum(_rel(t1 - tmin, t1), _rel(tmax - t1, t1)) <= CLEAN
            ok |= no_g & (edge | rng)
        assert ok.all(), f"{(~ok).sum()} low-margin rays outside the acceptable set, e.g. {low[~ok][:5]}"
    return {"rays": int(m), "clean": int(clean.sum()), "low_margin": int((~clean).sum()),
            "low_margin_differing": int(low.size), "hits": int((gid >= 0).sum())}


def canonical_compare(gpu_nodes, gpu_perm, tree: "oracle.Tree"):
    """GPU tree (breadth-first records, right = left + 1) equals the checker's
    tree (depth-first arrays): same boxes, ranges, depths, splits, flags, costs
    and the same leaf order."""
    assert np.array_equal(gpu_perm, tree.perm), "leaf orders differ"
    assert gpu_nodes.shape[0] == tree.n_nodes, "node counts differ"
    stack = [(0, 0)]
    while stack:
        g, o = stack.pop()
        gn = gpu_nodes[g]
        assert np.array_equal(gn["lo"].astype(np.float64), tree.lo[o]), f"lo at {o}"
        assert np.array_equal(gn["hi"].astype(np.float64), tree.hi[o]), f"hi at {o}"
        for f in ("first", "count", "depth", "axis", "plane", "flags"):
            assert gn[f] == getattr(tree, f)[o], f"{f} at oracle node {o}: {gn[f]} vs {getattr(tree, f)[o]}"
        assert gn["cost"] == tree.cost[o], f"cost at {o}: {gn['cost']!r} vs {tree.cost[o]!r}"
        if tree.left[o] < 0:
            assert gn["left"] < 0
        else:
            assert gn["left"] >= 0
            stack.append((gn["left"], tree.left[o]))
            stack.append((gn["left"] + 1, tree.right[o]))
