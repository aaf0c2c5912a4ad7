"""Comparison of GPU results with the CPU checker (oracle) on the same inputs.

Rule (closest hit): a ray is clean when the checker's margin exceeds 1e-4;
clean rays must give the checker's facet id exactly and t within relative
1e-5.  Every ray, clean or not, must give an answer in the acceptable set:
the checker's winner, a facet crossed within 1e-4 of its edges no later than
the winner's t (relative 1e-4), a miss when the winner itself lies within
1e-4 of an edge or of either end of the range, or -- when the winner lies
within 1e-4 of an edge, so that the ray may pass it -- the answer with the
winner removed (the same rule again, up to four facets deep: a ray tangent
to a thin slab passes both of its faces).
"""
import numpy as np

import oracle
from oracle import reception as rc

CLEAN = 1e-4
T_REL = 1e-5
BAND = 5e-3   # reception: relative distance from the Eq. (4) threshold treated as borderline


def _rel(a, s):
    with np.errstate(invalid="ignore"):  # inf - inf (two misses) gives nan, which compares false
        return a / np.maximum(np.abs(s), 1e-3)


def _edge_near(u, v):
    return min(u, v, 1 - u - v) <= CLEAN


def _passes_grazed(tris, ray, gid, winner, u, v, depth=4):
    """True when the GPU answer gid for one ray is acceptable after removing
    the checker's winners that the ray meets within CLEAN of an edge."""
    if winner < 0 or not _edge_near(u, v):
        return False
    cut = np.array(tris, np.float32, copy=True).reshape(-1, 9)
    removed = [winner]
    for _ in range(depth):
        cut[removed] = 0.0                     # zero-area facets are never hit
        nxt = oracle.brute(cut, ray[None])
        nid = int(nxt.id[0])
        if gid == nid:
            return True
        if gid >= 0:
            valid, tg, ug, vg = oracle.evaluate(tris, ray[None], np.array([gid], np.int32))
            out = max(-ug[0], -vg[0], ug[0] + vg[0] - 1)
            lim = nxt.t[0] * (1 + CLEAN) if nid >= 0 else np.inf
            if valid[0] and out <= CLEAN and tg[0] <= lim:
                return True
        if nid < 0 or not _edge_near(nxt.u[0], nxt.v[0]):
            return False
        removed.append(nid)
    return False


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
        if not ok.all() and skip is None:
            # a ray through an edge of the winner may pass it (a ray tangent to
            # a thin slab passes both of its faces): then the answer is the
            # one with that facet removed, the same rule applied again, up to
            # four facets deep
            for q in np.nonzero(~ok)[0]:
                ok[q] = _passes_grazed(tris, r[q], g[q], w[q], ref.u[low][q], ref.v[low][q])
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


def keyed(rec):
    rec = np.sort(rec, order=("rx", "ray", "order"))
    return rec, [tuple(int(x) for x in r) for r in zip(rec["rx"], rec["ray"], rec["order"])]


def oracle_quantities(ch, L, rx, keys, delta):
    """q = sqrt(3) dist / (l delta) and the foot's distance from the nearer end
    (fraction of the segment) for (rx, ray, order) keys on the checker's chains."""
    out = []
    for r, i, b in keys:
        s_row = ch.seg[b, i]
        o, d = s_row[0:3], s_row[4:7]
        t0 = s_row[3]
        t1 = ch.t[b, i] if ch.id[b, i] >= 0 else s_row[7]
        w = rx[r] - o
        s = (w @ d) / (d @ d)
        dist = np.linalg.norm(w - s * d)
        l = L[b, i] + np.linalg.norm(w)
        q = np.sqrt(3) * dist / (l * delta) if l * delta > 0 else np.inf
        edge = min(abs(s - t0), abs(s - t1)) / max(t1 - t0, 1e-9)
        out.append((q, edge))
    return out


def agree_with_checker(tris, rays, rx, delta, nb, params, got, ids_g, t_g, nthreads=16):
    """Receptions (Sec. III-C) on the checker's float64 chains against the
    GPU's.  On rays whose chains agree with the checker's (same facets, hit
    distances within 1e-5, margins above 1e-4) the receptions must agree,
    except where the checker's own test lies within BAND of its threshold
    (sqrt(3) dist / (l delta) = 1) or of a segment end; l and dist within
    2e-5 of l.  got: GPU records, ids_g / t_g: GPU hits [nb, m]."""
    tree = oracle.build_tree(tris, params)
    ch = oracle.bounces(tris, rays, nb, tree=tree, nthreads=nthreads)
    ref = rc.receive(ch.seg, ch.id, ch.t, rx, delta)
    L = rc.path_prefix(ch.seg, ch.id, ch.t)
    # rays whose chains agree up to segment b
    agree = np.zeros((nb, rays.shape[0]), bool)
    ok = np.ones(rays.shape[0], bool)
    for b in range(nb):
        same = (ids_g[b] == ch.id[b]) & (ch.margin[b] > 1e-4)
        hit = ch.id[b] >= 0
        with np.errstate(invalid="ignore"):
            tclose = ~hit | (np.abs(t_g[b] - ch.t[b]) <= 1e-5 * np.maximum(ch.t[b], 1e-3))
        ok = ok & same & tclose
        agree[b] = ok
        ok = ok & hit
    g, gk = keyed(got)
    r, rk = keyed(ref)
    gset, rset = set(gk), set(rk)
    only = [k for k in (gset ^ rset) if agree[k[2], k[1]]]
    bad = [(k, q, e) for k, (q, e) in zip(only, oracle_quantities(ch, L, rx, only, delta))
           if abs(q - 1) > BAND and e > BAND]
    assert not bad, f"{len(bad)} receptions differ away from the boundary, e.g. {bad[:3]}"
    both = sorted(k for k in gset & rset if agree[k[2], k[1]])
    gi = {k: n for n, k in enumerate(gk)}
    ri = {k: n for n, k in enumerate(rk)}
    lg = np.array([g["l"][gi[k]] for k in both])
    lr = np.array([r["l"][ri[k]] for k in both])
    dg = np.array([g["dist"][gi[k]] for k in both])
    dr = np.array([r["dist"][ri[k]] for k in both])
    assert np.all(np.abs(lg - lr) <= 2e-5 * lr), "path lengths"
    assert np.all(np.abs(dg - dr) <= 2e-5 * lr), "distances"
    return {"gpu": len(gk), "checker": len(rk), "compared": len(both), "borderline": len(only)}


U32 = 2.0 ** -24   # float32 unit roundoff


def chain_error_bounds(tris, seg, ids, t):
    """First-order bound on |t_gpu - t_64| for every segment of the checker's
    float64 chains (Sec. III-B re-launch), from how the GPU's float32 chain
    departs from them.  Both start from the same float32 rays.  At segment b
    let the GPU's origin and direction differ from the checker's by at most
    E_o and E_d (vector norms).  The exact hit of the GPU's ray on the same
    facet plane (unit normal n, incidence cos c = |n.d| / |d|) then moves by
    |dt| <= (E_o + t E_d) / (|d| c), and the hit point, which stays in the
    plane, by (E_o + t E_d)(1 + 1 / c).  The GPU's own arithmetic adds, per
    segment: its t for its float32 ray (compensated, one float32 rounding:
    2u t |d| at the hit point), the origin rounding of fma(t, d, o) (u per
    coordinate, sqrt(3) u max|p|), and the reflection (compensated, rounded
    once per component: at most 2u each, 2 sqrt(3) u max|r|).  Reflection is
    an isometry, so E_d only accumulates those roundings.  The allowed
    deviation is that propagated term plus the 1e-5 relative tolerance of
    the segment itself.  Returns allowed [max_b, m] (inf where the checker's
    segment missed or was never traced)."""
    v = tris.astype(np.float64).reshape(-1, 3, 3)
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-300)
    nb, m = ids.shape
    allowed = np.full((nb, m), np.inf)
    e_o = np.zeros(m)
    e_d = np.zeros(m)
    for b in range(nb):
        hit = ids[b] >= 0
        o, d = seg[b, :, 0:3], seg[b, :, 4:7]
        dn = np.linalg.norm(d, axis=1)
        tb = np.where(hit, t[b], 0.0)
        n = nrm[np.where(hit, ids[b], 0)]
        with np.errstate(divide="ignore", invalid="ignore"):
            cos = np.abs(np.einsum("ij,ij->i", n, d)) / dn
            w = e_o + tb * e_d
            allowed[b] = np.where(hit, 1e-5 * tb + w / (dn * cos), np.inf)
            p = o + tb[:, None] * d
            e_o = w * (1.0 + 1.0 / cos) + 2 * U32 * tb * dn + np.sqrt(3) * U32 * np.abs(p).max(1)
        if b + 1 < nb:
            r = seg[b + 1, :, 4:7]
            e_d = e_d + 2 * np.sqrt(3) * U32 * np.nan_to_num(np.abs(r).max(1))
    return allowed


def check_differing(city, tree, bvh, rays, nb, base, got, differ, tag):
    """Chains of a launch (lanes refilled, or live chains regrouped) that
    differ from the default launch: before
    the first differing segment both launches traced the same segment rays
    (same facets, same float32 arithmetic), so that segment's input is known
    from either launch; its checker margin must be at most 1e-4 and the
    other launch's answer must pass the closest-hit rule.  base and got are
    (hits, path lengths, hit counts) as numpy arrays; rays is on the device."""
    assert differ.size <= 1e-4 * rays.shape[0], f"{tag}: {differ.size} chains differ"
    import torch
    seg = torch.empty((nb, rays.shape[0], 8), dtype=torch.float32, device="cuda")
    bvh.trace_bounces(rays, nb, seg_rays=seg)
    torch.cuda.synchronize()
    seg_np = seg.cpu().numpy()
    first = np.argmax(np.any(got[0][:, differ] != base[0][:, differ], axis=2), axis=0)
    for j, b in zip(differ.tolist(), first.tolist()):
        ray = seg_np[b, j][None]
        skip = np.array([base[0][b - 1, j, 0] if b > 0 else -1], np.int32)
        ref = oracle.trace_bvh(tree, ray, skip=skip, nthreads=1)
        assert ref.margin[0] <= CLEAN, (tag, j, b, float(ref.margin[0]))
        t = got[0][b, j, 1:2].view(np.float32).astype(np.float64)
        compare_hits(city.tris, ray, got[0][b, j, 0:1], t, ref, skip=skip)
