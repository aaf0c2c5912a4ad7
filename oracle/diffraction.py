"""Edge diffraction of reflection chains (Sec. III-B: a ray meeting facets
gives reflected and diffracted rays) -- CPU checker, numpy float64, no FMA.

Test infrastructure only: the tests and the smoke check use this module; the
GPU library never does.

The paper names diffracted rays and a diffraction order (set to 0 in its
experiments) but not how they are made; the readings written out here are
the usual shooting-and-bouncing-rays construction:

Wedges (``wedges``).  The three edges of facet f are (v0, v1), (v1, v2),
(v2, v0), edge k starting at vertex k.  Two half-edges are the same edge when
their end points are the same float32 points in either order.  An edge of
exactly one facet is a free edge (neighbour -1).  An edge of exactly two
facets is a wedge when their normals n = (v1 - v0) x (v2 - v0) (float64)
satisfy (n_a . n_b)^2 < cos^2(1 degree) |n_a|^2 |n_b|^2, i.e. the facets are
not coplanar (neighbour = the other facet); otherwise, and for edges of more
than two facets, it does not diffract (neighbour -2).

Diffraction (``diffract``).  Segment b of ray i that hit facet f at
parameter t (origin o, direction d, both float32, path length L_b before
it) hits at p = o + t d, after a path l = L_b + t |d|.  Its ray tube has the
radius rho = l delta / sqrt(3) of Eq. (4).  For each diffracting edge
(a, b_) of f: e = b_ - a, s = clamp(((p - a) . e) / (e . e), 0, 1),
q = a + s e, dist = |p - q|; the nearest edge with dist <= rho (ties to the
lower edge index) diffracts.  On that edge, with unit edge direction
ê = e / |e| and unit incident direction î = d / |d|, c = î . ê,
r = î - c ê, sin(beta) = |r| (no diffraction when sin(beta) == 0),
u = r / |r|, w = ê x u, the Keller cone directions are
d_k = c ê + sin(beta) (cos_k u + sin_k w) for the caller's table of
(cos_k, sin_k).  For a wedge, a direction whose component across the edge
lies strictly inside the angle between the two facets (between a_in and
b_in, the in-plane unit vectors across the edge towards each facet's third
vertex) points into the solid and is dropped.  Each kept direction becomes a
ray from q (rounded to float32) along d_k (rounded to float32) with the
parent's tmin and tmax; its record carries the parent ray, segment, facet,
edge, cone index and the path length to q, L_b + |q - o|.
"""
from __future__ import annotations

import math

import numpy as np

COS2_COPLANAR = math.cos(math.radians(1.0)) ** 2

DIFFRACTED = np.dtype([("ray", np.int32), ("order", np.int32), ("facet", np.int32),
                       ("edge", np.int32), ("cone", np.int32), ("pad", np.int32),
                       ("path", np.float64), ("o", np.float32, 3), ("tmin", np.float32),
                       ("d", np.float32, 3), ("tmax", np.float32)])


def _normal(v):
    e1 = v[1] - v[0]
    e2 = v[2] - v[0]
    return np.array([e1[1] * e2[2] - e1[2] * e2[1],
                     e1[2] * e2[0] - e1[0] * e2[2],
                     e1[0] * e2[1] - e1[1] * e2[0]])


def wedges(tris) -> np.ndarray:
    """Neighbour of every half-edge, int32 [n, 3]: the other facet of a wedge
    edge, -1 for a free edge, -2 for an edge that does not diffract."""
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    n = tris.shape[0]
    groups = {}
    for f in range(n):
        for k in range(3):
            a = tuple(tris[f, k].tolist())
            b = tuple(tris[f, (k + 1) % 3].tolist())
            groups.setdefault((min(a, b), max(a, b)), []).append((f, k))
    nbr = np.full((n, 3), -2, np.int32)
    for members in groups.values():
        if len(members) == 1:
            f, k = members[0]
            nbr[f, k] = -1
        elif len(members) == 2:
            (fa, ka), (fb, kb) = members
            na = _normal(tris[fa].astype(np.float64))
            nb = _normal(tris[fb].astype(np.float64))
            dot = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2]
            aa = na[0] * na[0] + na[1] * na[1] + na[2] * na[2]
            bb = nb[0] * nb[0] + nb[1] * nb[1] + nb[2] * nb[2]
            if dot * dot < COS2_COPLANAR * aa * bb:
                nbr[fa, ka] = fb
                nbr[fb, kb] = fa
    return nbr


def cone_table(n_dirs: int) -> np.ndarray:
    """(cos, sin) of n_dirs angles 2 pi (k + 1/2) / n_dirs around the Keller
    cone: half a step off the forward direction (the shadow boundary, where
    edge diffraction is singular) and off directions along the facets."""
    a = 2 * np.pi * (np.arange(n_dirs) + 0.5) / n_dirs
    return np.stack([np.cos(a), np.sin(a)], 1)


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _across(ea, eb, third, ehat):
    """Unit vector in the facet's plane, perpendicular to the edge, towards
    the facet's third vertex."""
    x = third - ea
    x = x - _dot(x, ehat) * ehat
    return x / math.sqrt(_dot(x, x))


def diffract_one(tris, nbr, f, o, d, t, L, tmin, tmax, delta, cone):
    """The diffracted rays of one hit (list of tuples), following the module
    docstring step by step."""
    v = tris[f].astype(np.float64)
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    t = float(t)
    p = o + t * d
    dn = math.sqrt(_dot(d, d))
    l = L + t * dn
    rho = l * delta / math.sqrt(3.0)
    best, best_k = None, -1
    for k in range(3):
        if nbr[f, k] == -2:
            continue
        a, b = v[k], v[(k + 1) % 3]
        e = b - a
        s = _dot(p - a, e) / _dot(e, e)
        s = min(max(s, 0.0), 1.0)
        q = a + s * e
        dq = p - q
        dist = math.sqrt(_dot(dq, dq))
        if dist <= rho and (best is None or dist < best[0]):
            best, best_k = (dist, q, a, b, e), k
    if best is None:
        return []
    _, q, a, b, e = best
    k = best_k
    ehat = e / math.sqrt(_dot(e, e))
    ihat = d / dn
    c = _dot(ihat, ehat)
    r = ihat - c * ehat
    sb = math.sqrt(_dot(r, r))
    if sb == 0.0:
        return []
    u = r / sb
    w = _cross(ehat, u)
    g = int(nbr[f, k])
    if g >= 0:
        a_in = _across(a, b, v[(k + 2) % 3], ehat)
        vg = tris[g].astype(np.float64)
        third = [x for x in vg if not (np.array_equal(x, a) or np.array_equal(x, b))][0]
        b_in = _across(a, b, third, ehat)
        cab = _dot(_cross(a_in, b_in), ehat)
    qo = q - o
    path = L + math.sqrt(_dot(qo, qo))
    out = []
    for j in range(cone.shape[0]):
        cj, sj = float(cone[j, 0]), float(cone[j, 1])
        perp = sb * (cj * u + sj * w)
        dk = c * ehat + perp
        if g >= 0:
            s1 = _dot(_cross(a_in, perp), ehat)
            s2 = _dot(_cross(perp, b_in), ehat)
            if (s1 > 0 and s2 > 0 and cab > 0) or (s1 < 0 and s2 < 0 and cab < 0):
                continue
        out.append((k, j, path, q.astype(np.float32), dk.astype(np.float32)))
    return out


def diffract(tris, nbr, seg, hit_id, hit_t, delta, cone) -> np.ndarray:
    """Every diffracted ray of stored chains (seg [max_b, m, 8], hit_id /
    hit_t [max_b, m], as for reception), sorted by (ray, order, cone)."""
    from oracle.reception import path_prefix
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    seg = np.asarray(seg)
    hit_id = np.asarray(hit_id)
    hit_t = np.asarray(hit_t)
    L = path_prefix(seg, hit_id, hit_t)
    rows = []
    max_b, m = hit_id.shape
    for b in range(max_b):
        for i in np.nonzero(~np.isnan(L[b]) & (hit_id[b] >= 0))[0]:
            s = seg[b, i].astype(np.float64)
            for k, j, path, q, dk in diffract_one(tris, nbr, int(hit_id[b, i]), s[0:3], s[4:7],
                                                  hit_t[b, i], L[b, i], s[3], s[7], delta, cone):
                rows.append((i, b, int(hit_id[b, i]), k, j, 0, path, q, np.float32(s[3]), dk,
                             np.float32(s[7])))
    out = np.array(rows, dtype=DIFFRACTED) if rows else np.zeros(0, DIFFRACTED)
    return np.sort(out, order=("ray", "order", "cone"))
