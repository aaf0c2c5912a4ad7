"""Ray launching from a subdivided regular icosahedron (Sec. III-A).

The source point is joined to the vertices of an icosahedron whose 20
equilateral faces are split into smaller triangles; each vertex gives one
launch direction.  The paper does not say how the faces are subdivided, so
this module uses the usual geodesic construction:

* level 0 is the regular icosahedron, vertices at the cyclic permutations of
  (0, +-1, +-phi) scaled to unit length, 12 vertices and 20 faces;
* each further level splits every face into four by its edge midpoints and
  pushes the midpoints out to the unit sphere;
* vertices created at a level are appended in order of first appearance
  (faces in order, then edges ab, bc, ca of each face), so the vertex list of
  level L-1 is a prefix of the one of level L.

Level L has 10 * 4**L + 2 vertices (10,242 at L = 5, 2,621,442 at L = 9).
Everything is computed in float64 and rounded to float32 only when rays are
packed, so both the GPU path and the CPU checker see the same float32 rays.
This module holds input generation only, none of the tracing arithmetic.
"""
from __future__ import annotations

import functools

import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _unit(v: np.ndarray) -> np.ndarray:
    n = np.sqrt(v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1] + v[:, 2] * v[:, 2])
    return v / n[:, None]


def _base() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron: 12 unit vertices, 20 outward-oriented faces."""
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * PHI))
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((s1, s2 * PHI, 0.0))
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((s1 * PHI, 0.0, s2))
    raw = np.array(pts, dtype=np.float64)
    # adjacent vertices are exactly 2 apart before normalisation
    d2 = ((raw[:, None, :] - raw[None, :, :]) ** 2).sum(-1)
    adj = np.abs(d2 - 4.0) < 1e-9
    faces = []
    for a in range(12):
        for b in range(a + 1, 12):
            if not adj[a, b]:
                continue
            for c in range(b + 1, 12):
                if adj[a, c] and adj[b, c]:
                    n = np.cross(raw[b] - raw[a], raw[c] - raw[a])
                    if np.dot(n, raw[a] + raw[b] + raw[c]) < 0:
                        faces.append((a, c, b))
                    else:
                        faces.append((a, b, c))
    f = np.array(faces, dtype=np.int64)
    assert f.shape == (20, 3)
    return _unit(raw), f


def _subdivide(verts: np.ndarray, faces: np.ndarray):
    nv = verts.shape[0]
    # edges in face order: ab, bc, ca
    e = np.stack([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]], axis=1)
    e = e.reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo * nv + hi
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    # number the unique edges by first appearance
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    mid_index = nv + rank[inv]                      # per face-edge new vertex id
    ue_lo = (uniq // nv)[order]
    ue_hi = (uniq % nv)[order]
    mids = _unit(verts[ue_lo] + verts[ue_hi])
    new_verts = np.concatenate([verts, mids], axis=0)
    m = mid_index.reshape(-1, 3)                    # m_ab, m_bc, m_ca
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    mab, mbc, mca = m[:, 0], m[:, 1], m[:, 2]
    nf = np.stack([
        np.stack([a, mab, mca], 1),
        np.stack([b, mbc, mab], 1),
        np.stack([c, mca, mbc], 1),
        np.stack([mab, mbc, mca], 1),
    ], axis=1).reshape(-1, 3)
    return new_verts, nf


@functools.lru_cache(maxsize=4)
def _level(level: int):
    verts, faces = _base()
    for _ in range(level):
        verts, faces = _subdivide(verts, faces)
    verts.setflags(write=False)
    faces.setflags(write=False)
    return verts, faces


def vertex_count(level: int) -> int:
    return 10 * 4 ** level + 2


def directions(level: int) -> np.ndarray:
    """Unit launch directions (float64, [10*4**L+2, 3]) of a level-L icosphere."""
    if level < 0 or level > 10:
        raise ValueError("icosphere level must be in 0..10")
    return _level(level)[0]


def faces(level: int) -> np.ndarray:
    """Triangles (int64 vertex ids) of the level-L icosphere."""
    return _level(level)[1]


def directions_n(n: int) -> np.ndarray:
    """First n directions of the smallest level holding at least n vertices."""
    if n <= 0:
        raise ValueError("n must be positive")
    level = 0
    while vertex_count(level) < n:
        level += 1
    return directions(level)[:n]


def make_rays(src, dirs: np.ndarray, tmin: float, tmax: float) -> np.ndarray:
    """Pack rays as float32 [n, 8] = (ox, oy, oz, tmin, dx, dy, dz, tmax)."""
    dirs = np.asarray(dirs)
    n = dirs.shape[0]
    r = np.empty((n, 8), dtype=np.float32)
    r[:, 0:3] = np.asarray(src, dtype=np.float64)[None, :]
    r[:, 3] = tmin
    r[:, 4:7] = dirs.astype(np.float32)
    r[:, 7] = tmax
    return r


def angular_spacing(level: int) -> float:
    """Nominal angle (rad) between adjacent launch directions at a level:
    the icosahedron edge angle halved once per subdivision."""
    edge = np.arccos(1.0 / np.sqrt(5.0))   # 63.43 degrees
    return float(edge / 2 ** level)


@functools.lru_cache(maxsize=None)
def edge_angles(level: int) -> np.ndarray:
    """Angles (rad, float64) between the launch directions joined by an edge
    of the subdivided icosahedron at a level, one per edge.  Their mean and
    maximum are the usual choices for the angle between adjacent rays."""
    v = directions(level)
    f = faces(level)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e = np.sort(e, axis=1)
    # one key per undirected edge; sorted unique keys list the edges in
    # lexicographic (lo, hi) order
    key = np.unique(e[:, 0] * np.int64(v.shape[0]) + e[:, 1])
    e = np.stack([key // v.shape[0], key % v.shape[0]], 1)
    c = np.clip((v[e[:, 0]] * v[e[:, 1]]).sum(1), -1.0, 1.0)
    return np.arccos(c)
