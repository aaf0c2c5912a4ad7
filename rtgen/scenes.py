"""Seeded synthetic urban scenes standing in for the paper's SketchUp models.

The paper's indoor study room (2,778 facets) and outdoor campus (7,608
facets) are not available, so the workloads here are synthetic cities of the
same kind: a flat ground made of two triangles plus buildings made of
triangular facets (Sec. II-A stores every obstacle as triangular facets).
Units are metres, z is up, the ground is z = 0.

Every generator draws from ``numpy.random.default_rng(seed)`` in the order
written in its docstring, builds vertices in float64 and returns float32
triangles ``[n, 9] = (v0.xyz, v1.xyz, v2.xyz)``.  Nothing here computes any
part of the tracing or building method.
"""
from __future__ import annotations

import math

import numpy as np


def _ground(half: float) -> list:
    a = (-half, -half, 0.0)
    b = (half, -half, 0.0)
    c = (half, half, 0.0)
    d = (-half, half, 0.0)
    return [(a, b, c), (a, c, d)]


def _quad(p0, p1, p2, p3) -> list:
    """Two triangles of the planar quad p0 p1 p2 p3 (in order around it)."""
    return [(p0, p1, p2), (p0, p2, p3)]


def _box_tris(x0, y0, x1, y1, h, floor: bool) -> list:
    """Axis-aligned box building: 4 walls (2 tris each), roof (2), floor (2)."""
    c = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    tris = []
    for k in range(4):
        (ax, ay), (bx, by) = c[k], c[(k + 1) % 4]
        tris += _quad((ax, ay, 0.0), (bx, by, 0.0), (bx, by, h), (ax, ay, h))
    tris += _quad(*[(x, y, h) for (x, y) in c])
    if floor:
        tris += _quad(*[(x, y, 0.0) for (x, y) in reversed(c)])
    return tris


def _prism_tris(poly, h) -> list:
    """Extruded convex polygon: n walls (2 tris each) and a fan roof (n - 2)."""
    n = len(poly)
    tris = []
    for k in range(n):
        (ax, ay), (bx, by) = poly[k], poly[(k + 1) % n]
        tris += _quad((ax, ay, 0.0), (bx, by, 0.0), (bx, by, h), (ax, ay, h))
    r0 = (poly[0][0], poly[0][1], h)
    for k in range(1, n - 1):
        tris.append((r0, (poly[k][0], poly[k][1], h),
                     (poly[k + 1][0], poly[k + 1][1], h)))
    return tris


def _pack(tris: list) -> np.ndarray:
    return np.asarray(tris, dtype=np.float64).reshape(-1, 9).astype(np.float32)


def _covers(bx0, by0, bx1, by1, tx, ty, pad=1.0) -> bool:
    return (bx0 - pad <= tx <= bx1 + pad) and (by0 - pad <= ty <= by1 + pad)


def microcell(seed: int = 0, tx=(0.0, 0.0, 10.0)) -> np.ndarray:
    """200 x 200 m ground (2 tris) + 20 closed axis-aligned boxes (12 tris
    each) = 242 triangles.

    Per building, draws in order: side_x ~ U(10,30), side_y ~ U(10,30),
    centre_x ~ U(-100 + sx/2, 100 - sx/2), centre_y likewise,
    height ~ U(5,40).  A building whose footprint grown by 1 m covers the
    transmitter's (x, y) is discarded and drawn again.
    """
    rng = np.random.default_rng(seed)
    half = 100.0
    tris = _ground(half)
    placed = 0
    while placed < 20:
        sx = rng.uniform(10, 30)
        sy = rng.uniform(10, 30)
        cx = rng.uniform(-half + sx / 2, half - sx / 2)
        cy = rng.uniform(-half + sy / 2, half - sy / 2)
        h = rng.uniform(5, 40)
        x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
        if _covers(x0, y0, x1, y1, tx[0], tx[1]):
            continue
        tris += _box_tris(x0, y0, x1, y1, h, floor=True)
        placed += 1
    return _pack(tris)


def _draw_building(rng, half, tx, box_frac=0.733):
    """One floorless building; returns (footprint polygon, height, kind).

    Draw order: kind ~ U(0,1) (< box_frac: box), height ~ lognormal(ln 15,
    0.6) clipped to [3, 120]; box: side_x, side_y ~ U(10,30), centre_x,
    centre_y uniform with the footprint inside the area; prism: n ~ U{5..8},
    radius ~ U(6,15), rotation ~ U(0, 2 pi), n angle jitters ~ U(-0.3, 0.3)
    (fractions of the angular step), centre_x, centre_y uniform.
    """
    while True:
        kind = rng.uniform()
        h = float(np.clip(rng.lognormal(math.log(15.0), 0.6), 3.0, 120.0))
        if kind < box_frac:
            sx = rng.uniform(10, 30)
            sy = rng.uniform(10, 30)
            cx = rng.uniform(-half + sx / 2, half - sx / 2)
            cy = rng.uniform(-half + sy / 2, half - sy / 2)
            x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
            poly = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        else:
            n = int(rng.integers(5, 9))
            rad = rng.uniform(6, 15)
            rot = rng.uniform(0, 2 * math.pi)
            jit = rng.uniform(-0.3, 0.3, size=n)
            cx = rng.uniform(-half + rad, half - rad)
            cy = rng.uniform(-half + rad, half - rad)
            step = 2 * math.pi / n
            ang = rot + step * (np.arange(n) + jit)
            poly = [(cx + rad * math.cos(a), cy + rad * math.sin(a)) for a in ang]
        xs = [p[0] for p in poly]
        ys = [p[1] for p in poly]
        if tx is not None and _covers(min(xs), min(ys), max(xs), max(ys), tx[0], tx[1]):
            continue
        return poly, h


def city(seed: int = 0, n_buildings: int = 2000, half: float = 1000.0,
         tx=(0.0, 0.0, 25.0)) -> np.ndarray:
    """Ground (2 tris) + floorless buildings: about 73.3 % axis-aligned boxes
    (10 tris) and 26.7 % convex 5..8-gon prisms (3n - 2 tris), 12 tris per
    building on average; 2,000 buildings on 2 x 2 km give about 24k tris."""
    rng = np.random.default_rng(seed)
    tris = _ground(half)
    for _ in range(n_buildings):
        poly, h = _draw_building(rng, half, tx)
        tris += _prism_tris(poly, h) if len(poly) != 4 else _box_tris(
            poly[0][0], poly[0][1], poly[2][0], poly[2][1], h, floor=False)
    return _pack(tris)


def _grid_building(rng, poly, h, jitter=0.2) -> list:
    """Watertight tessellation of one building: every wall becomes a grid of
    cells, interior grid vertices are moved in the wall plane, and the roof is
    a fan from its centre over the (subdivided) top edges.

    Draw order: vertical cell ~ U(2,8) (shared by all walls, so neighbouring
    walls share their corner vertices); then per wall: cell ~ U(2,8), then the
    (nu - 1) * (nv - 1) interior jitters along the wall and in z.
    """
    n = len(poly)
    cv = rng.uniform(2, 8)
    nv = max(1, int(round(h / cv)))
    zs = [h * j / nv for j in range(nv + 1)]
    top = []
    tris = []
    for k in range(n):
        (ax, ay), (bx, by) = poly[k], poly[(k + 1) % n]
        length = math.hypot(bx - ax, by - ay)
        cu = rng.uniform(2, 8)
        nu = max(1, int(round(length / cu)))
        ex, ey = (bx - ax) / length, (by - ay) / length
        # vertex grid (nu+1) x (nv+1)
        g = [[None] * (nv + 1) for _ in range(nu + 1)]
        jit = rng.uniform(-jitter, jitter, size=(max(nu - 1, 0), max(nv - 1, 0), 2))
        for i in range(nu + 1):
            s = length * i / nu
            for j in range(nv + 1):
                x, y, z = ax + ex * s, ay + ey * s, zs[j]
                if 0 < i < nu and 0 < j < nv:
                    du, dz = jit[i - 1, j - 1]
                    x, y, z = x + ex * du, y + ey * du, z + dz
                g[i][j] = (x, y, z)
        # corners come from the polygon vertices exactly, shared by both walls
        for j in range(nv + 1):
            g[0][j] = (ax, ay, zs[j])
            g[nu][j] = (bx, by, zs[j])
        for i in range(nu):
            for j in range(nv):
                tris += _quad(g[i][j], g[i + 1][j], g[i + 1][j + 1], g[i][j + 1])
        top += [g[i][nv] for i in range(nu)]
    cx = sum(p[0] for p in poly) / n
    cy = sum(p[1] for p in poly) / n
    c = (cx, cy, h)
    m = len(top)
    for k in range(m):
        tris.append((c, top[k], top[(k + 1) % m]))
    return tris


def dense_city(seed: int = 0, min_tris: int = 200_000, half: float = 1500.0,
               tx_list=((-750.0, -750.0, 25.0), (750.0, -750.0, 25.0),
                        (-750.0, 750.0, 25.0), (750.0, 750.0, 25.0))) -> np.ndarray:
    """Ground + buildings drawn as in :func:`city` (rejected when they cover
    any of the transmitters) with tessellated facades, added until the scene
    holds at least ``min_tris`` triangles."""
    rng = np.random.default_rng(seed)
    tris = _ground(half)
    while len(tris) < min_tris:
        while True:
            poly, h = _draw_building(rng, half, None)
            xs = [p[0] for p in poly]
            ys = [p[1] for p in poly]
            if not any(_covers(min(xs), min(ys), max(xs), max(ys), t[0], t[1])
                       for t in tx_list):
                break
        tris += _grid_building(rng, poly, h)
    return _pack(tris)


_ROOF_BOXES: dict = {}


def _roof_boxes(tris: np.ndarray):
    """Footprint boxes (grown by 1 m) of the flat roof facets, cached per array."""
    key = (tris.__array_interface__["data"][0], tris.shape)
    hit = _ROOF_BOXES.get(key)
    if hit is not None and hit[0] is tris:
        return hit[1], hit[2]
    roofs = tris.reshape(-1, 3, 3)
    flat = (roofs[:, 0, 2] == roofs[:, 1, 2]) & (roofs[:, 1, 2] == roofs[:, 2, 2]) \
        & (roofs[:, 0, 2] > 0)
    r = roofs[flat].astype(np.float64)
    lo = r[:, :, :2].min(1) - 1.0
    hi = r[:, :, :2].max(1) + 1.0
    if len(_ROOF_BOXES) > 16:
        _ROOF_BOXES.clear()
    _ROOF_BOXES[key] = (tris, lo, hi)
    return lo, hi


def free_point(tris_seed_rng, half, tris: np.ndarray, z) -> tuple:
    """Uniform (x, y) in the area whose vertical line meets no roof facet,
    i.e. not inside a building (walls and roofs have z > 0 vertices)."""
    rng = tris_seed_rng
    lo, hi = _roof_boxes(tris)
    while True:
        x = rng.uniform(-half * 0.95, half * 0.95)
        y = rng.uniform(-half * 0.95, half * 0.95)
        if not np.any((lo[:, 0] <= x) & (x <= hi[:, 0]) & (lo[:, 1] <= y) & (y <= hi[:, 1])):
            return (float(x), float(y), float(z))
