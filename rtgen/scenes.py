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


def free_points(rng, half, tris: np.ndarray, z, count: int) -> np.ndarray:
    """`count` points drawn like free_point (uniform (x, y) not inside a
    building, height z), float64 [count, 3]."""
    lo, hi = _roof_boxes(tris)
    out = np.empty((0, 3))
    while out.shape[0] < count:
        xy = rng.uniform(-half * 0.95, half * 0.95, size=(2 * count, 2))
        inside = np.zeros(xy.shape[0], bool)
        for k in range(0, lo.shape[0], 256):
            a, b = lo[k:k + 256], hi[k:k + 256]
            inside |= ((a[None, :, 0] <= xy[:, None, 0]) & (xy[:, None, 0] <= b[None, :, 0]) &
                       (a[None, :, 1] <= xy[:, None, 1]) & (xy[:, None, 1] <= b[None, :, 1])).any(1)
        keep = xy[~inside]
        out = np.concatenate([out, np.column_stack([keep, np.full(keep.shape[0], float(z))])])
    return out[:count]


# ---------------------------------------------------------------------------
# Materials the paper names for its scenes (Sec. IV-A), as indices.
MATERIALS = ("concrete", "wood", "metal", "glass")
CONCRETE, WOOD, METAL, GLASS = range(4)


# ---------------------------------------------------------------------------
# Paper-size stand-ins: an 8 x 6 x 3.5 m study room of exactly 2,778 facets
# and a campus of exactly 7,608 facets (the paper's facet counts, Sec. IV-A).


def _box(x0, y0, z0, x1, y1, z1) -> list:
    """Closed axis-aligned box, 12 triangles."""
    c = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    tris = []
    for k in range(4):
        (ax, ay), (bx, by) = c[k], c[(k + 1) % 4]
        tris += _quad((ax, ay, z0), (bx, by, z0), (bx, by, z1), (ax, ay, z1))
    tris += _quad(*[(x, y, z1) for (x, y) in c])
    tris += _quad(*[(x, y, z0) for (x, y) in reversed(c)])
    return tris


def _disc(cx, cy, z, r, m) -> list:
    """Flat disc of radius r at height z as a fan of m >= 3 triangles."""
    pts = [(cx + r * math.cos(2 * math.pi * k / m), cy + r * math.sin(2 * math.pi * k / m), z)
           for k in range(m)]
    return [((cx, cy, z), pts[k], pts[(k + 1) % m]) for k in range(m)]


def study_room(seed: int = 0, target: int = 2778, materials: bool = False):
    """Study room 8 x 6 x 3.5 m ([0, 8] x [0, 6] x [0, 3.5]) furnished like
    the paper's indoor scene: shell (floor, ceiling, 4 walls: 12 facets), 12
    desks (top + 4 legs: 60 each) with 12 chairs (seat, back, 4 legs: 72
    each) in a 4 x 3 grid at x >= 2.8, 6 windows (pane 0.03 m inside the
    wall, 4 frame bars, 6 guard-rail bars: 122 each) on the walls y = 6 and
    x = 8, a door (slab + handle) on the wall y = 0, 3 cabinets and an open
    bookshelf (2 sides, back, 5 shelves), a podium, a whiteboard, 6 ceiling
    lamps, and a round table whose top is a fan of as many triangles as are
    needed to reach ``target`` facets.  The paper's Tx (1.46, 2.42, 2.1) and
    Rx (1.2, 1.2, 1.5) stay in free space.

    Draw order: per desk (row-major) dx, dy ~ U(-0.1, 0.1), width scale
    ~ U(0.95, 1.05); per lamp dx ~ U(-0.2, 0.2).

    With ``materials``, also returns the material index (``MATERIALS``) of
    every facet, as the paper describes the room: walls, floor and ceiling
    concrete; desks, chairs, door, cabinets, shelves, podium, whiteboard and
    table wood; window frames, guard rails, door handle and lamps metal;
    window panes glass."""
    rng = np.random.default_rng(seed)
    X, Y, H = 8.0, 6.0, 3.5
    t = []
    mat = []

    def tag(code):  # facets added since the last tag get this material
        mat.extend([code] * (len(t) - len(mat)))
    t += _quad((0, 0, 0), (X, 0, 0), (X, Y, 0), (0, Y, 0))
    t += _quad((0, 0, H), (0, Y, H), (X, Y, H), (X, 0, H))
    t += _quad((0, 0, 0), (0, Y, 0), (0, Y, H), (0, 0, H))
    t += _quad((X, 0, 0), (X, 0, H), (X, Y, H), (X, Y, 0))
    t += _quad((0, 0, 0), (0, 0, H), (X, 0, H), (X, 0, 0))
    t += _quad((0, Y, 0), (X, Y, 0), (X, Y, H), (0, Y, H))
    tag(CONCRETE)
    for row in range(3):
        for col in range(4):
            dx, dy = rng.uniform(-0.1, 0.1, 2)
            sw = rng.uniform(0.95, 1.05)
            x0, y0 = 2.9 + 1.25 * col + dx, 0.9 + 1.6 * row + dy
            w, d = 1.0 * sw, 0.6
            t += _box(x0, y0, 0.72, x0 + w, y0 + d, 0.75)
            for lx, ly in ((x0 + 0.03, y0 + 0.03), (x0 + w - 0.08, y0 + 0.03),
                           (x0 + 0.03, y0 + d - 0.08), (x0 + w - 0.08, y0 + d - 0.08)):
                t += _box(lx, ly, 0.0, lx + 0.05, ly + 0.05, 0.72)
            cx0, cy0 = x0 + 0.3, y0 + d + 0.15
            t += _box(cx0, cy0, 0.42, cx0 + 0.42, cy0 + 0.42, 0.46)
            t += _box(cx0, cy0 + 0.38, 0.46, cx0 + 0.42, cy0 + 0.42, 0.9)
            for lx, ly in ((cx0, cy0), (cx0 + 0.38, cy0), (cx0, cy0 + 0.38), (cx0 + 0.38, cy0 + 0.38)):
                t += _box(lx, ly, 0.0, lx + 0.04, ly + 0.04, 0.42)
    tag(WOOD)

    def window(u0, u1, wall):  # wall "y" (y = 6) or "x" (x = 8); u along the wall
        # returns (pane facets, frame and guard-rail facets)
        z0, z1, inset = 0.9, 2.3, 0.03
        w = []
        if wall == "y":
            p = lambda u, v, z: (u, Y - v, z)
        else:
            p = lambda u, v, z: (X - v, u, z)

        def slab(ua, ub, va, vb, za, zb):
            a, b = p(ua, va, za), p(ub, vb, zb)
            return _box(min(a[0], b[0]), min(a[1], b[1]), za, max(a[0], b[0]), max(a[1], b[1]), zb)

        pane = _quad(p(u0, inset, z0), p(u1, inset, z0), p(u1, inset, z1), p(u0, inset, z1))
        w += slab(u0 - 0.05, u1 + 0.05, 0.0, 0.06, z0 - 0.05, z0)
        w += slab(u0 - 0.05, u1 + 0.05, 0.0, 0.06, z1, z1 + 0.05)
        w += slab(u0 - 0.05, u0, 0.0, 0.06, z0, z1)
        w += slab(u1, u1 + 0.05, 0.0, 0.06, z0, z1)
        for k in range(6):
            u = u0 + (k + 0.5) * (u1 - u0) / 6
            w += slab(u - 0.01, u + 0.01, 0.12, 0.14, z0, z1)
        return pane, w

    for wall, centres in (("y", (4.0, 5.5, 7.0)), ("x", (1.5, 3.0, 4.5))):
        for uc in centres:
            pane, metal = window(uc - 0.6, uc + 0.6, wall)
            t += pane
            tag(GLASS)
            t += metal
            tag(METAL)
    t += _box(6.5, 0.02, 0.0, 7.4, 0.06, 2.1)
    tag(WOOD)
    t += _box(6.6, 0.06, 1.0, 6.75, 0.1, 1.05)
    tag(METAL)
    for cx in (0.3, 1.25, 2.2):
        t += _box(cx, 5.5, 0.0, cx + 0.9, 5.95, 2.0)
    t += _box(0.05, 3.8, 0.0, 0.4, 3.82, 2.2)
    t += _box(0.05, 5.28, 0.0, 0.4, 5.3, 2.2)
    t += _box(0.02, 3.8, 0.0, 0.05, 5.3, 2.2)
    for z in (0.02, 0.5, 1.0, 1.5, 2.0):
        t += _box(0.05, 3.82, z, 0.4, 5.28, z + 0.02)
    t += _box(0.6, 3.0, 0.0, 1.2, 3.5, 1.1)
    t += _box(0.02, 0.6, 0.9, 0.04, 2.9, 2.1)
    tag(WOOD)
    for k in range(6):
        lx = 2.4 + 1.8 * (k % 3) + rng.uniform(-0.2, 0.2)
        ly = 1.5 if k < 3 else 4.2
        t += _box(lx, ly, 3.34, lx + 1.2, ly + 0.3, 3.4)
    tag(METAL)
    rest = target - len(t) - 4 * 12
    if rest < 3:
        raise ValueError("study_room: target below the furniture's facet count")
    t += _disc(1.9, 4.4, 0.75, 0.55, rest)
    for lx, ly in ((1.85, 4.35), (1.85, 4.4), (1.9, 4.35), (1.9, 4.4)):
        t += _box(lx, ly, 0.0, lx + 0.03, ly + 0.03, 0.75)
    tag(WOOD)
    assert len(t) == target and len(mat) == target
    return (_pack(t), np.array(mat, np.int32)) if materials else _pack(t)


def _tessellated_building(rng, poly, h, cell) -> list:
    """Walls of an extruded convex polygon as grids of about cell x cell m
    quads, and a fan roof over the top edge points.  Draw order: nothing
    (deterministic)."""
    n = len(poly)
    nv = max(1, int(round(h / cell)))
    zs = [h * j / nv for j in range(nv + 1)]
    tris, top = [], []
    for k in range(n):
        (ax, ay), (bx, by) = poly[k], poly[(k + 1) % n]
        nu = max(1, int(round(math.hypot(bx - ax, by - ay) / cell)))
        g = [[(ax + (bx - ax) * i / nu, ay + (by - ay) * i / nu, z) for z in zs] for i in range(nu + 1)]
        for i in range(nu):
            for j in range(nv):
                tris += _quad(g[i][j], g[i + 1][j], g[i + 1][j + 1], g[i][j + 1])
        top += [g[i][nv] for i in range(nu)]
    cx = sum(p[0] for p in poly) / n
    cy = sum(p[1] for p in poly) / n
    c = (cx, cy, h)
    tris += [(c, top[k], top[(k + 1) % len(top)]) for k in range(len(top))]
    return tris


def campus(seed: int = 0, target: int = 7608, size: float = 1000.0,
           keep_free=((450.0, 450.0), (450.0, 550.0)), materials: bool = False):
    """Campus of exactly ``target`` facets on [0, size]^2: ground (2 facets),
    non-overlapping buildings with tessellated facades, and a playground whose
    flat oval track (a fan 0.05 m above the ground) takes the facets left over.

    Per building, draws in order: kind ~ U(0, 1) (< 0.7 rectangular), height
    ~ lognormal(ln 18, 0.5) clipped to [6, 60] m, facade cell ~ U(6, 15) m;
    rectangle: sides ~ U(20, 90) and U(15, 40) m, rotation 0 or 90 degrees
    ~ U{0, 1}; prism: n ~ U{5..8} corners on a circle of radius ~ U(12, 35)
    m; then the centre uniform with the footprint inside the area.  A
    building whose box (grown by 10 m) meets another's, or covers a point of
    ``keep_free`` (the paper's Tx and Rx), is drawn again; buildings are
    added while the facet count stays 300 below the target (at most 4,000
    draws).  With ``materials``, also returns a material index per facet:
    ground and playground concrete, each building concrete or (with
    probability 0.3, drawn from a second generator seeded seed + 1 in
    building order) glass."""
    rng = np.random.default_rng(seed)
    mrng = np.random.default_rng(seed + 1)
    t = _quad((0, 0, 0), (size, 0, 0), (size, size, 0), (0, size, 0))
    mat = [CONCRETE, CONCRETE]
    boxes = []
    play = (180.0, 780.0, 90.0, 55.0)   # playground centre and half-axes, kept free
    boxes.append((play[0] - play[2], play[1] - play[3], play[0] + play[2], play[1] + play[3]))
    draws = 0
    while draws < 4000 and len(t) < target - 300:
        draws += 1
        kind = rng.uniform()
        h = float(np.clip(rng.lognormal(math.log(18.0), 0.5), 6.0, 60.0))
        cell = rng.uniform(6.0, 15.0)
        if kind < 0.7:
            a, b = rng.uniform(20, 90), rng.uniform(15, 40)
            if rng.integers(0, 2):
                a, b = b, a
            cx, cy = rng.uniform(a / 2, size - a / 2), rng.uniform(b / 2, size - b / 2)
            poly = [(cx - a / 2, cy - b / 2), (cx + a / 2, cy - b / 2),
                    (cx + a / 2, cy + b / 2), (cx - a / 2, cy + b / 2)]
        else:
            n = int(rng.integers(5, 9))
            rad = rng.uniform(12, 35)
            cx, cy = rng.uniform(rad, size - rad), rng.uniform(rad, size - rad)
            poly = [(cx + rad * math.cos(2 * math.pi * k / n), cy + rad * math.sin(2 * math.pi * k / n))
                    for k in range(n)]
        xs, ys = [p[0] for p in poly], [p[1] for p in poly]
        bb = (min(xs) - 10, min(ys) - 10, max(xs) + 10, max(ys) + 10)
        if any(bb[0] <= fx <= bb[2] and bb[1] <= fy <= bb[3] for fx, fy in keep_free):
            continue
        if any(bb[0] < o[2] and o[0] < bb[2] and bb[1] < o[3] and o[1] < bb[3] for o in boxes):
            continue
        bt = _tessellated_building(rng, poly, h, cell)
        if len(t) + len(bt) > target - 64:
            continue
        boxes.append(bb)
        t += bt
        mat += [GLASS if mrng.uniform() < 0.3 else CONCRETE] * len(bt)
    rest = target - len(t)
    cx, cy, ax, ay = play
    pts = [(cx + ax * math.cos(2 * math.pi * k / rest), cy + ay * math.sin(2 * math.pi * k / rest), 0.05)
           for k in range(rest)]
    t += [((cx, cy, 0.05), pts[k], pts[(k + 1) % rest]) for k in range(rest)]
    mat += [CONCRETE] * rest
    assert len(t) == target and len(mat) == target
    return (_pack(t), np.array(mat, np.int32)) if materials else _pack(t)
