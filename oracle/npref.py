"""Second, independent closest-hit checker for tiny scenes: TEST INFRASTRUCTURE.

Each ray/facet crossing is found by solving the 3 x 3 linear system
``o + t d = v0 + u (v1 - v0) + v (v2 - v0)`` with LAPACK (numpy.linalg.solve,
LU with partial pivoting) instead of the cross-product formulation of the
C++ checker, so a slip in either formulation shows up as a disagreement.
Closest hit = lexicographic min of (t, facet id) over crossings inside the
closed triangle with t in the closed [tmin, tmax] (Sec. III-B keeps the
nearest facet).
"""
from __future__ import annotations

import numpy as np


def brute_solve(tris: np.ndarray, rays: np.ndarray, skip=None):
    """Returns (id int32, t float64) per ray; quadratic in size, tiny inputs only."""
    tris = np.asarray(tris, dtype=np.float32).astype(np.float64).reshape(-1, 3, 3)
    rays = np.asarray(rays, dtype=np.float32).astype(np.float64)
    m, n = rays.shape[0], tris.shape[0]
    o, tmin, d, tmax = rays[:, 0:3], rays[:, 3], rays[:, 4:7], rays[:, 7]
    v0 = tris[:, 0]
    e1 = tris[:, 1] - v0
    e2 = tris[:, 2] - v0
    ids = np.full(m, -1, np.int32)
    ts = np.full(m, np.inf)
    for i in range(m):
        a = np.empty((n, 3, 3))
        a[:, :, 0] = -d[i][None, :]
        a[:, :, 1] = e1
        a[:, :, 2] = e2
        rhs = o[i][None, :] - v0
        det = np.linalg.det(a)
        ok = det != 0.0
        sol = np.full((n, 3), np.nan)
        if ok.any():
            sol[ok] = np.linalg.solve(a[ok], rhs[ok][..., None])[..., 0]
        t, u, v = sol[:, 0], sol[:, 1], sol[:, 2]
        hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t >= tmin[i]) & (t <= tmax[i])
        if skip is not None and skip[i] >= 0:
            hit[skip[i]] = False
        if hit.any():
            cand = np.nonzero(hit)[0]
            order = np.lexsort((cand, t[cand]))
            j = cand[order[0]]
            ids[i] = j
            ts[i] = t[j]
    return ids, ts
