"""Ray reception by receiving spheres (Sec. III-C, Eq. (4)) -- CPU checker.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline use this module; the GPU library never does.

What is computed (plain definition, float64, no fused multiply-add):

A traced ray is a chain of segments.  Segment b of ray i starts at o_b with
direction d_b (not necessarily unit) and covers the ray parameters
[t0_b, t1_b], where t0_b is the ray's tmin and t1_b is the hit parameter if
the segment hit a facet, else its tmax.  Segment b exists when b == 0 or
segment b-1 hit.  The path length up to the start of segment b is
L_b = sum_{j<b} t_hit_j * |d_j|, the same sum the tracer reports as the
path length.

A field point R receives segment b when

  * the foot of the perpendicular from R onto the segment's line lies in the
    segment: with w = R - o_b and s = (w . d_b) / (d_b . d_b),
    t0_b <= s <= t1_b, and
  * R lies inside the receiving sphere of Eq. (4): with the distance
    dist^2 = |w - s d_b|^2 and the path length from the source to R along
    the ray, l = L_b + |w|, the test is 3 dist^2 <= (l delta)^2, i.e.
    dist <= l delta / sqrt(3), where delta is the angle between adjacent
    launched rays.

Readings the paper leaves open (it gives Eq. (4) and the meaning of l and
delta only): l is measured to the field point itself (the unfolded path
source -> reflection points -> R); a segment counts only when the foot of
the perpendicular falls inside it; delta is one number per launch, passed
in.  The arithmetic order above is the definition both this checker and the
GPU kernel follow, so that the same float inputs give the same decisions.

Duplicates: neighbouring rays can all be received for one propagation path,
because their receiving spheres overlap.  ``dedup`` keeps one reception per
(receiver, order, sequence of facets hit before the segment): the one with
the smallest dist, ties to the smaller ray index.  The paper does not say how
the received rays are grouped before they are superposed; this is the
usual shooting-and-bouncing-rays treatment and is a reading.
"""
from __future__ import annotations

import numpy as np

RECEPTION = np.dtype([("rx", np.int32), ("ray", np.int32), ("order", np.int32),
                      ("keep", np.int32), ("l", np.float64), ("dist", np.float64)])


def path_prefix(seg: np.ndarray, hit_id: np.ndarray, hit_t: np.ndarray) -> np.ndarray:
    """Path length before each segment (Sec. III-C: l counts the whole path
    from the source; Sec. III-B: a reflected ray starts at the hit point).
    L_b for every segment: [max_b, m] float64, L_0 = 0 and
    L_{b+1} = L_b + t_hit_b * sqrt(d_b . d_b) (NaN where the segment does
    not exist)."""
    max_b, m = hit_id.shape
    L = np.full((max_b, m), np.nan)
    L[0] = 0.0
    for b in range(1, max_b):
        prev = hit_id[b - 1] >= 0
        d = seg[b - 1, :, 4:7].astype(np.float64)
        dd = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        step = hit_t[b - 1].astype(np.float64) * np.sqrt(dd)
        L[b] = np.where(prev & ~np.isnan(L[b - 1]), L[b - 1] + step, np.nan)
    return L


def segment_receives(o, d, t0, t1, L, rx, delta):
    """Sec. III-C, Eq. (4): the receiving-sphere test of one field point rx against many segments (arrays
    of float64 of length k).  Returns (received, l, dist)."""
    wx, wy, wz = rx[0] - o[:, 0], rx[1] - o[:, 1], rx[2] - o[:, 2]
    dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
    dd = dx * dx + dy * dy + dz * dz
    with np.errstate(invalid="ignore", divide="ignore"):
        s = (wx * dx + wy * dy + wz * dz) / dd
        px, py, pz = wx - s * dx, wy - s * dy, wz - s * dz
        dist2 = px * px + py * py + pz * pz
        l = L + np.sqrt(wx * wx + wy * wy + wz * wz)
        rr = l * delta
        ok = (s >= t0) & (s <= t1) & (3.0 * dist2 <= rr * rr)
    return ok, l, np.sqrt(dist2)


def receive(seg, hit_id, hit_t, receivers, delta) -> np.ndarray:
    """Every (receiver, ray, segment) reception of the chains (Sec. III-C).

    seg: [max_b, m, 8] segment rays (o, tmin, d, tmax), float32 or float64;
    hit_id, hit_t: [max_b, m] the segments' closest hits (id -1 = miss);
    receivers: [n_rx, 3] float64 field points; delta: angle in radians.
    Returns a RECEPTION array sorted by (rx, ray, order), keep = 0."""
    seg = np.asarray(seg)
    hit_id = np.asarray(hit_id)
    hit_t = np.asarray(hit_t)
    receivers = np.asarray(receivers, np.float64).reshape(-1, 3)
    max_b, m = hit_id.shape
    L = path_prefix(seg, hit_id, hit_t)
    rows = []
    for b in range(max_b):
        live = ~np.isnan(L[b])
        idx = np.nonzero(live)[0]
        if idx.size == 0:
            continue
        sb = seg[b, idx].astype(np.float64)
        o, d = sb[:, 0:3], sb[:, 4:7]
        t0 = sb[:, 3]
        t1 = np.where(hit_id[b, idx] >= 0, hit_t[b, idx].astype(np.float64), sb[:, 7])
        for r in range(receivers.shape[0]):
            ok, l, dist = segment_receives(o, d, t0, t1, L[b, idx], receivers[r], float(delta))
            k = np.nonzero(ok)[0]
            if k.size:
                rec = np.zeros(k.size, RECEPTION)
                rec["rx"] = r
                rec["ray"] = idx[k]
                rec["order"] = b
                rec["l"] = l[k]
                rec["dist"] = dist[k]
                rows.append(rec)
    out = np.concatenate(rows) if rows else np.zeros(0, RECEPTION)
    return np.sort(out, order=("rx", "ray", "order"))


def dedup(rec: np.ndarray, hit_id) -> np.ndarray:
    """Sets keep = 1 on one reception per (rx, order, facets hit before the
    segment): the smallest dist, then the smaller ray.  Returns a copy."""
    hit_id = np.asarray(hit_id)
    out = rec.copy()
    out["keep"] = 0
    best = {}
    for k in range(out.size):
        e = out[k]
        o = int(e["order"])
        key = (int(e["rx"]), o, tuple(int(x) for x in hit_id[:o, int(e["ray"])]))
        cand = (float(e["dist"]), int(e["ray"]))
        if key not in best or cand < best[key][0]:
            best[key] = (cand, k)
    for _, k in best.values():
        out["keep"][k] = 1
    return out

