"""Pins of the CPU checker's energy stop rule (Sec. III-B: a chain ends when
its energy falls below a threshold) against closed forms: after hit j the
power ratio is prod(g) * k0 / l_j^2 with the path lengths of the image-source
constructions."""
import math

import numpy as np
import pytest

import oracle

from _scenes import corridor, ground_and_wall


def corridor_powers(w, nb, g_left, g_right, k0):
    """Zig-zag from (w/2, 0, 0) along (1, 0.5, 0): hit k (k = 1..) is on the
    right wall for odd k, path length (w/2 + (k - 1) w) sqrt(1.25)."""
    gain, out = 1.0, []
    for k in range(1, nb + 1):
        gain *= g_right if k % 2 else g_left
        l = (w / 2 + (k - 1) * w) * math.sqrt(1.25)
        out.append(gain * k0 / (l * l))
    return out


@pytest.mark.parametrize("g_left,g_right,k0", [(0.5, 0.25, 1.0), (0.9, 0.7, 1e-4), (1.0, 1.0, 3.0)])
def test_corridor_stop_point(g_left, g_right, k0):
    w, nb = 10.0, 8
    tris = corridor(width=w)
    material = np.array([0, 0, 1, 1], np.int32)           # facets 0-1: x = 0, 2-3: x = w
    refl = np.array([g_left, g_right])
    rays = np.array([[w / 2, 0, 0, 1e-4, 1, 0.5, 0, 1e3]], dtype=np.float32)
    P = corridor_powers(w, nb, g_left, g_right, k0)
    fixed = oracle.bounces(tris, rays, nb)
    for j in range(nb - 1):
        # a threshold between P[j + 1] and P[j]: the chain continues after hit
        # j + 1 (1-based) and stops after hit j + 2
        thr = math.sqrt(P[j] * P[j + 1]) if P[j + 1] < P[j] else P[j + 1] * 0.5
        ch, pw = oracle.bounces_energy(tris, rays, nb, material, refl, k0, thr)
        stop = next(k for k in range(nb) if P[k] < thr) + 1 if any(p < thr for p in P) else nb
        assert ch.n_hits[0] == stop, (j, ch.n_hits[0], stop)
        assert abs(pw[0] - P[stop - 1]) <= 1e-12 * P[stop - 1]
        assert np.array_equal(ch.id[:stop, 0], fixed.id[:stop, 0])
        assert np.all(ch.id[stop:, 0] == -1) and np.all(np.isnan(ch.seg[stop:, 0]))
        expect = (w / 2 + (stop - 1) * w) * math.sqrt(1.25)
        assert abs(ch.path_len[0] - expect) <= 1e-12 * expect


def test_ground_then_wall_two_materials():
    tris = ground_and_wall(wall_x=20.0)
    material = np.array([0, 0, 1, 1], np.int32)           # ground, wall
    refl = np.array([0.5, 0.1])
    k0 = 1e-3
    d = (np.float32([1, 0, -1]) / np.float32(np.sqrt(2))).astype(np.float32)
    rays = np.array([[0, 0, 10, 1e-4, d[0], d[1], d[2], 1e3]], dtype=np.float32)
    l1, l2 = 10 * math.sqrt(2), 20 * math.sqrt(2)
    p1, p2 = 0.5 * k0 / l1 ** 2, 0.05 * k0 / l2 ** 2
    ch, pw = oracle.bounces_energy(tris, rays, 4, material, refl, k0, (p1 + p2) / 2)
    assert ch.n_hits[0] == 2 and abs(pw[0] - p2) < 1e-9 * p2
    ch, pw = oracle.bounces_energy(tris, rays, 4, material, refl, k0, p1 * 1.01)
    assert ch.n_hits[0] == 1 and abs(pw[0] - p1) < 1e-9 * p1 and ch.id[1, 0] == -1
    ch, pw = oracle.bounces_energy(tris, rays, 4, material, refl, k0, p2 * 0.99)
    assert ch.n_hits[0] == 2                                # then it leaves the scene


def test_zero_threshold_equals_fixed_order_chains():
    tris = corridor(width=10.0)
    g = np.random.default_rng(0)
    rays = np.zeros((200, 8), np.float32)
    rays[:, 0] = g.uniform(1, 9, 200)
    rays[:, 3] = 1e-4
    rays[:, 4:7] = g.normal(size=(200, 3))
    rays[:, 7] = 1e3
    fixed = oracle.bounces(tris, rays, 6)
    ch, pw = oracle.bounces_energy(tris, rays, 6, np.zeros(4, np.int32), np.array([0.3]), 1.0, 0.0)
    for f in ("id", "t", "u", "v", "path_len", "n_hits"):
        assert np.array_equal(getattr(ch, f), getattr(fixed, f)), f
    assert np.all(pw[fixed.n_hits == 0] == 0) and np.all(pw[fixed.n_hits > 0] > 0)


def test_absorbing_or_unknown_material_stops_at_the_first_hit():
    tris = corridor(width=10.0)
    rays = np.array([[5, 0, 0, 1e-4, 1, 0.5, 0, 1e3]], dtype=np.float32)
    for mat in ([-1, -1, -1, -1], [0, 0, 5, 5]):
        ch, pw = oracle.bounces_energy(tris, rays, 6, np.array(mat, np.int32), np.array([0.5]),
                                       1.0, 1e-30)
        assert ch.n_hits[0] == 1 and pw[0] == 0.0
