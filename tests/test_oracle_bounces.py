"""Pins of the CPU checker's reflection chains (Sec. III-B: reflected rays
until the set order) against image-source closed forms."""
import numpy as np

import oracle

from _scenes import corridor, ground_and_wall


def test_ground_then_wall_image_source():
    tris = ground_and_wall(wall_x=20.0)
    d = (np.float32([1, 0, -1]) / np.float32(np.sqrt(2))).astype(np.float32)
    rays = np.array([[0, 0, 10, 1e-4, d[0], d[1], d[2], 1e3]], dtype=np.float32)
    for tree in (None, oracle.build_tree(tris, oracle.SplitParams(max_leaf=1))):
        c = oracle.bounces(tris, rays, 4, tree=tree)
        assert c.n_hits[0] == 2
        assert c.id[0, 0] in (0, 1) and c.id[1, 0] in (2, 3) and c.id[2, 0] == -1
        dx, dz = float(d[0]), float(d[2])
        norm = np.sqrt(dx * dx + dz * dz)
        # ground at t = 10/|dz|, wall at t = 10/dx; the reflected direction
        # keeps |d|; the image of the source in the ground is (0, 0, -10)
        assert abs(c.t[0, 0] - 10 / abs(dz)) < 1e-13 and abs(c.t[1, 0] - 10 / dx) < 1e-12
        expect = (10 / abs(dz) + 10 / dx) * norm
        assert abs(c.path_len[0] - expect) < 1e-12 * expect
        assert abs(c.path_len[0] - np.hypot(20, 20)) < 1e-5
        np.testing.assert_allclose(c.seg[1, 0, 0:3], [10, 0, 0], atol=1e-12)
        np.testing.assert_allclose(c.seg[2, 0, 0:3], [20, 0, 10], atol=1e-12)
        np.testing.assert_allclose(c.seg[2, 0, 4:7], [-dx, 0, -dz], atol=1e-15)


def test_corridor_zigzag():
    w = 10.0
    tris = corridor(width=w)
    rays = np.array([[5, 0, 0, 1e-4, 1, 0.5, 0, 1e3]], dtype=np.float32)
    nb = 6
    c = oracle.bounces(tris, rays, nb)
    assert c.n_hits[0] == nb
    # horizontal run w/2 then w per hit, |d| / |dx| = sqrt(1.25)
    expect = (w / 2 + (nb - 1) * w) * np.sqrt(1.25)
    assert abs(c.path_len[0] - expect) < 1e-12 * expect
    ys = c.seg[1:, 0, 1]
    np.testing.assert_allclose(ys, [2.5 + 5 * k for k in range(nb - 1)], atol=1e-12)
    walls = c.id[:, 0] // 2
    assert list(walls) == [1, 0, 1, 0, 1, 0]


def test_miss_stops_chain():
    tris = corridor()
    rays = np.array([[5, 0, 0, 1e-4, 0, 1, 0, 1e3]], dtype=np.float32)   # parallel to both walls
    c = oracle.bounces(tris, rays, 3)
    assert c.n_hits[0] == 0 and c.path_len[0] == 0.0 and np.all(c.id[:, 0] == -1)
    assert np.all(np.isnan(c.seg[1:, 0]))


def test_tmax_per_segment():
    tris = corridor(width=10.0)
    # tmax bounds the ray parameter t of every segment: the first needs t = 5,
    # every later one t = 10, so tmax = 9 ends the chain after one hit
    rays = np.array([[5, 0, 0, 1e-4, 1, 0.5, 0, 9.0]], dtype=np.float32)
    c = oracle.bounces(tris, rays, 4)
    assert c.n_hits[0] == 1


def _float32_chain(tris, tree, rays, nb):
    """Chains whose re-launched rays are rounded to float32, as the GPU stores
    them: origin fl32(o + t d) and direction fl32(reflected d), every segment
    the checker's exact closest hit of that float32 ray."""
    v = tris.astype(np.float64).reshape(-1, 3, 3)
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    m = rays.shape[0]
    ids = np.full((nb, m), -1, np.int32)
    ts = np.full((nb, m), np.inf)
    cur = rays.astype(np.float32).copy()
    prev = np.full(m, -1, np.int32)
    live = np.ones(m, bool)
    for b in range(nb):
        k = np.nonzero(live)[0]
        if k.size == 0:
            break
        ref = oracle.trace_bvh(tree, cur[k], skip=prev[k], nthreads=8)
        ids[b, k], ts[b, k] = ref.id, ref.t
        hit = ref.id >= 0
        kh, idh, th = k[hit], ref.id[hit], ref.t[hit]
        o = cur[kh, 0:3].astype(np.float64)
        d = cur[kh, 4:7].astype(np.float64)
        n = nrm[idh]
        r = d - (2 * np.einsum("ij,ij->i", d, n) / np.einsum("ij,ij->i", n, n))[:, None] * n
        cur[kh, 0:3] = (o + th[:, None] * d).astype(np.float32)
        cur[kh, 4:7] = r.astype(np.float32)
        prev[kh] = idh
        live[k[~hit]] = False
    return ids, ts


def test_float32_chain_error_model():
    """The error model the GPU chains are gated with (tests/_parity.py,
    chain_error_bounds): float32-rounded re-launched rays traced exactly must
    stay within it of the float64 chains on every compared segment of a
    100,000-ray sample of the city launch, while the segment tolerance alone
    (1e-5 relative) is exceeded on some of them, so the propagated term is
    needed."""
    from _parity import chain_error_bounds
    from rtgen import workloads
    w = workloads.city24k()
    rays = w.rays[np.sort(np.random.default_rng(7).choice(w.n_rays, 100_000, replace=False))]
    tree = oracle.build_tree(w.tris, oracle.SplitParams(alpha=0.4, src=w.tx))
    nb = w.max_bounces
    ch = oracle.bounces(w.tris, rays, nb, tree=tree, nthreads=8)
    ids32, t32 = _float32_chain(w.tris, tree, rays, nb)
    allowed = chain_error_bounds(w.tris, ch.seg, ch.id, ch.t)
    ok = np.ones(rays.shape[0], bool)
    worst, over_segment_tol, compared = 0.0, 0, 0
    for b in range(nb):
        m = ok & (ch.margin[b] > 1e-4)
        assert np.array_equal(ids32[b, m], ch.id[b, m]), b
        hit = m & (ch.id[b] >= 0)
        dt = np.abs(t32[b, hit] - ch.t[b, hit])
        assert np.all(dt <= allowed[b, hit]), b
        if dt.size:
            worst = max(worst, float((dt / allowed[b, hit]).max()))
            over_segment_tol += int(np.sum(dt > 1e-5 * ch.t[b, hit]))
        compared += int(hit.sum())
        ok = m & (ch.id[b] >= 0)
    print("float32 chains: %d hits compared, worst deviation / bound %.3f, %d over 1e-5 "
          "relative" % (compared, worst, over_segment_tol))
    assert compared > 50_000 and over_segment_tol > 0
