"""Node formats at the edges of the box test's rounding argument (GPU,
through the C ABI).

The 4-wide formats cross box planes with one fused multiply-add on per-ray
offsets -o/d rounded outward, and the 8-bit nodes add a node term rounded
outward once per axis; both rely on the exact 8-bit decode enclosing each
child.  These cases stress that argument: scenes moved far from the origin
(large |o/d|), ray origins exactly on axis-aligned box planes, directions
with exact zero and tiny components.  Every format must follow the
closest-hit rule against brute force (tests/_parity.py), and the three
formats must return the same facet and the same t bits on every clean ray.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import icosphere, workloads

from _parity import compare_hits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


def plane_origins(tris, rng, count):
    """Points exactly on axis-aligned facets' planes, inside the facet's
    bounding rectangle (so some lie on edges and corners)."""
    t3 = tris.reshape(-1, 3, 3)
    out = []
    for f in rng.permutation(t3.shape[0]):
        v = t3[f]
        flat = [a for a in range(3) if v[0, a] == v[1, a] == v[2, a]]
        if not flat:
            continue
        a = flat[0]
        lo, hi = v.min(0), v.max(0)
        for _ in range(4):
            p = lo + (hi - lo) * rng.choice([0.0, 0.5, 1.0, rng.random()], size=3)
            p = p.astype(np.float32)
            p[a] = v[0, a]
            out.append(p)
        if len(out) >= count:
            break
    return np.array(out[:count], np.float32)


def directions(rng):
    d = icosphere.directions(4).astype(np.float64)          # includes exact zero components
    tiny = []
    for e in (1e-7, 1e-12, 1e-20):
        for axis in np.eye(3):
            for other in np.eye(3):
                if np.array_equal(axis, other):
                    continue
                for s in (1.0, -1.0):
                    tiny.append(s * axis + e * other * rng.choice([-1.0, 1.0]))
    d = np.concatenate([d, np.array(tiny), np.eye(3), -np.eye(3)])
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("offset", [(0.0, 0.0, 0.0), (1.0e5, 0.0, 0.0), (-3.0e4, 7.0e4, 0.0)])
def test_formats_agree_at_far_coordinates_and_plane_origins(offset):
    rng = np.random.default_rng(5)
    base = workloads.microcell()
    tris = (base.tris.reshape(-1, 3, 3) + np.array(offset, np.float32)).reshape(-1, 9)
    tris = np.ascontiguousarray(tris, np.float32)
    org = plane_origins(tris, rng, 120)
    dirs = directions(rng)
    o = np.repeat(org, dirs.shape[0], 0)
    d = np.tile(dirs, (org.shape[0], 1))
    rays = np.zeros((o.shape[0], 8), np.float32)
    rays[:, 0:3], rays[:, 3], rays[:, 4:7], rays[:, 7] = o, 1e-4, d, 500.0
    ref = oracle.brute(tris, rays, nthreads=NTHREADS)
    got = {}
    for fmt in ("bin2", "f4", "q4"):
        src = tuple(float(x) for x in np.array(offset) + np.array([0.0, 0.0, 10.0]))
        bvh = R.BVH(torch.from_numpy(tris).cuda(), R.SplitParams(alpha=0.4, src=src, node_format=fmt))
        out = bvh.trace(torch.from_numpy(rays).cuda()).cpu().numpy()
        gid, gt = out[:, 0], out[:, 1].view(np.float32)
        compare_hits(tris, rays, gid, gt, ref)
        got[fmt] = (gid, gt.view(np.uint32))
        bvh.close()
    clean = ref.margin > 1e-4
    assert clean.mean() > 0.5 and (ref.id >= 0).sum() > 1000
    for fmt in ("f4", "q4"):
        assert np.array_equal(got[fmt][0][clean], got["bin2"][0][clean]), fmt
        assert np.array_equal(got[fmt][1][clean], got["bin2"][1][clean]), fmt
