"""Persistent launch shapes of the chain trace (GPU, through the C ABI).

rt_trace_ex with grid > 0 launches that many persistent work-groups, each
taking 64-ray batches from an atomic queue of the handle (Sec. III-B chains,
one per lane); with refill = 1 a wave tops up the lanes whose chains ended
with new rays at every segment (ballot + prefix count).  On the benchmark's
launch (city24k: 2,621,442 rays, <= 6 segments) in all three node formats:

* refill = 0 hands every wave the same 64 consecutive rays as the default
  launch, so hits, path lengths and hit counts are bit-identical to it;
* refill = 1 mixes chains of different rays in one wave.  A lane's result
  cannot depend on its neighbours except through the order in which the
  speculative traversal tests leaves, which can move the answer only where
  the hit is not decided by more than rounding: every chain must equal the
  default launch, or differ first at a segment whose checker margin is at
  most 1e-4 and whose answer passes the closest-hit rule (tests/_parity.py);
* a 100,000-chain sample of each persistent launch passes the closest-hit
  rule segment by segment against the checker re-tracing the GPU's own
  float32 segment rays.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import workloads

from _parity import check_differing, compare_hits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NTHREADS = min(16, os.cpu_count() or 1)
# work-groups of the one-wave trace kernel that fit at once (4 SIMDs x 7 waves
# of 72 registers per compute unit)
WAVES_PER_CU = 28


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def city():
    return workloads.city24k()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(out, pl, nh):
    torch.cuda.synchronize()
    return out.cpu().numpy(), pl.cpu().numpy(), nh.cpu().numpy()


def oracle_params(p):
    return oracle.SplitParams(alpha=p.alpha, src=p.src, max_leaf=p.max_leaf)


def check_sample(city, tree, seg, out, idx):
    """Every segment of the sampled chains against the checker's re-trace of
    the GPU's own segment ray (the facet just left is skipped)."""
    nb = city.max_bounces
    ids = out[:, idx, 0]
    t = out[:, idx, 1].view(np.float32).astype(np.float64)
    live = np.ones(idx.size, bool)
    prev = np.full(idx.size, -1, np.int32)
    counts = {"segments": 0, "clean": 0}
    for b in range(nb):
        k = np.nonzero(live)[0]
        if k.size == 0:
            break
        rays_b = seg[b, idx[k]]
        ref = oracle.trace_bvh(tree, rays_b, skip=prev[k], nthreads=NTHREADS)
        st = compare_hits(city.tris, rays_b, ids[b, k], t[b, k], ref, skip=prev[k])
        counts["segments"] += k.size
        counts["clean"] += st["clean"]
        prev[k] = ids[b, k]
        live[k[ids[b, k] < 0]] = False
    return counts


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_persistent_and_refill_launches(city, fmt):
    p = R.SplitParams(alpha=0.4, src=city.tx, node_format=fmt)
    bvh = R.BVH(dev(city.tris), p)
    rays = dev(city.rays)
    n, nb = city.n_rays, city.max_bounces
    base = host(*bvh.trace_bounces(rays, nb))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    resident = cus * WAVES_PER_CU
    tree = oracle.build_tree(city.tris, oracle_params(p))
    sample = np.sort(np.random.default_rng(3).choice(n, 100_000, replace=False))
    seg = torch.empty((nb, n, 8), dtype=torch.float32, device="cuda")
    for grid in (resident, 2 * resident):
        for refill in (0, 1):
            tag = f"{fmt} grid {grid} refill {refill}"
            log("launch:", tag)
            got = host(*bvh.trace_bounces(rays, nb, grid=grid, refill=refill))
            same = np.all(got[0] == base[0], axis=(0, 2)) & (got[2] == base[2]) & \
                (got[1].view(np.int64) == base[1].view(np.int64))
            differ = np.nonzero(~same)[0]
            log(f"{tag}: {differ.size} of {n} chains differ from the default launch")
            if refill == 0:
                assert differ.size == 0, tag
            elif differ.size:
                check_differing(city, tree, bvh, rays, nb, base, got, differ, tag)
            # the same launch again with the segment rays: sampled chains against the checker
            out, _, _ = bvh.trace_bounces(rays, nb, seg_rays=seg, grid=grid, refill=refill)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            if refill == 0:
                assert np.array_equal(o, base[0]), tag
            counts = check_sample(city, tree, seg.cpu().numpy(), o, sample)
            log(f"{tag}: sample {counts}")
            assert counts["clean"] > 0.99 * counts["segments"]
    bvh.close()
