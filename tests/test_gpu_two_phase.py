"""Two-launch chain trace (rt_trace_opts.cut, GPU, through the C ABI).

The first launch traces every reflection chain's first `cut` segments (Sec.
III-B re-launch) and appends the chains still alive to the caller's
workspace (one atomic add per wave); the second launch traces them from
segment `cut` on, 64 per wave.  On
the benchmark's launch (city24k: 2,621,442 rays, <= 6 segments) in all three
node formats and for cut 1, 2 and 3:

* every chain's hits, path length and hit count equal the one-launch trace,
  or differ first at a segment whose checker margin is at most 1e-4 and
  whose answer passes the closest-hit rule (a wave's lanes are other chains
  than in the one-launch trace, which can change only the order in which the
  speculative traversal tests leaves; tests/_parity.py);
* the live count (the workspace's header) is exactly the number of chains
  with a hit in each of their first `cut` segments, and a second call with
  the same workspace gives the same results (the count restarts from zero
  every call);
* cut >= max_bounces is the one-launch trace, bit for bit;
* invalid workspaces and option mixes are refused with RT_EINVAL.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import workloads

from _parity import check_differing

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def differing(base, got):
    same = np.all(got[0] == base[0], axis=(0, 2)) & (got[2] == base[2]) & \
        (got[1].view(np.int64) == base[1].view(np.int64))
    return np.nonzero(~same)[0]


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_two_launches_equal_one_launch(city, fmt):
    p = R.SplitParams(alpha=0.4, src=city.tx, node_format=fmt)
    bvh = R.BVH(dev(city.tris), p)
    rays = dev(city.rays)
    n, nb = city.n_rays, city.max_bounces
    base = host(*bvh.trace_bounces(rays, nb))
    ws = R.chain_workspace(n)
    tree = oracle.build_tree(city.tris, oracle.SplitParams(alpha=p.alpha, src=p.src,
                                                           max_leaf=p.max_leaf))
    for cut in (1, 2, 3):
        tag = f"{fmt} cut {cut}"
        log("launch:", tag)
        got = host(*bvh.trace_bounces(rays, nb, cut=cut, chain_ws=ws))
        live = int(ws[:8].cpu().numpy().view(np.int64)[0])
        alive = int((got[2] >= cut).sum())  # chains with a hit in each of their first cut segments
        log(f"{tag}: {live} chains continued ({alive} with >= {cut} hits)")
        assert live == alive, tag
        differ = differing(base, got)
        log(f"{tag}: {differ.size} of {n} chains differ from the one-launch trace")
        if differ.size:
            check_differing(city, tree, bvh, rays, nb, base, got, differ, tag)
        again = host(*bvh.trace_bounces(rays, nb, cut=cut, chain_ws=ws))
        assert all(np.array_equal(x, y) for x, y in zip(got, again)), tag
    bvh.close()


def test_cut_at_or_past_the_last_segment_is_one_launch(city):
    p = R.SplitParams(alpha=0.4, src=city.tx)
    bvh = R.BVH(dev(city.tris), p)
    rays = dev(city.rays[: 200_000])
    base = host(*bvh.trace_bounces(rays, 3))
    ws = R.chain_workspace(rays.shape[0])
    for cut in (3, 7):
        got = host(*bvh.trace_bounces(rays, 3, cut=cut, chain_ws=ws))
        assert all(np.array_equal(x, y) for x, y in zip(base, got)), cut
    bvh.close()


def test_two_launch_arguments_are_checked(city):
    p = R.SplitParams(alpha=0.4, src=city.tx)
    bvh = R.BVH(dev(city.tris), p)
    n = 1000
    rays = dev(city.rays[:n])
    out = bvh.hits_buffer(n, 4)
    ws = R.chain_workspace(n)
    small = torch.empty(R.rt_trace_chain_ws_bytes(n) - 64, dtype=torch.uint8, device="cuda")
    seg = torch.empty((4, n, 8), dtype=torch.float32, device="cuda")
    bad = [dict(cut=-1, chain_ws=ws), dict(cut=2), dict(cut=2, chain_ws=small),
           dict(cut=2, chain_ws=ws[16:]), dict(cut=2, chain_ws=ws, grid=64),
           dict(cut=2, chain_ws=ws, seg_rays=seg), dict(cut=2, chain_ws=ws, lanes_per_ray=4)]
    for kw in bad:
        with pytest.raises(R.RtError) as e:
            R.rt_trace_ex(bvh.handle, rays, 4, out, **kw)
        assert e.value.code == R.RT_EINVAL, kw
    torch.cuda.synchronize()
    bvh.close()
