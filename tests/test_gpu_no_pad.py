"""Trace without miss padding (rt_trace_opts.flags = RT_TRACE_NO_PAD, GPU,
through the C ABI).

A reflection chain ends at its first miss (Sec. III-B); by default the rows of
the hit array after that miss are written as misses too.  With the flag they
are left as they were, and n_hits tells where each chain ends.  On the
benchmark's launch (city24k: 2,621,442 rays, <= 6 segments) in all three node
formats, with the output pre-filled with a sentinel:

* rows 0 .. min(h, max_bounces - 1) of a chain with h hits, its path length
  and its hit count are those of the padded trace of the same launch shape,
  bit for bit for one launch (64 rays or 16 rays per wave) and for persistent
  work-groups taking 64 consecutive rays; with lane refill and under the
  two-launch trace (cut 2) they equal the one-launch trace or differ only as
  tests/_parity.py allows;
* every later row still holds the sentinel;
* the flag without n_hits, and unknown flag bits, are refused with RT_EINVAL.
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

SENTINEL = 0x5A5A5A5A
WAVES_PER_CU = 28  # resident trace waves per compute unit (7 per SIMD)


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


def split_rows(got, nb):
    """(written, untouched) row masks, shape (nb, n), from each chain's hit count."""
    last = np.minimum(got[2], nb - 1)
    q = np.arange(nb)[:, None]
    return q <= last[None, :], q > last[None, :]


def padded(got, base, written):
    """got with its unwritten rows replaced by the miss record the padded trace
    writes there (every padded row after a miss holds the same record)."""
    nb = got[0].shape[0]
    pad_rows = ~split_rows(base, nb)[0]
    assert pad_rows.any()
    miss = base[0][pad_rows]
    assert (miss == miss[0]).all(), "padded rows hold one miss record"
    out = got[0].copy()
    out[~written] = miss[0]
    return out, got[1], got[2]


def differing(base, got):
    same = np.all(got[0] == base[0], axis=(0, 2)) & (got[2] == base[2]) & \
        (got[1].view(np.int64) == base[1].view(np.int64))
    return np.nonzero(~same)[0]


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_no_pad_writes_only_the_traced_rows(city, fmt):
    p = R.SplitParams(alpha=0.4, src=city.tx, node_format=fmt)
    bvh = R.BVH(dev(city.tris), p)
    rays = dev(city.rays)
    n, nb = city.n_rays, city.max_bounces
    ws = R.chain_workspace(n)
    tree = None
    one = host(*bvh.trace_bounces(rays, nb))
    resident = torch.cuda.get_device_properties(0).multi_processor_count * WAVES_PER_CU
    shapes = (dict(), dict(lanes_per_ray=4), dict(grid=resident, refill=0),
              dict(grid=resident, refill=1), dict(cut=2, chain_ws=ws))
    for kw in shapes:
        tag = f"{fmt} " + (", ".join(f"{k} {v}" for k, v in kw.items() if k != "chain_ws") or "default")
        log("launch:", tag)
        # launches that regroup chains (lane refill, two launches) are held to
        # the one-launch trace, as without the flag
        regroup = "cut" in kw or kw.get("refill") == 1
        base = one if regroup else host(*bvh.trace_bounces(rays, nb, **kw))
        out = bvh.hits_buffer(n, nb)
        out.fill_(SENTINEL)
        got = host(*bvh.trace_bounces(rays, nb, out=out, pad=False, **kw))
        written, untouched = split_rows(got, nb)
        assert (got[0][untouched] == SENTINEL).all(), tag
        assert not (got[0][written] == SENTINEL).all(axis=-1).any(), tag
        log(f"{tag}: {int(untouched.sum())} of {nb * n} rows left untouched")
        full = padded(got, base, written)
        differ = differing(base, full)
        if not regroup:
            assert differ.size == 0, tag
        elif differ.size:
            log(f"{tag}: {differ.size} of {n} chains differ from the one-launch trace")
            if tree is None:
                tree = oracle.build_tree(city.tris, oracle.SplitParams(
                    alpha=p.alpha, src=p.src, max_leaf=p.max_leaf))
            check_differing(city, tree, bvh, rays, nb, base, full, differ, tag)
    bvh.close()


def test_no_pad_arguments_are_checked(city):
    p = R.SplitParams(alpha=0.4, src=city.tx)
    bvh = R.BVH(dev(city.tris), p)
    n = 1000
    rays = dev(city.rays[:n])
    out = bvh.hits_buffer(n, 4)
    pl = torch.empty(n, dtype=torch.float64, device="cuda")
    nh = torch.empty(n, dtype=torch.int32, device="cuda")
    for kw in (dict(flags=R.RT_TRACE_NO_PAD), dict(flags=2, n_hits=nh),
               dict(flags=R.RT_TRACE_NO_PAD | 4, n_hits=nh)):
        with pytest.raises(R.RtError) as e:
            R.rt_trace_ex(bvh.handle, rays, 4, out, path_len=pl, **kw)
        assert e.value.code == R.RT_EINVAL, kw
    torch.cuda.synchronize()
    bvh.close()
