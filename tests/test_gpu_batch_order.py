"""Batch dispatch order and split compute units (GPU, through the C ABI).

rt_rays_batch_order ranks the rays' batches of 64 by how close their
directions lie to the plane normal to an axis; rt_trace_opts.batch_order makes
the launch start its batches in a given order; rt_streams_split_cus gives two
streams disjoint compute units.  None of them may change a result:

* the batch keys equal the same float32 arithmetic done on the host, bit for
  bit, and the order equals the host's stable ordering by class, a
  permutation (ragged last batches, a single ray, zero and non-finite
  directions, one tile of 1024 batches and several, every axis);
* on the benchmark's launch (city24k: 2,621,442 rays, <= 6 segments) in all
  three node formats, the traces started in the library's order, in a random
  order and in reverse order equal the default launch bit for bit, with and
  without miss padding; with cut 2 (the order applies to the first launch)
  they are held to the one-launch trace as the two-launch tests are;
* an order entry outside the batches leaves that batch's rows untouched, a
  repeated entry changes nothing, and batch_order with grid > 0, with more
  than one lane per ray or misaligned is refused;
* a build on the small stream and a trace on the large one give the default
  stream's tree and chains.
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


def host_keys(rays, axis):
    """The batch keys in the kernel's float32 arithmetic (each operation
    rounded): the smallest q among each batch's rays."""
    d = np.ascontiguousarray(rays[:, 4:7], dtype=np.float32)
    n = d.shape[0]
    with np.errstate(all="ignore"):
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        da = d[:, axis]
        t = (da * da) / d2
        valid = (d2 > 0) & np.isfinite(d2)
        q = np.zeros(n, np.int64)
        q[valid] = np.clip(np.floor(np.float32(1023) * t[valid]).astype(np.int64), 0, 1023)
    q = np.concatenate([q, np.full((-n) % 64, 1023, np.int64)])
    return q.reshape(-1, 64).min(axis=1)


def host_order(keys):
    """Stable order of the batches by class (|d_a| / |d| in sixteenths)."""
    thr = np.array([(1023 * k * k) // 256 for k in range(1, 16)])
    cls = (keys[:, None] >= thr[None, :]).sum(axis=1)
    return np.argsort(cls, kind="stable"), cls


def check_order(rays_np, axis):
    n = rays_np.shape[0]
    nb = (n + 63) // 64
    rays = dev(rays_np)
    keys = torch.full((R.rt_rays_batch_order_ws_bytes(n) // 4,), -7, dtype=torch.int32, device="cuda")
    order = R.rt_rays_batch_order(rays, axis=axis, keys=keys)
    torch.cuda.synchronize()
    o, k = order.cpu().numpy(), keys.cpu().numpy()[:nb]
    ref = host_keys(rays_np, axis)
    assert np.array_equal(k, ref), (axis, np.nonzero(k != ref)[0][:5])
    ref_o, cls = host_order(ref)
    assert np.array_equal(o, ref_o), (axis, np.nonzero(o != ref_o)[0][:5])
    assert np.array_equal(np.sort(o), np.arange(nb)) and np.all(np.diff(cls[o]) >= 0)
    return o


def test_batch_order_keys_and_permutation(city):
    for axis in (0, 1, 2):
        o = check_order(city.rays, axis)
        log(f"axis {axis}: {o.size} batches, first {o[:4]}")
    rng = np.random.default_rng(5)
    for n in (1, 17, 63, 64, 65, 1000, 4097, 65_536, 65_537, 200_000):
        r = np.zeros((n, 8), np.float32)
        r[:, 4:7] = rng.normal(size=(n, 3)).astype(np.float32)
        r[:, 7] = 1.0
        if n > 40:
            r[0, 4:7] = 0.0              # zero direction
            r[16, 4:7] = (np.nan, 1.0, 0.0)
            r[32, 4:7] = (np.inf, 0.0, 0.0)
            r[48, 4:7] = (0.0, 0.0, -1e-30)  # tiny: d2 underflows to 0
        check_order(r, 2)


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_ordered_launch_equals_default(city, fmt):
    p = R.SplitParams(alpha=0.4, src=city.tx, node_format=fmt)
    bvh = R.BVH(dev(city.tris), p)
    rays = dev(city.rays)
    n, nb = city.n_rays, city.max_bounces
    nbat = (n + 63) // 64
    base = host(*bvh.trace_bounces(rays, nb))
    orders = {"library": R.rt_rays_batch_order(rays),
              "random": dev(np.random.default_rng(1).permutation(nbat).astype(np.int32)),
              "reverse": dev(np.arange(nbat, dtype=np.int32)[::-1].copy())}
    for name, order in orders.items():
        got = host(*bvh.trace_bounces(rays, nb, batch_order=order))
        assert all(np.array_equal(x, y) for x, y in zip(base, got)), (fmt, name)
        out = bvh.hits_buffer(n, nb)
        out.fill_(SENTINEL)
        got = host(*bvh.trace_bounces(rays, nb, out=out, pad=False, batch_order=order))
        assert np.array_equal(got[2], base[2]) and np.array_equal(got[1], base[1]), (fmt, name)
        last = np.minimum(got[2], nb - 1)
        rows = np.arange(nb)[:, None] <= last[None, :]
        assert np.array_equal(got[0][rows], base[0][rows]), (fmt, name)
        assert (got[0][~rows] == SENTINEL).all(), (fmt, name)
        log(f"{fmt} {name}: equal to the default launch")
    ws = R.chain_workspace(n)
    got = host(*bvh.trace_bounces(rays, nb, cut=2, chain_ws=ws, batch_order=orders["library"]))
    same = np.all(got[0] == base[0], axis=(0, 2)) & (got[2] == base[2]) & \
        (got[1].view(np.int64) == base[1].view(np.int64))
    differ = np.nonzero(~same)[0]
    log(f"{fmt} cut 2 ordered: {differ.size} chains differ from the one-launch trace")
    if differ.size:
        tree = oracle.build_tree(city.tris, oracle.SplitParams(alpha=p.alpha, src=p.src,
                                                               max_leaf=p.max_leaf))
        check_differing(city, tree, bvh, rays, nb, base, got, differ, f"{fmt} cut 2 ordered")
    bvh.close()


def test_order_entries_outside_and_repeated(city):
    p = R.SplitParams(alpha=0.4, src=city.tx)
    bvh = R.BVH(dev(city.tris), p)
    n = 10_000
    rays = dev(city.rays[:n])
    nbat = (n + 63) // 64
    base = host(*bvh.trace_bounces(rays, 4))
    perm = np.random.default_rng(2).permutation(nbat).astype(np.int32)
    skipped = int(perm[3])
    bad = perm.copy()
    bad[3] = -1
    bad[7] = nbat + 5
    skipped2 = int(perm[7])
    out = bvh.hits_buffer(n, 4)
    out.fill_(SENTINEL)
    pl = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    nh = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    got = host(*bvh.trace_bounces(rays, 4, out=out, path_len=pl, n_hits=nh, batch_order=dev(bad)))
    batch = np.arange(n) // 64
    untouched = (batch == skipped) | (batch == skipped2)
    assert (got[0][:, untouched] == SENTINEL).all() and (got[2][untouched] == -9).all()
    assert np.array_equal(got[0][:, ~untouched], base[0][:, ~untouched])
    assert np.array_equal(got[2][~untouched], base[2][~untouched])
    rep = perm.copy()
    rep[5] = rep[4]  # batch perm[4] twice, batch perm[5] not at all
    out.fill_(SENTINEL)
    got = host(*bvh.trace_bounces(rays, 4, out=out, batch_order=dev(rep)))
    twice = batch == perm[4]
    assert np.array_equal(got[0][:, twice], base[0][:, twice])
    bvh.close()


def test_batch_order_arguments_are_checked(city):
    p = R.SplitParams(alpha=0.4, src=city.tx)
    bvh = R.BVH(dev(city.tris), p)
    n = 1000
    rays = dev(city.rays[:n])
    out = bvh.hits_buffer(n, 4)
    order = R.rt_rays_batch_order(rays)
    raw = torch.zeros(4 * order.numel() + 8, dtype=torch.uint8, device="cuda")
    odd = raw[1:1 + 4 * order.numel()].view(torch.uint8)
    for kw in (dict(batch_order=order, grid=64), dict(batch_order=order, lanes_per_ray=4)):
        with pytest.raises(R.RtError) as e:
            R.rt_trace_ex(bvh.handle, rays, 4, out, **kw)
        assert e.value.code == R.RT_EINVAL, kw
    with pytest.raises(R.RtError) as e:
        R.rt_trace_ex(bvh.handle, rays, 4, out, batch_order=odd)
    assert e.value.code == R.RT_EINVAL
    with pytest.raises(R.RtError) as e:
        R.rt_rays_batch_order(rays, axis=3)
    assert e.value.code == R.RT_EINVAL
    torch.cuda.synchronize()
    bvh.close()


def test_split_streams_give_the_same_results(city):
    for k in (0, 12, 136):
        with pytest.raises(R.RtError) as e:
            R.SplitStreams(k)
        assert e.value.code == R.RT_EINVAL, k
    p = R.SplitParams(alpha=0.4, src=city.tx)
    tris = dev(city.tris)
    rays = dev(city.rays[:300_000])
    ref = R.BVH(tris, p)
    base = host(*ref.trace_bounces(rays, 6))
    ss = R.SplitStreams(32)
    bvh = R.BVH(tris, p, stream=ss.small)
    R.rt_rebuild(bvh.handle, tris, p, stream=ss.small)
    ss.large.wait_stream(ss.small)
    got = host(*bvh.trace_bounces(rays, 6, stream=ss.large,
                                  batch_order=R.rt_rays_batch_order(rays, stream=ss.large)))
    assert all(np.array_equal(x, y) for x, y in zip(base, got))
    assert np.array_equal(ref.download()[0], bvh.download()[0])
    ss.close()
    ref.close()
    bvh.close()
