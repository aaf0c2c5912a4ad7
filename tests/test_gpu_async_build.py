"""Asynchronous rebuild (rt_rebuild_async + rt_bvh_wait, GPU, through the C
ABI).

rt_rebuild_async queues the same Eq. (2) build as rt_rebuild (Sec. II-B,
II-C) and returns; rt_bvh_wait reads the build's record and makes the tree
usable.  Checked:

* the tree after rt_bvh_wait equals the synchronous build's byte for byte
  (binary nodes and facet order, traversal nodes of every format), and its
  info matches; until then the handle is refused (RT_EINVAL) and reports
  n_tris = 0;
* an error found on the device (a non-finite vertex) comes back from
  rt_bvh_wait, the handle stays refused, and a valid rebuild restores it;
  an argument error comes back at once, with the same effect;
* two handles driven as a transmitter sweep that queues the next build before
  waiting for the current one (builds on one stream, traces on another,
  ordered by events) give every step the hits, path lengths and hit counts
  of a synchronous build and trace of the same transmitter.
"""
import numpy as np
import pytest

import paper_2208_10008_amd as R
from rtgen import icosphere, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def city():
    return workloads.city24k(level=7)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def reachable(raw, fmt):
    """The traversal records reachable from node 0, depth first (a wide-node
    array also has slots no traversal reads, which keep older contents)."""
    rec = {"bin2": 64, "f4": 128, "q4": 64}[fmt]
    w = raw.view(np.int32).reshape(-1, rec // 4)
    seen, stack, parts = set(), [0], []
    while stack:
        k = stack.pop()
        if k in seen:
            continue
        seen.add(k)
        parts.append(raw[k * rec:(k + 1) * rec].tobytes())
        if fmt == "bin2":
            refs, m = [int(w[k, 12]), int(w[k, 13])], 3
        elif fmt == "f4":
            refs, m = [int(x) for x in w[k, 24:28]], int(w[k, 28])
        else:
            refs, m = [int(x) for x in w[k, 12:16]], (int(w[k, 3]) >> 24) & 0xF
        stack += [r for c, r in enumerate(refs) if (m >> c) & 1 and r >= 0]
    return b"".join(parts)


def tree_bytes(bvh):
    nodes, perm = bvh.download()
    return nodes.tobytes(), perm.tobytes(), reachable(bvh.trace_nodes(), bvh.params.node_format)


INFO_FIELDS = ("n_tris", "n_nodes", "n_internal", "n_leaves", "depth", "n_levels", "node_format",
               "n_trace_nodes", "trace_bytes")


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_async_rebuild_equals_the_synchronous_build(city, fmt):
    tris = dev(city.tris)
    p = R.SplitParams(alpha=0.4, src=city.tx, node_format=fmt)
    ref = R.BVH(tris, p)
    want = tree_bytes(ref)
    # a handle holding another tree first (traditional split), rebuilt asynchronously
    b = R.BVH(tris, R.SplitParams(alpha=1.0, src=city.tx, node_format=fmt))
    s = torch.cuda.Stream()
    b.rebuild_async(tris, p, stream=s)
    assert b.info().n_tris == 0
    with pytest.raises(R.RtError):
        b.trace(dev(city.rays[:64]))
    b.wait()
    b.wait()  # no build in flight: returns at once
    assert tree_bytes(b) == want
    bi, ri = b.info(), ref.info()
    for f in INFO_FIELDS:
        assert getattr(bi, f) == getattr(ri, f), f
    rays = dev(city.rays)
    assert torch.equal(b.trace(rays), ref.trace(rays))
    # a synchronous rebuild queued behind an asynchronous one ends it first
    b.rebuild_async(tris, R.SplitParams(alpha=1.0, src=city.tx, node_format=fmt), stream=s)
    b.rebuild(tris, p)
    assert tree_bytes(b) == want
    b.close()
    ref.close()


def test_device_error_comes_back_from_wait(city):
    tris = city.tris.copy()
    bad = tris.copy()
    bad[5, 4] = np.nan
    p = R.SplitParams(alpha=0.4, src=city.tx)
    b = R.BVH(dev(tris), p)
    bad_d = dev(bad)
    b.rebuild_async(bad_d, p)        # the vertex check runs on the device
    with pytest.raises(R.RtError):
        b.wait()
    assert b.info().n_tris == 0
    with pytest.raises(R.RtError):
        b.trace(dev(city.rays[:64]))
    b.rebuild(dev(tris), p)
    assert b.info().n_tris == tris.shape[0]
    b.close()


def test_argument_errors_return_at_once(city):
    """An argument rt_rebuild refuses is refused by rt_rebuild_async before
    anything is queued; the handle is then unusable (as after a failed
    rt_rebuild) until a valid rebuild, synchronous or not."""
    tris = dev(city.tris)
    p = R.SplitParams(alpha=0.4, src=city.tx)
    b = R.BVH(tris, p)
    with pytest.raises(R.RtError):
        b.rebuild_async(tris, R.SplitParams(alpha=0.4, src=city.tx, max_leaf=0))
    assert b.info().n_tris == 0
    b.wait()                         # nothing in flight
    with pytest.raises(R.RtError):
        b.trace(dev(city.rays[:64]))
    b.rebuild_async(tris, p)
    b.wait()
    assert b.info().n_tris == city.tris.shape[0]
    b.close()


def test_pipelined_sweep_matches_synchronous_steps(city):
    """Steps k = 0..7 move the transmitter; step k builds tree k mod 2
    asynchronously on the build stream while step k - 1's rays are traced on
    the trace stream, the next build queued before waiting for the current."""
    tris = dev(city.tris)
    nb = city.max_bounces
    txs = [(40.0 * k - 140.0, 15.0 * (k % 3), 25.0) for k in range(8)]
    dirs = icosphere.directions(7)
    rays = [dev(icosphere.make_rays(tx, dirs, 1e-4, 2000.0)) for tx in txs]
    n = rays[0].shape[0]
    params = [R.SplitParams(alpha=0.4, src=tx, node_format="f4") for tx in txs]
    trees = [R.BVH(tris, params[0]), R.BVH(tris, params[1])]
    sb, st = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [(torch.empty((nb, n, 4), dtype=torch.int32, device="cuda"),
             torch.empty(n, dtype=torch.float64, device="cuda"),
             torch.empty(n, dtype=torch.int32, device="cuda")) for _ in txs]
    done = [torch.cuda.Event(), torch.cuda.Event()]
    built = [torch.cuda.Event(), torch.cuda.Event()]

    def queue_build(k):
        i = k % 2
        sb.wait_event(done[i])     # tree i's previous trace has finished
        trees[i].rebuild_async(tris, params[k], stream=sb)
        built[i].record(sb)

    queue_build(0)
    for k in range(len(txs)):
        i = k % 2
        if k + 1 < len(txs):
            queue_build(k + 1)     # queued before this step's build is waited for
        trees[i].wait()
        st.wait_event(built[i])
        R.rt_trace_bounces(trees[i].handle, rays[k], nb, *outs[k], stream=st)
        done[i].record(st)
    torch.cuda.synchronize()
    ref = R.BVH(tris, params[0])
    for k in range(len(txs)):
        ref.rebuild(tris, params[k])
        o, pl, nh = (torch.empty_like(t) for t in outs[k])
        R.rt_trace_bounces(ref.handle, rays[k], nb, o, pl, nh)
        torch.cuda.synchronize()
        assert torch.equal(o, outs[k][0]), k
        assert torch.equal(pl, outs[k][1]), k
        assert torch.equal(nh, outs[k][2]), k
    ref.close()
    for t in trees:
        t.close()
