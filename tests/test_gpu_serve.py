"""Serving on the GPU: a query's results through the continuous-batching
server are the same, bit for bit, as the same query traced alone, while
other batches share the device -- full hit records, and receptions for
queries with field points; a short Poisson stream reports latency."""
import sys
import time

import numpy as np
import pytest

import paper_2208_10008_amd as R
from paper_2208_10008_amd import serve
from rtgen import icosphere, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def scenes():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return serve.resident_scenes(range(3))


def test_device_rays_equal_host_rays(scenes):
    dirs = torch.from_numpy(icosphere.directions(9).astype(np.float32)).cuda()
    for tx, n in (((1.5, -20.25, 7.0), 1), ((300.1, 12.7, 33.3), 40_961), ((0.0, 0.0, 25.0), 999_999)):
        dev_rays = R.rt_rays_from_directions(dirs, n, tx, 1e-4, 2000.0).cpu().numpy()
        host = icosphere.make_rays(tx, icosphere.directions_n(n), 1e-4, 2000.0)
        assert np.array_equal(dev_rays.view(np.uint32), host.view(np.uint32))


def test_many_launch_rays_equal_one_launch_each(scenes):
    """rt_rays_from_directions_many: every valid record writes exactly the rays
    of rt_rays_from_directions into its rows; records past the table or with
    too many rays write nothing; rows no record covers keep their values."""
    dirs = torch.from_numpy(icosphere.directions(6).astype(np.float32)).cuda()
    launches = [((1.5, -2.0, 7.0), 0, 1000), ((300.0, 12.5, 33.0), 1000, 0),
                ((-5.0, 8.0, 2.5), 1000, 40_962), ((0.0, 0.0, 25.0), 41_962, 64),
                ((9.0, 9.0, 9.0), 42_100, 50_000),            # more rays than directions: skipped
                ((1.0, 2.0, 3.0), 42_200, 17)]                # runs past total: skipped
    total = 42_210
    table = np.zeros(len(launches), R.RAY_LAUNCH_DTYPE)
    for k, (src, first, n) in enumerate(launches):
        table[k] = (src, 0, first, n)
    rays = torch.full((total, 8), -3.0, dtype=torch.float32, device="cuda")
    R.rt_rays_from_directions_many(dirs, torch.from_numpy(table.view(np.uint8)).cuda(), 1e-4,
                                   2000.0, rays)
    got = rays.cpu().numpy()
    want = np.full((total, 8), -3.0, np.float32)
    for src, first, n in launches[:4]:
        if n:
            want[first:first + n] = R.rt_rays_from_directions(dirs, n, src, 1e-4, 2000.0).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_results_equal_alone_in_the_mix(scenes):
    """Stepped by hand: a first group of large queries (several ms on the
    device) is launched, a second mixed group is admitted into other slots
    right after, so both are on the device together; a third group follows
    through the running server."""
    rng = np.random.default_rng(11)
    ex = serve.GpuExecutor(scenes, slots=3, max_batch=4)
    srv = serve.Server(ex, budget_bytes=4 << 30, slots=3, max_batch=4)

    def query(n=None, nb=None):
        s = int(rng.integers(0, 3))
        tris, half = workloads.multiscene_scene(s)
        tx = tuple(float(x) for x in (rng.uniform(-0.4, 0.4) * half, rng.uniform(-0.4, 0.4) * half,
                                      rng.uniform(5, 40)))
        n = n or int(round(10 ** rng.uniform(3.0, 5.3)))
        nb = nb or int(rng.integers(1, 7))
        return srv.submit(s, nb, tx=tx, n_rays=n)
    reqs = [query(1_000_000, 6) for _ in range(4)]
    srv.step()                                  # first group on the device
    reqs += [query() for _ in range(6)]
    srv.step()                                  # admitted while the first group runs
    assert srv.max_running >= 2, "the second group did not overlap the first"
    srv.start()
    for _ in range(6):
        reqs.append(query())
        time.sleep(float(rng.uniform(0.0, 0.004)))
    while not srv.idle():
        time.sleep(1e-3)
    srv.stop()
    m = srv.metrics()
    log("mix:", m)
    assert m["queries"] == len(reqs) and m["failed"] == 0
    for r in reqs:
        assert r.status == serve.DONE
        rays = torch.from_numpy(icosphere.make_rays(r.tx, icosphere.directions_n(r.n_rays),
                                                    1e-4, 2000.0)).cuda()
        out, pl, nh = scenes[r.scene].trace_bounces(rays, r.max_bounces)
        assert np.array_equal(out.cpu().numpy(), r.out), f"query {r.rid}: hits differ"
        assert np.array_equal(pl.cpu().numpy(), r.path_len), f"query {r.rid}: path lengths differ"
        assert np.array_equal(nh.cpu().numpy(), r.n_hits), f"query {r.rid}: hit counts differ"
        assert r.segments == serve.count_segments(r), f"query {r.rid}: device segment count"


def test_short_poisson_stream(scenes):
    stream = serve.poisson_queries(duration=1.5, rate=150.0, seed=4, scenes=range(3))
    srv = serve.Server(serve.GpuExecutor(scenes, slots=4, max_batch=16), budget_bytes=4 << 30,
                       slots=4, max_batch=16)
    serve.run_stream(srv, stream)
    m = srv.metrics()
    log("poisson:", m)
    assert m["queries"] == len(stream) and m["failed"] == 0
    assert 0 < m["latency_ms_p50"] <= m["latency_ms_p99"] < 5000
    assert m["mrays_s"] > 0


def test_reception_queries_equal_alone_in_the_mix(scenes):
    """Queries with field points come back as reception records and hit
    counts only; each equals the fused reception trace of the same rays run
    alone (same count, same records bit for bit), while plain queries share
    the slots."""
    rng = np.random.default_rng(23)
    ex = serve.GpuExecutor(scenes, slots=3, max_batch=4)
    srv = serve.Server(ex, budget_bytes=4 << 30, slots=3, max_batch=4)
    stream = serve.poisson_queries(duration=0.2, rate=60.0, seed=9, scenes=range(3), receivers=24,
                                   rec_cap=1 << 16)
    assert len(stream) >= 6
    reqs = []
    for k, (_, s, tx, n, nb, extra) in enumerate(stream):
        reqs.append(srv.submit(s, nb, tx=tx, n_rays=n, **extra))
        if k % 2 == 0:                      # plain queries in between
            reqs.append(srv.submit(s, nb, tx=tx, n_rays=int(rng.integers(1000, 50_000))))
        srv.step()
    srv.run_until_idle()
    got_recv = 0
    for r in reqs:
        assert r.status == serve.DONE, r.error
        if r.receivers is None:
            assert r.out is not None and r.receptions is None
            continue
        assert r.out is None and r.n_receptions >= 0
        rays = torch.from_numpy(icosphere.make_rays(r.tx, icosphere.directions_n(r.n_rays),
                                                    1e-4, 2000.0)).cuda()
        rcv = R.Receivers(torch.from_numpy(r.receivers).cuda(), r.delta, r.rec_cap)
        _, _, nh = scenes[r.scene].trace_receive(rays, r.max_bounces, rcv)
        assert r.n_receptions == rcv.count(), f"query {r.rid}: reception count differs"
        assert r.n_receptions <= r.rec_cap   # every record stored: the set is deterministic
        assert np.array_equal(np.sort(r.receptions, order=("rx", "ray", "order")),
                              np.sort(rcv.records(), order=("rx", "ray", "order"))), r.rid
        assert np.array_equal(nh.cpu().numpy(), r.n_hits), f"query {r.rid}: hit counts differ"
        assert r.segments == serve.count_segments(r), f"query {r.rid}: device segment count"
        got_recv += r.n_receptions
    log("receptions through the server:", got_recv)
    assert got_recv > 0
