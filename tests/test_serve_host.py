"""Serving loop policy on the host (no GPU): admission by memory budget and
free slots in arrival order, malformed and oversize queries, cancellation,
and overlapping batches.  The device is replaced by a host stand-in that
finishes a batch after a set number of polls."""
import numpy as np
import pytest

from paper_2208_10008_amd.serve import (CANCELLED, DONE, FAILED, Request, Scheduler, Server,
                                        check_request)


class HostExecutor:
    def __init__(self, scenes=(0, 1, 2), polls=3):
        self.scenes = {s: None for s in scenes}
        self.polls = polls
        self.left = {}
        self.work = {}
        self.launches = []      # (slot, [rid], slots busy at launch)

    def launch(self, slot, reqs):
        self.left[slot] = self.polls
        self.work[slot] = reqs
        self.launches.append((slot, [r.rid for r in reqs], len(self.work)))

    def poll(self, slot):
        self.left[slot] -= 1
        return self.left[slot] <= 0

    def collect(self, slot):
        reqs = self.work.pop(slot)
        for r in reqs:
            r.out = np.zeros((r.max_bounces, r.n, 4), np.int32)
            r.path_len = np.zeros(r.n)
            r.n_hits = np.zeros(r.n, np.int32)
        return reqs


def rays(n, bad=False):
    r = np.zeros((n, 8), np.float32)
    r[:, 6] = 1.0
    r[:, 7] = 10.0
    if bad:
        r[0, 0] = np.nan
    return r


def make(budget=10 ** 9, slots=2, max_batch=4, polls=3):
    ex = HostExecutor(polls=polls)
    return Server(ex, budget, slots, max_batch), ex


def test_malformed_queries_never_enter_the_queue():
    srv, ex = make()
    bad = [srv.submit(7, 2, rays(4)), srv.submit(0, 2, rays(4, bad=True)),
           srv.submit(0, 0, rays(4)), srv.submit(0, 1, rays(4).astype(np.float64)),
           srv.submit(0, 1, np.zeros((0, 8), np.float32)),
           srv.submit(0, 1, tx=(0.0, float("inf"), 1.0), n_rays=10),
           srv.submit(0, 1, tx=(0.0, 0.0, 1.0), n_rays=0), srv.submit(0, 1, tx=(0.0, 1.0), n_rays=5)]
    for r in bad:
        assert r.status == FAILED and r.error
    assert "not resident" in bad[0].error and "finite" in bad[1].error
    assert "transmitter" in bad[5].error and "ray count" in bad[6].error
    srv.run_until_idle()
    assert ex.launches == []


def test_budget_backlog_runs_in_arrival_order():
    one = Request(0, 0, 2, 0.0, rays=rays(100)).device_bytes()
    srv, ex = make(budget=one, slots=2)   # room for a single query at a time
    reqs = [srv.submit(0, 2, rays(100)) for _ in range(5)]
    srv.run_until_idle()
    assert all(r.status == DONE for r in reqs)
    assert [ids for _, ids, _ in ex.launches] == [[0], [1], [2], [3], [4]]
    assert srv.sched.admission_waits > 0
    assert srv.sched.used == 0


def test_oversize_query_fails_and_the_rest_run():
    one = Request(0, 0, 2, 0.0, rays=rays(100)).device_bytes()
    srv, ex = make(budget=2 * one)
    small = srv.submit(0, 2, rays(100))
    big = srv.submit(0, 6, rays(1000))
    after = srv.submit(1, 2, rays(100))
    srv.run_until_idle()
    assert big.status == FAILED and "budget" in big.error
    assert small.status == DONE and after.status == DONE
    assert big in srv.finished


def test_cancel_pending_query():
    srv, ex = make(slots=1, max_batch=1, polls=5)
    a = srv.submit(0, 1, rays(10))
    srv.step()                    # a runs in the only slot
    b = srv.submit(0, 1, rays(10))
    c = srv.submit(0, 1, rays(10))
    srv.step()
    assert srv.cancel(b)
    srv.run_until_idle()
    assert a.status == DONE and c.status == DONE and b.status == CANCELLED
    assert all(b.rid not in ids for _, ids, _ in ex.launches)


def test_batches_overlap_across_slots():
    srv, ex = make(slots=3, max_batch=2, polls=4)
    first = [srv.submit(0, 1, rays(10)) for _ in range(2)]
    srv.step()                    # batch 1 on slot 0
    later = [srv.submit(1, 3, rays(10)) for _ in range(3)]
    srv.step()                    # admitted while batch 1 still runs
    assert max(busy for _, _, busy in ex.launches) >= 2
    srv.run_until_idle()
    assert all(r.status == DONE for r in first + later)
    m = srv.metrics()
    assert m["queries"] == 5 and m["failed"] == 0


def test_scheduler_never_overtakes_the_head():
    s = Scheduler(budget_bytes=Request(0, 0, 1, 0.0, rays=rays(100)).device_bytes(), slots=4, max_batch=8)
    big = Request(0, 0, 1, 0.0, rays=rays(100))
    small = Request(1, 0, 1, 0.0, rays=rays(1))
    s.enqueue(big)
    s.enqueue(small)
    slot, batch = s.admit()
    assert batch == [big]         # the small one waits behind the head
    assert s.admit() is None
    s.release(slot, batch)
    assert s.admit()[1] == [small]


def test_check_request_limits():
    ok = Request(0, 0, 6, 0.0, rays=rays(3))
    assert check_request(ok, {0: None}) == ""
    assert check_request(Request(0, 0, 65, 0.0, rays=rays(3)), {0: None})
    assert check_request(Request(0, 0, 1, 0.0, tx=(0, 0, 1), n_rays=11), {0: None}, 10)
    assert check_request(Request(0, 0, 1, 0.0, tx=(0, 0, 1), n_rays=10), {0: None}, 10) == ""


def test_consumer_sees_every_finished_query_and_can_release_results():
    from paper_2208_10008_amd.serve import count_segments, release_results
    seen = []

    def consumer(r):
        assert r.status == DONE and r.out is not None
        r.n_hits[:] = np.arange(r.n) % (r.max_bounces + 2)   # chains of every length
        want = int(np.minimum(r.n_hits + 1, r.max_bounces).sum())
        assert count_segments(r) == want
        release_results(r)
        assert r.segments == want and r.out is None and r.n_hits is None
        seen.append(r.rid)

    ex = HostExecutor(polls=2)
    srv = Server(ex, 10 ** 9, 2, 3, on_done=consumer)
    reqs = [srv.submit(0, 1 + k % 4, rays(10 + k)) for k in range(7)]
    srv.run_until_idle()
    assert sorted(seen) == [r.rid for r in reqs]
    m = srv.metrics()
    assert m["queries"] == 7 and m["segments"] == sum(r.segments for r in reqs)


def test_field_point_queries_are_checked_and_sized():
    from paper_2208_10008_amd.serve import MAX_RECEIVERS
    srv, ex = make()
    pts = np.zeros((4, 3))
    bad = [srv.submit(0, 2, rays(4), receivers=pts.astype(np.float32), delta=0.01, rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=np.zeros((4, 2)), delta=0.01, rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=np.zeros((0, 3)), delta=0.01, rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=np.full((4, 3), np.nan), delta=0.01, rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=pts, delta=float("nan"), rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=pts, delta=-1.0, rec_cap=8),
           srv.submit(0, 2, rays(4), receivers=pts, delta=0.01, rec_cap=-1),
           srv.submit(0, 2, rays(4), receivers=np.zeros((MAX_RECEIVERS + 1, 3)), delta=0.01)]
    for r in bad:
        assert r.status == FAILED and r.error
    ok = Request(0, 0, 3, 0.0, rays=rays(100), receivers=pts, delta=0.01, rec_cap=50)
    plain = Request(1, 0, 3, 0.0, rays=rays(100))
    assert check_request(ok, {0: None}) == ""
    # receptions replace the hit records in host memory, and add their records on the device
    assert ok.result_bytes() < plain.result_bytes()
    assert ok.device_bytes() == plain.device_bytes() + 4 * 24 + 50 * 32 + 8
