"""Continuous-batching trace server over resident scenes.

Scenes and their trees stay resident in HBM, and so does a table of launch
directions (a level-9 icosphere, first-appearance order).  A query is
(scene, transmitter, ray count, bounce depth) -- its rays are the first
`count` table directions from the transmitter, made on the device -- or
(scene, host rays, bounce depth); it may also carry field points (Sec. III-C,
Eq. (4)), and then only its receptions and hit counts come back instead of
every hit record.  It is checked when it is
submitted (a malformed query gets an error status and never enters the
queue), waits in arrival order, and is admitted when an execution slot is
free and its device memory (rays, hits, path lengths, hit counts) fits the
HBM budget.  Each slot owns a stream and a batch (rt_batch): the admitted
queries are uploaded, traced in one batched launch and copied back on that
stream, so a batch admitted while others are still on the device overlaps
with them.  Results are copied straight into pinned host buffers that the
query owns (from torch's caching pinned allocator) and handed out as numpy
views of them, without a host-side copy; dropping the arrays returns the
buffers to the pool.  Latency is measured from a query's arrival to its
results being in host memory.

    python -m paper_2208_10008_amd.serve --duration 60 --rate 200

runs the Poisson workload over the 8 scenes of the multi-scene set and
prints one JSON line (p50 / p99 latency, aggregate segments per second,
queue depth, admission waits).
"""
from __future__ import annotations

import argparse
import ctypes
import collections
import dataclasses
import itertools
import json
import math
import threading
import time
from typing import Callable, Optional

import numpy as np

from . import RAY_LAUNCH_DTYPE, RECEPTION_DTYPE


def _align(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


# request states
PENDING, RUNNING, DONE, FAILED, CANCELLED = "pending", "running", "done", "failed", "cancelled"
MAX_RAYS = 1 << 26
MAX_RECEIVERS = 1 << 16
MAX_RECORDS = 1 << 24


@dataclasses.dataclass
class Request:
    rid: int
    scene: int
    max_bounces: int
    arrival: float            # time.perf_counter() at submission
    tx: Optional[tuple] = None            # transmitter of generated rays
    n_rays: int = 0                       # ... and their count
    rays: Optional[np.ndarray] = None     # or float32 [n, 8] host rays
    receivers: Optional[np.ndarray] = None  # float64 [m, 3] field points: receptions come back
    delta: float = 0.0                      # ... the launch's ray spacing (radians, Eq. (4))
    rec_cap: int = 0                        # ... reception records kept (the count may exceed it)
    status: str = PENDING
    error: str = ""
    admitted: float = math.nan
    done: float = math.nan
    out: Optional[np.ndarray] = None       # int32 [max_bounces, n, 4] (rt_hit records)
    path_len: Optional[np.ndarray] = None  # float64 [n]
    n_hits: Optional[np.ndarray] = None    # int32 [n]
    segments: int = -1                     # traced segments, once counted
    receptions: Optional[np.ndarray] = None  # RECEPTION_DTYPE, the first min(count, rec_cap)
    n_receptions: int = -1                   # receptions found (may exceed rec_cap)

    @property
    def n(self) -> int:
        return self.rays.shape[0] if self.rays is not None else self.n_rays

    def device_bytes(self) -> int:
        """Device memory the query holds while it runs."""
        b = self.n * (32 + 16 * self.max_bounces + 8 + 4)
        if self.receivers is not None:
            b += self.receivers.shape[0] * 24 + max(self.rec_cap, 1) * 32 + 8
        return b

    def result_bytes(self) -> int:
        """Pinned host memory its results take: hits, path lengths and hit
        counts, or (with field points) reception records, their count and
        the hit counts."""
        if self.receivers is not None:
            return _align(max(self.rec_cap, 1) * 32) + _align(8) + _align(self.n * 4)
        return _align(self.n * 16 * self.max_bounces) + _align(self.n * 8) + _align(self.n * 4)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def check_request(req: Request, scenes, max_generated: int = MAX_RAYS) -> str:
    """Why a query cannot run ('' when it can)."""
    if req.scene not in scenes:
        return f"scene {req.scene} is not resident"
    if req.rays is None:
        if req.tx is None or len(req.tx) != 3 or not np.isfinite(np.asarray(req.tx, float)).all():
            return "transmitter must be three finite coordinates"
        if not 1 <= req.n_rays <= max_generated:
            return f"ray count must lie in 1..{max_generated}"
    else:
        r = req.rays
        if not isinstance(r, np.ndarray) or r.dtype != np.float32 or r.ndim != 2 or r.shape[1] != 8:
            return "rays must be float32 [n, 8]"
        if not 1 <= r.shape[0] <= MAX_RAYS:
            return f"ray count must lie in 1..{MAX_RAYS}"
        if not np.isfinite(r).all():
            return "rays must be finite"
    if not 1 <= req.max_bounces <= 64:
        return "bounce depth must lie in 1..64"
    if req.receivers is not None:
        p = req.receivers
        if not isinstance(p, np.ndarray) or p.dtype != np.float64 or p.ndim != 2 or p.shape[1] != 3:
            return "field points must be float64 [m, 3]"
        if not 1 <= p.shape[0] <= MAX_RECEIVERS:
            return f"field point count must lie in 1..{MAX_RECEIVERS}"
        if not np.isfinite(p).all():
            return "field points must be finite"
        if not (math.isfinite(req.delta) and req.delta >= 0.0):
            return "ray spacing delta must be finite and >= 0"
        if not 0 <= req.rec_cap <= MAX_RECORDS:
            return f"reception capacity must lie in 0..{MAX_RECORDS}"
    return ""


class Scheduler:
    """Admission policy, independent of the device: arrival order, a free
    slot and room in the memory budget; the head of the queue is never
    overtaken (no starvation)."""

    def __init__(self, budget_bytes: int, slots: int, max_batch: int,
                 max_batch_bytes: int = 1 << 62):
        self.budget = budget_bytes
        self.max_batch_bytes = max_batch_bytes  # pinned result bytes one batch may hold
        self.used = 0
        self.free_slots = list(range(slots))
        self.max_batch = max_batch
        self.pending: collections.deque = collections.deque()
        self.rejected = []         # queries that can never fit the budget
        self.admission_waits = 0   # passes where the head waited for memory or a slot

    def enqueue(self, req: Request):
        self.pending.append(req)

    def cancel(self, req: Request) -> bool:
        if req.status == PENDING and req in self.pending:
            self.pending.remove(req)
            req.status = CANCELLED
            return True
        return False

    def admit(self):
        """Returns (slot, requests) for the next batch, or None."""
        if not self.pending:
            return None
        if not self.free_slots:
            self.admission_waits += 1
            return None
        batch, need, staged = [], 0, 0
        while self.pending and len(batch) < self.max_batch:
            req = self.pending[0]
            b, rb = req.device_bytes(), req.result_bytes()
            if b > self.budget or rb > self.max_batch_bytes:  # can never fit
                self.pending.popleft()
                req.status, req.error = FAILED, "query exceeds the memory budget"
                self.rejected.append(req)
                continue
            if self.used + need + b > self.budget or staged + rb > self.max_batch_bytes:
                break
            batch.append(self.pending.popleft())
            need += b
            staged += rb
        if not batch:
            self.admission_waits += 1
            return None
        self.used += need
        return self.free_slots.pop(0), batch

    def release(self, slot: int, batch):
        self.used -= sum(r.device_bytes() for r in batch)
        self.free_slots.append(slot)


class GpuExecutor:
    """Resident scenes and launch directions, one stream and one rt_batch per
    slot.  Generated rays run from tmin to tmax along each direction."""

    def __init__(self, scenes, slots: int, max_batch: int, level: int = 9, tmin: float = 1e-4,
                 tmax: float = 2000.0, stage_bytes: int = 1 << 30):
        import torch
        from rtgen import icosphere
        from . import Batch
        self.torch = torch
        self.scenes = scenes
        self.dirs = torch.from_numpy(icosphere.directions(level).astype(np.float32)).cuda()
        self.max_generated = self.dirs.shape[0]
        self.tmin, self.tmax = tmin, tmax
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.batches = [Batch(max_batch) for _ in range(slots)]
        self.stage_bytes = stage_bytes  # pinned result bytes one batch may hold
        self.events = [None] * slots
        self.work = [None] * slots

    def launch(self, slot: int, reqs):
        """One batch on the slot's stream.  Per kind of array the batch takes
        one device allocation and one pinned host buffer, and each query a
        16-byte-aligned slice of them: the host work per query is a ray launch
        and a table entry (pointers into the pools).  Results are copied back
        with one copy per array kind and handed out as numpy views of the
        pinned buffers."""
        from . import load, rt_query, rt_receivers, _stream
        torch = self.torch
        lib = load()
        s = self.streams[slot]
        sp = _stream(s)
        plain = [r for r in reqs if r.receivers is None]
        recv = [r for r in reqs if r.receivers is not None]
        dev = {}
        with torch.cuda.stream(s):
            def pool(name, count, dtype):
                dev[name] = torch.empty(max(count, 1), dtype=dtype, device="cuda")
                return dev[name].data_ptr()

            base_rays = pool("rays", 8 * sum(r.n for r in reqs), torch.float32)
            # plain queries: hits, path lengths, hit counts (all copied back)
            p_out = pool("p_out", sum(4 * r.n * r.max_bounces for r in plain), torch.int32)
            p_pl = pool("p_pl", sum(r.n for r in plain), torch.float64)
            p_nh = pool("p_nh", sum(r.n for r in plain), torch.int32)
            # queries with field points: hits and path lengths stay on the device
            r_out = pool("r_out", sum(4 * r.n * r.max_bounces for r in recv), torch.int32)
            r_pl = pool("r_pl", sum(r.n for r in recv), torch.float64)
            r_nh = pool("r_nh", sum(r.n for r in recv), torch.int32)
            r_rec = pool("r_rec", sum(8 * max(r.rec_cap, 1) for r in recv), torch.int32)
            r_cnt = pool("r_cnt", len(recv), torch.int64)
            r_pos = 0
            if recv:
                pos_host = torch.from_numpy(np.concatenate([r.receivers for r in recv])).pin_memory()
                r_pos = pool("r_pos", pos_host.numel(), torch.float64)
                dev["r_pos"].copy_(pos_host.view(-1), non_blocking=True)
                dev["pos_host"] = pos_host
            arr = (rt_query * max(len(reqs), 1))()
            keep = []   # rt_receivers structs, read by rt_batch_set
            # the generated rays of the whole batch: one launch from a table
            first = np.cumsum([0] + [r.n for r in reqs[:-1]])
            gen = [k for k, r in enumerate(reqs) if r.rays is None]
            if gen:
                table = np.zeros(len(gen), RAY_LAUNCH_DTYPE)
                table["src"] = [reqs[k].tx for k in gen]
                table["first"] = first[gen]
                table["n"] = [reqs[k].n for k in gen]
                dev["table_host"] = torch.from_numpy(table.view(np.uint8)).pin_memory()
                dev["table"] = dev["table_host"].to("cuda", non_blocking=True)
                _check_rc(lib.rt_rays_from_directions_many(
                    self.dirs.data_ptr(), self.dirs.shape[0], dev["table"].data_ptr(), len(gen),
                    self.tmin, self.tmax, base_rays, sum(r.n for r in reqs), sp))
            o_ray = o_p = o_po = o_r = o_ro = o_rec = o_pos = 0
            for k, r in enumerate(reqs):
                n, nb = r.n, r.max_bounces
                rays = base_rays + 32 * o_ray
                o_ray += n
                if r.rays is not None:
                    dev[f"host_rays{k}"] = torch.from_numpy(r.rays).pin_memory()
                    dev["rays"][8 * (o_ray - n):8 * o_ray].view(n, 8).copy_(
                        dev[f"host_rays{k}"], non_blocking=True)
                q = arr[k]
                q.bvh, q.rays, q.n, q.max_bounces = self.scenes[r.scene].handle, rays, n, nb
                if r.receivers is None:
                    q.out, q.path_len, q.n_hits = p_out + 16 * o_po, p_pl + 8 * o_p, p_nh + 4 * o_p
                    o_po += n * nb
                    o_p += n
                else:
                    m, cap = r.receivers.shape[0], max(r.rec_cap, 1)
                    q.out, q.path_len, q.n_hits = r_out + 16 * o_ro, r_pl + 8 * o_r, r_nh + 4 * o_r
                    c = rt_receivers()
                    c.pos, c.n, c.reserved, c.delta = r_pos + 24 * o_pos, m, 0, r.delta
                    c.rec, c.cap, c.count = r_rec + 32 * o_rec, r.rec_cap, r_cnt + 8 * len(keep)
                    keep.append(c)
                    q.receivers = ctypes.addressof(c)
                    o_ro += n * nb
                    o_r += n
                    o_rec += cap
                    o_pos += m
            st = self.batches[slot].set_table(arr, len(reqs))
            if any(st):
                raise RuntimeError(f"serving table entries rejected: {st}")
            self.batches[slot].launch(stream=s)
            # segments each query traced, counted on the device (a segment per
            # hit plus the final miss, at most the bounce limit per chain)
            dev["p_seg"] = self._segments(plain, dev["p_nh"])
            dev["r_seg"] = self._segments(recv, dev["r_nh"])

            def to_host(name):
                t = dev[name]
                h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                h.copy_(t, non_blocking=True)
                return h
            host = {k: to_host(k) for k in (("p_out", "p_pl", "p_nh", "p_seg") if plain else ())}
            if recv:
                host.update({k: to_host(k) for k in ("r_nh", "r_rec", "r_cnt", "r_seg")})
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot] = ev
        self.work[slot] = (plain, recv, host, dev, keep)

    def _segments(self, reqs, n_hits):
        torch = self.torch
        if not reqs:
            return torch.zeros(1, dtype=torch.int64, device="cuda")
        n = torch.tensor([r.n for r in reqs], dtype=torch.int64).to("cuda", non_blocking=True)
        nb = torch.tensor([r.max_bounces for r in reqs], dtype=torch.int32).to("cuda",
                                                                             non_blocking=True)
        total = sum(r.n for r in reqs)
        seg = torch.minimum(n_hits[:total] + 1, torch.repeat_interleave(nb, n, output_size=total))
        c = torch.cumsum(seg, 0, dtype=torch.int64)
        ends = torch.cumsum(n, 0) - 1
        per = c[ends]
        return torch.cat([per[:1], per[1:] - per[:-1]])

    def poll(self, slot: int) -> bool:
        return self.events[slot] is not None and self.events[slot].query()

    def collect(self, slot: int):
        plain, recv, host, dev, keep = self.work[slot]
        if plain:  # numpy views of the batch's pinned buffers (they keep them alive)
            out, pl, nh = host["p_out"].numpy(), host["p_pl"].numpy(), host["p_nh"].numpy()
            p = po = 0
            seg = host["p_seg"].numpy()
            for k, r in enumerate(plain):
                n, nb = r.n, r.max_bounces
                r.out = out[4 * po:4 * (po + n * nb)].reshape(nb, n, 4)
                r.path_len, r.n_hits = pl[p:p + n], nh[p:p + n]
                r.segments = int(seg[k])
                p += n
                po += n * nb
        if recv:
            cnt, recs, nh = host["r_cnt"].numpy(), host["r_rec"].numpy(), host["r_nh"].numpy()
            q = rec = 0
            for k, r in enumerate(recv):
                n = r.n
                r.n_receptions = int(cnt[k])
                got = min(r.n_receptions, r.rec_cap)
                r.receptions = (recs[8 * rec:8 * (rec + got)].reshape(got, 8)
                                .view(RECEPTION_DTYPE).reshape(-1))
                r.n_hits = nh[q:q + n]
                r.segments = int(host["r_seg"][k])
                q += n
                rec += max(r.rec_cap, 1)
        self.events[slot] = None
        self.work[slot] = None
        return plain + recv


def _check_rc(rc: int):
    if rc != 0:
        from . import RtError, load
        raise RtError(rc, load().rt_last_error().decode())


class Server:
    """Continuous batching: one thread admits, launches and completes.

    executor: GpuExecutor (or any object with launch / poll / collect and a
    `scenes` mapping, e.g. a host stand-in in tests)."""

    def __init__(self, executor, budget_bytes: int, slots: int = 4, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter,
                 on_done: Optional[Callable[[Request], None]] = None):
        self.ex = executor
        self.on_done = on_done  # called with each finished query (e.g. a consumer)
        self.sched = Scheduler(budget_bytes, slots, max_batch,
                               getattr(executor, "stage_bytes", 1 << 62))
        self.clock = clock
        self.lock = threading.Lock()
        self.inbox: collections.deque = collections.deque()
        self.running = {}
        self.finished = []
        self.depth_samples = []
        self.max_running = 0       # most batches on the device at once
        self.ids = itertools.count()
        self.thread = None
        self.stop_flag = False

    def submit(self, scene: int, max_bounces: int, rays: Optional[np.ndarray] = None,
               tx=None, n_rays: int = 0, receivers: Optional[np.ndarray] = None,
               delta: float = 0.0, rec_cap: int = 0) -> Request:
        """A query: host rays, or a transmitter and a ray count; with field
        points (and the ray spacing delta), only receptions come back."""
        req = Request(next(self.ids), scene, int(max_bounces), self.clock(), tx=tx,
                      n_rays=int(n_rays), rays=rays, receivers=receivers, delta=float(delta),
                      rec_cap=int(rec_cap))
        err = check_request(req, self.ex.scenes, getattr(self.ex, "max_generated", MAX_RAYS))
        if err:  # never enters the queue
            req.status, req.error = FAILED, err
            with self.lock:
                self.finished.append(req)
            return req
        self.inbox.append(req)
        return req

    def cancel(self, req: Request) -> bool:
        with self.lock:
            return self.sched.cancel(req)

    def step(self) -> bool:
        """One scheduling pass; returns True when anything happened."""
        busy = False
        with self.lock:
            while self.inbox:
                self.sched.enqueue(self.inbox.popleft())
            self.depth_samples.append(len(self.sched.pending))
            # completions
            for slot in list(self.running):
                if self.ex.poll(slot):
                    reqs = self.ex.collect(slot)
                    now = self.clock()
                    for r in reqs:
                        r.done, r.status = now, DONE
                        if self.on_done is not None:
                            self.on_done(r)
                    self.sched.release(slot, reqs)
                    self.finished.extend(reqs)
                    del self.running[slot]
                    busy = True
            # admissions
            while True:
                got = self.sched.admit()
                if self.sched.rejected:
                    self.finished.extend(self.sched.rejected)
                    self.sched.rejected.clear()
                if got is None:
                    break
                slot, reqs = got
                now = self.clock()
                for r in reqs:
                    r.admitted, r.status = now, RUNNING
                self.ex.launch(slot, reqs)
                self.running[slot] = reqs
                self.max_running = max(self.max_running, len(self.running))
                busy = True
        return busy

    def idle(self) -> bool:
        with self.lock:
            return not self.inbox and not self.sched.pending and not self.running

    def run_until_idle(self, timeout: float = 600.0):
        t0 = time.perf_counter()
        while not self.idle():
            if not self.step():
                time.sleep(2e-5)
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")

    def start(self):
        def loop():
            while not self.stop_flag:
                if not self.step():
                    time.sleep(2e-5)
        self.stop_flag = False
        self.thread = threading.Thread(target=loop, daemon=True)
        self.thread.start()

    def stop(self):
        self.stop_flag = True
        if self.thread:
            self.thread.join()
            self.thread = None

    def metrics(self) -> dict:
        done = [r for r in self.finished if r.status == DONE]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        segs = sum(r.segments if r.segments >= 0 else count_segments(r) for r in done)
        span = (max(r.done for r in done) - min(r.arrival for r in done)) if done else 0.0
        return {"queries": len(done), "failed": sum(r.status == FAILED for r in self.finished),
                "latency_ms_p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                "latency_ms_p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                "latency_ms_max": round(1e3 * float(lat.max()), 3),
                "segments": segs, "rays": sum(r.n for r in done),
                "mrays_s": round(segs / span / 1e6, 2) if span > 0 else 0.0,
                "queue_depth_mean": round(float(np.mean(self.depth_samples or [0])), 2),
                "queue_depth_max": int(max(self.depth_samples or [0])),
                "admission_waits": self.sched.admission_waits,
                "max_batches_in_flight": self.max_running,
                "receptions": sum(max(r.n_receptions, 0) for r in done)}


def count_segments(r: Request) -> int:
    """Segments a finished query traced (a segment per hit, plus the final
    miss unless the chain reached its bounce limit)."""
    return int(np.minimum(r.n_hits + 1, r.max_bounces).sum())


def release_results(r: Request):
    """Consumer for throughput runs: keeps the query's segment count (counted
    on the device by the executor, else here) and drops its result arrays,
    returning their pinned buffers to the pool."""
    if r.segments < 0:
        r.segments = count_segments(r)
    r.out = r.path_len = r.n_hits = r.receptions = None


def poisson_queries(duration: float, rate: float, seed: int = 0, scenes=range(8),
                    receivers: int = 0, rec_cap: int = 1 << 14):
    """The serving query stream: Poisson arrivals; per query a scene (uniform), a
    transmitter uniform over the scene outside buildings at 5-40 m, a ray
    count log-uniform in 10k-1M (icosphere prefix) and a bounce depth uniform
    in 1-6.  Returns [(arrival_s, scene, tx, n_rays, max_bounces)]; with
    `receivers` > 0 each entry also carries that many field points (drawn from
    a pool of points outside buildings, 1.5 m up), the ray spacing delta of the
    launch (the mean edge angle of the smallest icosphere level that holds
    the rays) and a record capacity, as keyword arguments of Server.submit."""
    from rtgen import icosphere, scenes as sc, workloads
    rng = np.random.default_rng(seed)
    geo = {s: workloads.multiscene_scene(s) for s in scenes}
    pool, deltas = {}, {}
    if receivers:
        prng = np.random.default_rng(seed + 1)
        pool = {s: sc.free_points(prng, geo[s][1], geo[s][0], 1.5, 512) for s in scenes}
    out, t = [], 0.0
    scene_ids = list(scenes)
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        s = scene_ids[int(rng.integers(len(scene_ids)))]
        tris, half = geo[s]
        tx = sc.free_point(rng, half, tris, float(rng.uniform(5.0, 40.0)))
        n = int(round(10 ** rng.uniform(4.0, 6.0)))
        nb = int(rng.integers(1, 7))
        entry = (t, s, tuple(float(x) for x in tx), n, nb)
        if receivers:
            lv = next(L for L in range(16) if icosphere.vertex_count(L) >= n)
            if lv not in deltas:
                deltas[lv] = float(icosphere.edge_angles(lv).mean())
            pts = pool[s][rng.choice(pool[s].shape[0], receivers, replace=False)]
            entry += ({"receivers": np.ascontiguousarray(pts), "delta": deltas[lv],
                       "rec_cap": rec_cap},)
        out.append(entry)
    return out


def resident_scenes(ids=range(8)):
    """Trees of the multi-scene set built once (source point: scene centre,
    25 m up)."""
    import torch
    from . import BVH, SplitParams
    from rtgen import workloads
    out = {}
    for s in ids:
        tris, _ = workloads.multiscene_scene(s)
        out[s] = BVH(torch.from_numpy(tris).cuda(),
                     SplitParams(alpha=0.4, src=workloads.MULTI_SRC))
    return out


def run_stream(server: Server, stream, clock=time.perf_counter, progress=None):
    """Feeds the query stream at its arrival times (relative to now) while
    the server thread runs; returns when every query has finished.
    progress: seconds between status lines on stderr (None: quiet)."""
    import sys
    server.start()
    t0 = last = clock()

    def report():
        nonlocal last
        if progress and clock() - last >= progress:
            last = clock()
            print(f"[serve] t={last - t0:.1f}s finished={len(server.finished)} "
                  f"pending={len(server.sched.pending)} running={len(server.running)}",
                  file=sys.stderr, flush=True)
    for item in stream:
        at, s, tx, n, nb = item[:5]
        extra = item[5] if len(item) > 5 else {}
        while clock() - t0 < at:
            time.sleep(max(0.0, min(1e-3, at - (clock() - t0))))
        server.submit(s, nb, tx=tx, n_rays=n, **extra)
        report()
    while not server.idle():
        time.sleep(1e-3)
        report()
    server.stop()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--receivers", type=int, default=0,
                    help="field points per query: only receptions and hit counts come back")
    ap.add_argument("--rec-cap", type=int, default=1 << 14)
    a = ap.parse_args()
    import sys
    import torch
    t0 = time.perf_counter()
    stream = poisson_queries(a.duration, a.rate, a.seed, receivers=a.receivers, rec_cap=a.rec_cap)
    print(f"[serve] {len(stream)} queries drawn", file=sys.stderr, flush=True)
    scenes = resident_scenes()
    torch.cuda.synchronize()
    print("[serve] scenes resident", file=sys.stderr, flush=True)
    ex = GpuExecutor(scenes, a.slots, a.max_batch)
    # warm-up (not timed): one small query per scene through every slot
    warm = Server(ex, int(a.budget_gib * 2 ** 30), a.slots, a.max_batch)
    for _ in range(a.slots):
        for sc in scenes:
            warm.submit(sc, 2, tx=(0.0, 0.0, 25.0), n_rays=10_000)
    warm.run_until_idle()
    srv = Server(ex, int(a.budget_gib * 2 ** 30), a.slots, a.max_batch, on_done=release_results)
    setup = time.perf_counter() - t0
    run_stream(srv, stream, progress=5.0)
    m = srv.metrics()
    m.update({"workload": f"poisson {a.rate:g}/s for {a.duration:g} s over 8 scenes "
                          f"(1k-200k facets), 10k-1M rays, 1-6 bounces"
                          + (f", {a.receivers} field points per query (receptions only)"
                             if a.receivers else ""),
              "slots": a.slots, "max_batch": a.max_batch, "budget_gib": a.budget_gib,
              "setup_s": round(setup, 1)})
    print(json.dumps(m), flush=True)


if __name__ == "__main__":
    main()
