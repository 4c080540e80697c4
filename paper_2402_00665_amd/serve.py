"""Continuous-batching request loop for build + query requests.

A request asks for the rope-LBVH of n points (63-bit codes) and the CSR
answer of m sphere queries against it.  The loop

  * admits requests in arrival order while the batch being formed, the
    batches in flight and the trees kept resident fit an HBM byte budget
    (footprints are exact: they come from the library's workspace-size
    functions plus the input, tree and result arrays);
  * groups every admitted request that has arrived into one batch: one
    batched build (all trees at once) and one batched count + fill over all
    the batch's queries, on one of ``executor.slots`` streams, so batches
    formed while others run overlap on the device;
  * keeps finished trees resident (least recently finished evicted first
    when admission needs the memory) so they can be queried again;
  * keeps each finished batch's results (CSR offsets and indices, on the
    device), counted in the budget; when memory is needed, resident trees
    (a cache) are evicted first, least recently finished first, and kept
    results only once no tree is left.  ``keep_results=False`` drops the
    results as soon as an ``on_done`` callback has seen them;
  * reports every request's latency (completion - arrival), hits, status.

The executor does the work; ``GpuExecutor`` drives the batched entry points
and ``PlainExecutor`` the single-tree ones, one request at a time (the FIFO
baseline).  The loop itself never touches device memory, so it can be
driven by a host-side executor and a virtual clock.

Failure handling: a request whose n, m or payload is invalid ends with
LBVH_EINVAL, one whose footprint alone exceeds the budget with
LBVH_ENOSPACE, one not admitted before its deadline with ERR_DEADLINE; an
exception raised by the executor for a batch of several requests makes the
loop retry each of them alone, and a request that fails alone ends with
ERR_EXECUTOR while the loop goes on.
"""

from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

LBVH_OK = 0
LBVH_EINVAL = -1
LBVH_ENOSPACE = -2
LBVH_EDEVICE = -4
ERR_DEADLINE = -100
ERR_EXECUTOR = -101

MAX_PRIMS = (1 << 30) - 1
MAX_BATCH = 1024          # requests per batch the GPU executors accept


@dataclass
class Request:
    """One build + query request.  The payload is named, not carried: points
    are rows [p_off, p_off + n) of the executor's point pool, sphere centres
    rows [q_off, q_off + m) of its centre pool, all spheres of radius
    ``radius``.  Times are seconds from the start of the trace."""
    rid: int
    arrival: float
    n: int
    m: int
    p_off: int = 0
    q_off: int = 0
    radius: float = 0.0
    deadline: float | None = None


@dataclass
class Response:
    rid: int
    status: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    batch: int = -1
    hits: int = 0
    error: str = ""
    _handle: object = field(default=None, repr=False)
    _k: int = -1

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    def csr(self, out=None):
        """(offsets [m+1] from 0, indices [hits]) of this request, as the
        executor's arrays (device tensors for the GPU executors).  With
        ``out`` = (offsets [m+1] int64, indices [hits] int32) caller-owned
        buffers, the answer is written there (enqueued on the current
        stream, nothing allocated) and ``out`` is returned.  KeyError once
        the server has dropped the results (evicted, or not kept)."""
        if self.status != LBVH_OK:
            raise RuntimeError(f"request {self.rid} has no result (status {self.status})")
        if out is None:
            return self._handle.csr(self._k)
        return self._handle.csr(self._k, out)


class WallClock:
    """Seconds since construction; idle() yields the CPU briefly."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, until: float | None):
        # poll (yield only) while work is in flight; sleep most of the way
        # to a known next arrival, then poll
        rem = 0.0 if until is None else until - self.now()
        time.sleep(rem - 2e-4 if rem > 3e-4 else 0)


class VirtualClock:
    """Discrete-event time: idle() jumps to the next event."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def idle(self, until: float | None):
        if until is None:
            raise RuntimeError("virtual clock idles with no event ahead")
        self.t = max(self.t, until)


def request_valid(r: Request, pool_points: int, pool_centres: int) -> bool:
    return (0 <= r.n <= MAX_PRIMS and 0 <= r.m <= (1 << 31) - 1 and r.p_off >= 0 and r.q_off >= 0
            and r.p_off + r.n <= pool_points and r.q_off + r.m <= pool_centres
            and r.radius >= 0.0 and r.p_off % 4 == 0)


class _InFlight:
    __slots__ = ("bid", "reqs", "slot", "handle", "bytes", "resident_bytes", "admitted",
                 "tree_bytes", "result_bytes")

    def __init__(self, bid, reqs, slot, handle, nbytes, resident_bytes, admitted):
        self.tree_bytes = self.result_bytes = 0   # held on the device after completion
        self.bid, self.reqs, self.slot, self.handle = bid, reqs, slot, handle
        self.bytes, self.resident_bytes, self.admitted = nbytes, resident_bytes, admitted


class Server:
    """The request loop.  ``budget_bytes`` bounds in-flight plus resident
    device memory; ``max_batch`` and ``max_batch_points`` cap a batch.
    A finished batch keeps its tree (``keep_resident``) and its results
    (``keep_results``) on the device, both counted in the budget; trees are
    evicted before results.  ``on_done(response)`` is called for each
    finished request
    while its results are still on the device, with the executor's stream
    for that batch current (GPU executors), so device work it enqueues on
    the results runs before their memory can be reused."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 64,
                 max_batch_points: int = 1 << 25, clock=None, keep_resident: bool = True,
                 pause_gc: bool | None = None, keep_results: bool = True, on_done=None):
        self.ex = executor
        self.keep_results = keep_results
        self.on_done = on_done
        # Python's cyclic collector, when it walks a heap holding tens of
        # thousands of responses and tensors, stalls the loop for tens of
        # milliseconds (it set the latency tail); run() collects once and
        # pauses it, reference counting still frees everything (default: on
        # with the wall clock, off with a virtual one)
        self.pause_gc = pause_gc
        self.budget = int(budget_bytes)
        self.max_batch = max(1, int(max_batch))
        self.max_points = int(max_batch_points)
        self.clock = clock or WallClock()
        if self.pause_gc is None:
            self.pause_gc = isinstance(self.clock, WallClock)
        self.keep_resident = keep_resident
        self.resident = collections.OrderedDict()   # bid -> (_InFlight, {rid: k}): resident trees
        self.kept = collections.OrderedDict()       # bid -> _InFlight: batches whose results are kept
        self.where = {}                              # rid -> bid of its resident tree
        self.resident_bytes = 0                      # resident trees + kept results
        self.kept_bytes = 0                          # ... of which kept results
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.batches = []                            # (bid, size, points) per batch started
        self._bid = 0

    # -------------------------------------------------------------- memory

    def _evictable(self) -> bool:
        return bool(self.resident or self.kept)

    def _evict_one(self):
        """Free the least recently finished tree, or, with no tree left, the
        least recently finished batch's kept results."""
        if self.resident:
            bid, (b, _) = self.resident.popitem(last=False)
            for r in b.reqs:
                if self.where.get(r.rid) == bid:
                    del self.where[r.rid]
            self.resident_bytes -= b.tree_bytes
            b.tree_bytes = 0
            self.ex.evict(b.handle)
        else:
            _, b = self.kept.popitem(last=False)
            self.resident_bytes -= b.result_bytes
            self.kept_bytes -= b.result_bytes
            b.result_bytes = 0
            self.ex.drop_results(b.handle)

    def _used(self) -> int:
        return self.inflight_bytes + self.resident_bytes

    def evict_all(self):
        """Drop every resident tree and every kept result."""
        while self._evictable():
            self._evict_one()

    # --------------------------------------------------------------- loop

    def run(self, requests) -> list[Response]:
        gc_was_on = gc.isenabled()
        if self.pause_gc:
            gc.collect()
            gc.disable()
        if isinstance(self.clock, WallClock):
            self.clock.t0 = time.perf_counter()   # arrivals count from the loop's start
        try:
            return self._run(requests)
        finally:
            if gc_was_on:
                gc.enable()

    def _run(self, requests) -> list[Response]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        out = {r.rid: Response(r.rid, LBVH_OK, r.arrival) for r in reqs}
        waiting = collections.deque()
        retry_alone = collections.deque()
        slots = list(range(self.ex.slots))
        inflight: list[_InFlight] = []
        nxt = 0

        def finish_req(r, status, err=""):
            o = out[r.rid]
            o.status, o.error, o.done = status, err, self.clock.now()

        def fail_batch(b: _InFlight, err: str):
            self.inflight_bytes -= b.bytes
            slots.append(b.slot)
            try:
                self.ex.release(b.handle)
                self.ex.evict(b.handle)
                self.ex.drop_results(b.handle)
            except Exception:   # noqa: BLE001  (a failed batch may not release cleanly)
                pass
            if len(b.reqs) == 1:
                finish_req(b.reqs[0], ERR_EXECUTOR, err)
            else:
                retry_alone.extend(b.reqs)

        while nxt < len(reqs) or waiting or inflight or retry_alone:
            progressed = False
            now = self.clock.now()
            # arrivals
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                progressed = True
                if not self.ex.valid(r):
                    finish_req(r, LBVH_EINVAL, "invalid request")
                elif self.ex.footprint([r])[0] > self.budget:
                    finish_req(r, LBVH_ENOSPACE, "footprint exceeds the budget")
                else:
                    waiting.append(r)
            # progress of batches in flight
            for b in list(inflight):
                try:
                    done = self.ex.advance(b.handle)
                except Exception as e:  # noqa: BLE001
                    inflight.remove(b)
                    fail_batch(b, f"{type(e).__name__}: {e}")
                    progressed = True
                    continue
                if not done:
                    continue
                progressed = True
                inflight.remove(b)
                t = self.clock.now()
                hits = self.ex.hits(b.handle)
                for k, r in enumerate(b.reqs):
                    o = out[r.rid]
                    o.done, o.hits, o._handle, o._k = t, int(hits[k]), b.handle, k
                    o.status = LBVH_OK
                if self.on_done is not None:
                    # on the batch's own stream: work the callback enqueues
                    # on the results is ordered before their memory is reused
                    with self.ex.stream_context(b.handle):
                        for r in b.reqs:
                            self.on_done(out[r.rid])
                self.ex.release(b.handle)
                self.inflight_bytes -= b.bytes
                slots.append(b.slot)
                # what stays on the device: the tree and/or the results
                if self.keep_resident:
                    b.tree_bytes = b.resident_bytes
                    self.resident[b.bid] = (b, {r.rid: k for k, r in enumerate(b.reqs)})
                    for r in b.reqs:
                        self.where[r.rid] = b.bid
                else:
                    self.ex.evict(b.handle)
                if self.keep_results:
                    b.result_bytes = self.ex.result_bytes(b.handle)
                    self.kept[b.bid] = b
                else:
                    self.ex.drop_results(b.handle)
                self.resident_bytes += b.tree_bytes + b.result_bytes
                self.kept_bytes += b.result_bytes
                while self._evictable() and self._used() > self.budget:
                    self._evict_one()
                self.peak_bytes = max(self.peak_bytes, self._used())
            # deadlines
            now = self.clock.now()
            for q in (waiting, retry_alone):
                for r in [r for r in q if r.deadline is not None and r.deadline < now]:
                    q.remove(r)
                    finish_req(r, ERR_DEADLINE, "not admitted before its deadline")
                    progressed = True
            # form batches while a slot is free
            while slots and (retry_alone or waiting):
                alone = bool(retry_alone)
                src = retry_alone if alone else waiting
                cap = 1 if alone else self.max_batch
                # resident trees can be evicted for a new batch, kept results not
                room = self.budget - self.inflight_bytes - self.kept_bytes
                take, pts = [], 0
                fp = (0, 0)
                for r in src:
                    if len(take) >= cap or (take and pts + r.n > self.max_points):
                        break
                    f = self.ex.footprint(take + [r])
                    if f[0] > room:
                        break
                    take.append(r)
                    pts += r.n
                    fp = f
                if not take:
                    break
                while self.resident and self._used() + fp[0] > self.budget:
                    self._evict_one()
                if self._used() + fp[0] > self.budget:
                    break
                for _ in take:
                    src.popleft()
                slot = slots.pop(0)
                bid = self._bid
                self._bid += 1
                t = self.clock.now()
                for r in take:
                    out[r.rid].admitted = t
                    out[r.rid].batch = bid
                try:
                    h = self.ex.submit(take, slot)
                except Exception as e:  # noqa: BLE001
                    slots.append(slot)
                    if len(take) == 1:
                        finish_req(take[0], ERR_EXECUTOR, f"{type(e).__name__}: {e}")
                    else:
                        retry_alone.extend(take)
                    progressed = True
                    continue
                b = _InFlight(bid, take, slot, h, fp[0], fp[1], t)
                inflight.append(b)
                self.inflight_bytes += fp[0]
                self.peak_bytes = max(self.peak_bytes, self._used())
                self.batches.append((bid, len(take), pts))
                progressed = True
            if not progressed:
                ahead = [reqs[nxt].arrival] if nxt < len(reqs) else []
                for b in inflight:
                    t = self.ex.ready_time(b.handle)
                    if t is None:
                        ahead = None
                        break
                    ahead.append(t)
                if ahead is not None and not ahead and (waiting or retry_alone):
                    # nothing in flight, nothing arriving, and the head does
                    # not fit: only resident trees can be holding the memory
                    if self._evictable():
                        self._evict_one()
                        continue
                    raise RuntimeError("request loop stalled with work waiting")
                self.clock.idle(None if ahead is None else min(ahead))
        return [out[r.rid] for r in sorted(requests, key=lambda r: r.rid)]

    # ------------------------------------------------------------ queries

    def query_resident(self, rid: int, centres, radius: float):
        """Query the resident tree of finished request ``rid`` with spheres
        (executor-side arrays).  Returns (offsets, indices); KeyError if the
        tree was evicted.  The tree becomes the most recently used.  These
        answers are the caller's: the budget does not count them."""
        bid = self.where[rid]
        b, ks = self.resident[bid]
        self.resident.move_to_end(bid)
        return self.ex.query_resident(b.handle, ks[rid], centres, radius)


def summarize(responses: list[Response], wall: float | None = None) -> dict:
    """p50/p99/mean latency (ms) and throughput of the finished requests."""
    import numpy as np
    ok = [r for r in responses if r.status == LBVH_OK]
    errors = collections.Counter(f"{r.status}: {r.error}" for r in responses if r.status != LBVH_OK)
    if not ok:
        return {"requests": len(responses), "ok": 0, "errors": dict(errors.most_common(3))}
    lat = np.array([r.latency for r in ok]) * 1e3
    first = min(r.arrival for r in ok)
    last = max(r.done for r in ok)
    span = wall if wall is not None else last - first
    return {"requests": len(responses), "ok": len(ok),
            "failed": len(responses) - len(ok),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "max_ms": round(float(lat.max()), 3),
            "makespan_s": round(span, 3),
            "throughput_rps": round(len(ok) / span, 1),
            "hits": int(sum(r.hits for r in ok)),
            **({"errors": dict(errors.most_common(3))} if errors else {})}


# ----------------------------------------------------------- GPU executors

def _footprint_common(ns, ms, hits_per_query):
    """Bytes of the arrays both executors allocate per request set, apart
    from the library workspaces: staged points (12 B/point), staged
    spheres (16 B/query), CSR offsets (8 B/query + 8) and the expected
    result indices (4 B/hit)."""
    N, M = sum(ns), sum(ms)
    return 12 * N + 16 * M + 8 * (M + len(ms)) + int(4 * hits_per_query * M)


class _GpuBase:
    """Shared parts of the GPU executors: the payload pools, streams and
    per-slot workspaces, request validation."""

    def __init__(self, pool_points, pool_centres, slots: int, hits_per_query: float = 8.0):
        import torch
        import paper_2402_00665_amd as lb
        self.torch, self.lb = torch, lb
        if not (pool_points.is_cuda and pool_points.dtype == torch.float32
                and pool_points.dim() == 2 and pool_points.shape[1] == 3):
            raise TypeError("pool_points must be a float32 CUDA [P,3] tensor")
        if not (pool_centres.is_cuda and pool_centres.dtype == torch.float32
                and pool_centres.dim() == 2 and pool_centres.shape[1] == 3):
            raise TypeError("pool_centres must be a float32 CUDA [Q,3] tensor")
        self.pts, self.ctr = pool_points.contiguous(), pool_centres.contiguous()
        self.slots = int(slots)
        self.dev = pool_points.device
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(self.slots)]
        self.bws = [lb.Workspace(self.dev) for _ in range(self.slots)]
        self.qws = [lb.Workspace(self.dev) for _ in range(self.slots)]
        self.hits_per_query = hits_per_query
        # per-slot pinned buffers, allocated once: the batch metadata sent to
        # the device and the words read back (error flag, hit bases).  A slot
        # holds one batch at a time, so reusing them never overlaps a copy.
        self.pin_meta = [torch.zeros(3 * MAX_BATCH + 3, dtype=torch.int64, pin_memory=True)
                         for _ in range(self.slots)]
        self.pin_rad = [torch.zeros(MAX_BATCH, dtype=torch.float32, pin_memory=True)
                        for _ in range(self.slots)]
        self.pin_back = [torch.zeros(2 + MAX_BATCH + 1, dtype=torch.int64, pin_memory=True)
                         for _ in range(self.slots)]
        torch.cuda.synchronize(self.dev)   # pools written before side streams read them

    def valid(self, r: Request) -> bool:
        return request_valid(r, int(self.pts.shape[0]), int(self.ctr.shape[0]))

    def submit(self, reqs, slot):
        try:
            return self._submit(reqs, slot)
        except Exception:
            # the slot goes back to the free list: let whatever was enqueued
            # before the failure finish before its buffers are reused
            self.streams[slot].synchronize()
            raise

    def ready_time(self, h):
        return None

    def stream_context(self, h):
        """The batch's stream as torch's current stream."""
        return self.torch.cuda.stream(h.stream)

    def _stage(self, reqs, prims, queries, radius_dev, ms_dev, M):
        """Copy each request's payload rows into the packed arrays."""
        a = qa = 0
        for r in reqs:
            if r.n:
                prims[a:a + r.n].copy_(self.pts[r.p_off:r.p_off + r.n], non_blocking=True)
            if r.m:
                queries[qa:qa + r.m, :3].copy_(self.ctr[r.q_off:r.q_off + r.m], non_blocking=True)
            a += r.n
            qa += r.m
        if M:
            queries[:M, 3] = self.torch.repeat_interleave(radius_dev, ms_dev, output_size=M)


class _Handle:
    """A batch in flight on one stream and, after it finishes, its resident
    trees and results."""

    def __init__(self):
        self.phase = 0
        self.ev = None
        self.pinned = None
        self.offsets = None
        self.indices = None
        self.qbase = None
        self.hits = None

    def csr(self, k, out=None):
        if self.indices is None:
            raise KeyError("results dropped (evicted or not kept)")
        a, b = self.qbase[k], self.qbase[k + 1]
        h0, h1 = int(self.hit_base[k]), int(self.hit_base[k + 1])
        if out is None:
            return self.offsets[a:b + 1] - h0, self.indices[h0:h1]
        off, idx = out
        if off.numel() != b - a + 1 or idx.numel() != h1 - h0:
            raise ValueError(f"out holds {off.numel()} offsets and {idx.numel()} indices; "
                             f"the answer has {b - a + 1} and {h1 - h0}")
        import torch
        torch.sub(self.offsets[a:b + 1], h0, out=off)
        idx.copy_(self.indices[h0:h1])
        return out

    def result_bytes(self) -> int:
        n = 0
        for t in (self.offsets, self.indices):
            if t is not None:
                n += t.numel() * t.element_size()
        return n

    def drop_results(self):
        self.offsets = self.indices = None


class GpuExecutor(_GpuBase):
    """Batched executor: a batch is packed (one copy per request payload),
    built with lbvh_build_batched and queried with the batched count and
    fill on the slot's stream.  The host waits for nothing: the total hit
    count and the build's error flag come back through pinned memory and
    are read once the stream's event has fired."""

    def footprint(self, reqs):
        lb = self.lb
        ns = [r.n for r in reqs]
        ms = [r.m for r in reqs]
        N, S, M = sum(ns), len(reqs), sum(ms)
        wb = lb.lbvh_build_batched_workspace_bytes(N, S, max(ns) if ns else 0, 63, lb.LBVH_POINTS)
        wq = lb.lbvh_query_batched_workspace_bytes(M)
        if wb < 0 or wq < 0:
            return (1 << 62, 0)
        resident = 2 * max(N, 1) * 32 + 8 * N + 4 * N + 2 * 8 * (S + 1)
        return (resident + wb + wq + _footprint_common(ns, ms, self.hits_per_query), resident)

    def _submit(self, reqs, slot):
        torch, lb = self.torch, self.lb
        if not 1 <= len(reqs) <= MAX_BATCH:
            raise ValueError(f"a batch holds 1..{MAX_BATCH} requests")
        h = _Handle()
        s = self.streams[slot]
        h.stream, h.slot = s, slot
        ns = [r.n for r in reqs]
        ms = [r.m for r in reqs]
        N, S, M = sum(ns), len(reqs), sum(ms)
        seg = [0]
        qseg = [0]
        for r in reqs:
            seg.append(seg[-1] + r.n)
            qseg.append(qseg[-1] + r.m)
        h.qbase = qseg
        host = self.pin_meta[slot][:2 * (S + 1) + S]
        host.copy_(torch.tensor(seg + qseg + ms, dtype=torch.int64))
        hrad = self.pin_rad[slot][:S]
        hrad.copy_(torch.tensor([r.radius for r in reqs], dtype=torch.float32))
        with torch.cuda.stream(s):
            meta = host.to(self.dev, non_blocking=True)
            rad = hrad.to(self.dev, non_blocking=True)
            seg_d, qseg_d, ms_d = meta[:S + 1], meta[S + 1:2 * (S + 1)], meta[2 * (S + 1):]
            prims = torch.empty((max(N, 1), 3), dtype=torch.float32, device=self.dev)
            queries = torch.empty((max(M, 1), 4), dtype=torch.float32, device=self.dev)
            self._stage(reqs, prims, queries, rad, ms_d, M)
            h.batch = lb.alloc_batch(seg_d, 63, max(ns), self.dev, total_n=N)
            lb.build_batched(prims[:max(N, 1)], seg_d, 63, max(ns), kind=lb.LBVH_POINTS,
                             workspace=self.bws[slot], batch=h.batch, stream=s)
            h.pinned = self.pin_back[slot][:2 + S + 1]
            h.pinned.zero_()
            lb._check(lb.lbvh_build_batched_status_async(
                h.batch.workspace.data_ptr(), h.batch.desc, h.pinned.data_ptr(),
                int(s.cuda_stream)), "lbvh_build_batched_status_async")
            h.offsets = lb.query_batched_count(h.batch, queries[:M], qseg_d, lb.SPHERES,
                                               self.qws[slot], stream=s)
            # per-request hit bases (offsets at the request boundaries)
            h.pinned[2:].copy_(h.offsets.index_select(0, qseg_d), non_blocking=True)
            h.queries, h.qseg_d, h.prims = queries, qseg_d, prims
            h.ev = torch.cuda.Event()
            h.ev.record(s)
        h.M = M
        return h

    def advance(self, h) -> bool:
        torch, lb = self.torch, self.lb
        if not h.ev.query():
            return False
        if h.phase == 0:
            back = h.pinned.tolist()
            h.pinned = None
            if back[0] & 0xFFFFFFFF:
                raise RuntimeError("batched build flagged a device error (LBVH_EDEVICE)")
            h.hit_base = back[2:]
            total = h.hit_base[-1]
            with torch.cuda.stream(h.stream):
                h.indices = torch.empty(max(total, 1), dtype=torch.int32, device=self.dev)
                if h.M:
                    lb.query_batched_fill(h.batch, h.queries[:h.M], h.qseg_d, lb.SPHERES, h.offsets,
                                          h.indices, self.qws[h.slot], stream=h.stream)
                h.ev = torch.cuda.Event()
                h.ev.record(h.stream)
            h.phase = 1
            return False
        h.phase = 2
        return True

    def hits(self, h):
        return [h.hit_base[k + 1] - h.hit_base[k] for k in range(len(h.qbase) - 1)]

    def release(self, h):
        # staged inputs are no longer needed; workspaces and pinned buffers
        # belong to the slot
        h.prims = h.queries = h.pinned = None

    def evict(self, h):
        h.batch = None

    def result_bytes(self, h) -> int:
        return h.result_bytes()

    def drop_results(self, h):
        h.drop_results()

    def query_resident(self, h, k, centres, radius):
        torch, lb = self.torch, self.lb
        if h.batch is None:
            raise KeyError("tree evicted")
        S = h.batch.num_scenes
        m = int(centres.shape[0])
        q = torch.empty((max(m, 1), 4), dtype=torch.float32, device=self.dev)
        q[:m, :3] = centres
        q[:m, 3] = radius
        qseg = torch.tensor([0] * (k + 1) + [m] * (S - k), dtype=torch.int64, device=self.dev)
        ws = lb.Workspace(self.dev)
        off, idx = lb.query_batched(h.batch, q[:m], qseg, lb.SPHERES, workspace=ws)
        return off, idx


class PlainExecutor(_GpuBase):
    """One request at a time with the single-tree entry points (lbvh_build,
    lbvh_query_spheres_count / _fill): the per-scene baseline."""

    def __init__(self, pool_points, pool_centres, hits_per_query: float = 8.0):
        super().__init__(pool_points, pool_centres, 1, hits_per_query)

    def footprint(self, reqs):
        lb = self.lb
        ns = [r.n for r in reqs]
        ms = [r.m for r in reqs]
        wb = sum(max(lb.lbvh_build_workspace_bytes(n, 63, lb.LBVH_POINTS), 0) for n in ns)
        wq = sum(max(lb.lbvh_query_workspace_bytes(m), 0) for m in ms)
        resident = sum(max(2 * n - 1, 0) * 32 + 8 * n + 4 * n for n in ns)
        return (resident + wb + wq + _footprint_common(ns, ms, self.hits_per_query), resident)

    def _submit(self, reqs, slot):
        torch, lb = self.torch, self.lb
        if len(reqs) != 1:
            raise ValueError("the plain executor takes one request per batch")
        r = reqs[0]
        h = _Handle()
        s = self.streams[slot]
        h.stream, h.slot = s, slot
        h.qbase = [0, r.m]
        with torch.cuda.stream(s):
            prims = torch.empty((max(r.n, 1), 3), dtype=torch.float32, device=self.dev)
            queries = torch.empty((max(r.m, 1), 4), dtype=torch.float32, device=self.dev)
            if r.n:
                prims[:r.n].copy_(self.pts[r.p_off:r.p_off + r.n], non_blocking=True)
            if r.m:
                queries[:r.m, :3].copy_(self.ctr[r.q_off:r.q_off + r.m], non_blocking=True)
                queries[:r.m, 3] = r.radius
            h.tree = lb.build(prims[:r.n], 63, kind=lb.LBVH_POINTS, workspace=self.bws[slot], stream=s)
            h.offsets = lb.query_count(h.tree, queries[:r.m], lb.SPHERES, self.qws[slot], stream=s)
            h.pinned = self.pin_back[slot][:2]
            h.pinned[1:2].copy_(h.offsets[r.m:r.m + 1], non_blocking=True)
            h.ev = torch.cuda.Event()
            h.ev.record(s)
        h.queries, h.prims, h.m = queries, prims, r.m
        return h

    def advance(self, h) -> bool:
        torch, lb = self.torch, self.lb
        if not h.ev.query():
            return False
        if h.phase == 0:
            total = int(h.pinned[1])
            h.pinned = None
            h.hit_base = [0, total]
            with torch.cuda.stream(h.stream):
                h.indices = torch.empty(max(total, 1), dtype=torch.int32, device=self.dev)
                lb.query_fill(h.tree, h.queries[:h.m], lb.SPHERES, h.indices, self.qws[h.slot],
                              stream=h.stream)
                h.ev = torch.cuda.Event()
                h.ev.record(h.stream)
            h.phase = 1
            return False
        h.phase = 2
        return True

    def hits(self, h):
        return [h.hit_base[1]]

    def release(self, h):
        h.prims = h.queries = h.pinned = None

    def evict(self, h):
        h.tree = None

    def result_bytes(self, h) -> int:
        return h.result_bytes()

    def drop_results(self, h):
        h.drop_results()

    def query_resident(self, h, k, centres, radius):
        torch, lb = self.torch, self.lb
        if h.tree is None:
            raise KeyError("tree evicted")
        m = int(centres.shape[0])
        q = torch.empty((max(m, 1), 4), dtype=torch.float32, device=self.dev)
        q[:m, :3] = centres
        q[:m, 3] = radius
        return lb.query(h.tree, q[:m], lb.SPHERES)
