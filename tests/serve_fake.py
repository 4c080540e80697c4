"""Host-side executor for the serving loop's CPU tests: the oracle does the
work (per scene, on the same packed arrays the GPU executor builds) and a
linear cost model gives each batch a duration on a virtual clock."""

import numpy as np

import oracle


class FakeHandle:
    def __init__(self):
        self.evicted = False
        self.released = False

    def csr(self, k):
        if self.indices is None:
            raise KeyError("results dropped")
        a, b = self.qbase[k], self.qbase[k + 1]
        h0, h1 = int(self.offsets[a]), int(self.offsets[b])
        return self.offsets[a:b + 1] - h0, self.indices[h0:h1]


class FakeExecutor:
    """slots batches in flight at once; a batch of N points and M queries
    takes fixed + per_point*N + per_query*M virtual seconds.  Requests whose
    rid is in ``fail_submit`` make submit raise; in ``fail_advance`` make the
    batch fail while in flight."""

    def __init__(self, clock, pool_points, pool_centres, slots=2, fixed=1e-3, per_point=2e-9,
                 per_query=1e-8, fail_submit=(), fail_advance=()):
        self.clock = clock
        self.pts, self.ctr = pool_points, pool_centres
        self.slots = slots
        self.fixed, self.per_point, self.per_query = fixed, per_point, per_query
        self.fail_submit, self.fail_advance = set(fail_submit), set(fail_advance)
        self.submitted = []       # (time, [rids], slot)
        self.evictions = 0
        self.busy_slots = set()

    def valid(self, r):
        from paper_2402_00665_amd.serve import request_valid
        return request_valid(r, self.pts.shape[0], self.ctr.shape[0])

    def footprint(self, reqs):
        N = sum(r.n for r in reqs)
        M = sum(r.m for r in reqs)
        S = len(reqs)
        resident = 76 * N + 16 * (S + 1)
        return (resident + 40 * N + 64 * M + 12 * N + 16 * M + 8 * (M + S) + 32 * M, resident)

    def submit(self, reqs, slot):
        assert slot not in self.busy_slots, "slot handed out twice"
        if any(r.rid in self.fail_submit for r in reqs):
            raise RuntimeError("injected submit failure")
        self.busy_slots.add(slot)
        self.submitted.append((self.clock.now(), [r.rid for r in reqs], slot))
        h = FakeHandle()
        h.slot = slot
        h.reqs = reqs
        # pack exactly as the GPU executor does, then run the oracle per scene
        seg, qseg = [0], [0]
        for r in reqs:
            seg.append(seg[-1] + r.n)
            qseg.append(qseg[-1] + r.m)
        pts = np.concatenate([self.pts[r.p_off:r.p_off + r.n] for r in reqs] + [np.zeros((0, 3), np.float32)])
        q = np.zeros((qseg[-1], 4), np.float32)
        for k, r in enumerate(reqs):
            q[qseg[k]:qseg[k + 1], :3] = self.ctr[r.q_off:r.q_off + r.m]
            q[qseg[k]:qseg[k + 1], 3] = np.float32(r.radius)
        offs, idxs, h.trees = [np.zeros(1, np.int64)], [], []
        for k in range(len(reqs)):
            t = oracle.build(0, pts[seg[k]:seg[k + 1]], 63)
            o, i, _ = oracle.query_traverse(0, q[qseg[k]:qseg[k + 1]], t)
            offs.append(o[1:] + offs[-1][-1])
            idxs.append(i)
            h.trees.append(t)
        h.offsets = np.concatenate(offs)
        h.indices = np.concatenate(idxs + [np.zeros(0, np.int32)])
        h.qbase = qseg
        h.done_at = self.clock.now() + self.fixed + self.per_point * seg[-1] + self.per_query * qseg[-1]
        return h

    def advance(self, h):
        if self.clock.now() < h.done_at:
            return False
        if any(r.rid in self.fail_advance for r in h.reqs):
            self.busy_slots.discard(h.slot)
            raise RuntimeError("injected device failure")
        self.busy_slots.discard(h.slot)
        return True

    def ready_time(self, h):
        return h.done_at

    def stream_context(self, h):
        import contextlib
        return contextlib.nullcontext()

    def hits(self, h):
        return [int(h.offsets[h.qbase[k + 1]] - h.offsets[h.qbase[k]]) for k in range(len(h.reqs))]

    def release(self, h):
        h.released = True

    def evict(self, h):
        if not h.evicted:
            self.evictions += 1
        h.evicted = True

    def result_bytes(self, h):
        return 0 if h.indices is None else h.offsets.nbytes + h.indices.nbytes

    def drop_results(self, h):
        h.offsets = h.indices = None

    def query_resident(self, h, k, centres, radius):
        if h.evicted:
            raise KeyError("tree evicted")
        q = np.concatenate([centres, np.full((centres.shape[0], 1), radius, np.float32)], 1)
        o, i, _ = oracle.query_traverse(0, q, h.trees[k])
        return o, i
