"""The serving loop on the CPU: an oracle-backed executor on a virtual
clock stands in for the GPU, so admission, batching, residency, failure
handling and the alone-versus-mix property are tested without a device."""

import numpy as np
import pytest

import oracle
import workloads
from paper_2402_00665_amd import serve
from serve_fake import FakeExecutor

POOL_P, POOL_Q = 1 << 16, 4096


@pytest.fixture(scope="module")
def pools():
    return workloads.serving_pools(POOL_P, POOL_Q)


def plan_requests(rate=4000.0, seconds=0.03, m=30, lo=50, hi=3000, seed=2):
    p = workloads.serving_plan(rate, seconds, m, lo, hi, pool_points=POOL_P, pool_centres=POOL_Q,
                               seed_stream=seed)
    return [serve.Request(k, float(p["arrival"][k]), int(p["n"][k]), int(p["m"][k]),
                          int(p["p_off"][k]), int(p["q_off"][k]), float(p["radius"][k]))
            for k in range(len(p["n"]))]


def run(pools, reqs, budget=1 << 40, slots=2, max_batch=64, **kw):
    clock = serve.VirtualClock()
    ex = FakeExecutor(clock, *pools, slots=slots, **{k: v for k, v in kw.items()
                                                     if k in ("fixed", "per_point", "per_query",
                                                              "fail_submit", "fail_advance")})
    srv = serve.Server(ex, budget, max_batch=max_batch, clock=clock,
                       **{k: v for k, v in kw.items() if k in ("keep_resident", "max_batch_points",
                                                               "keep_results", "on_done")})
    return srv, ex, srv.run(reqs)


def direct(pools, r):
    """The request's answer computed straight from its definition: oracle
    tree of its points, Alg. 1 for its spheres."""
    pts, ctr = pools
    t = oracle.build(0, pts[r.p_off:r.p_off + r.n], 63)
    q = np.concatenate([ctr[r.q_off:r.q_off + r.m],
                        np.full((r.m, 1), r.radius, np.float32)], 1)
    o, i, _ = oracle.query_traverse(0, q, t)
    return o, i


def test_plan_is_seeded_and_well_formed():
    a = workloads.serving_plan(2000, 0.5, 100, pool_points=POOL_P, pool_centres=POOL_Q)
    b = workloads.serving_plan(2000, 0.5, 100, pool_points=POOL_P, pool_centres=POOL_Q)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert np.all(np.diff(a["arrival"]) > 0) and a["arrival"][-1] < 0.5
    assert np.all(a["p_off"] % 4 == 0) and np.all(a["p_off"] + a["n"] <= POOL_P)
    assert np.all(a["q_off"] + a["m"] <= POOL_Q)
    # Poisson count at rate 2000 over 0.5 s: 1000 +- a few sigma
    assert 850 < a["n"].size < 1150
    full = workloads.serving_plan()
    assert full["n"].min() >= 1000 and full["n"].max() <= 4_000_000
    # log-uniform sizes: the median is close to sqrt(lo * hi)
    assert abs(np.log(np.median(full["n"])) - 0.5 * np.log(1e3 * 4e6)) < 0.05


def test_every_request_answered_and_alone_equals_mix(pools):
    reqs = plan_requests()
    srv, ex, out = run(pools, reqs)
    assert all(o.status == serve.LBVH_OK for o in out)
    assert max(len(b[1]) for b in ex.submitted) > 1, "no batching happened"
    for r, o in zip(reqs, out):
        mo, mi = o.csr()
        _, _, alone = run(pools, [serve.Request(r.rid, 0.0, r.n, r.m, r.p_off, r.q_off, r.radius)])
        ao, ai = alone[0].csr()
        do, di = direct(pools, r)
        assert np.array_equal(mo, ao) and np.array_equal(mi, ai), f"request {r.rid}: mix != alone"
        assert np.array_equal(mo, do) and np.array_equal(mi, di), f"request {r.rid}: != oracle"
        assert o.hits == len(di)


def test_batches_hold_only_arrived_requests_in_order(pools):
    reqs = plan_requests(seed=3)
    srv, ex, out = run(pools, reqs, slots=3)
    arrival = {r.rid: r.arrival for r in reqs}
    seen = []
    for t, rids, slot in ex.submitted:
        assert all(arrival[i] <= t for i in rids)
        seen.extend(rids)
    assert seen == sorted(seen), "admission left arrival order"
    assert all(o.admitted >= o.arrival and o.done >= o.admitted for o in out)


def test_slots_bound_concurrency(pools):
    reqs = plan_requests(rate=20000, seconds=0.01, seed=4)
    for slots in (1, 2, 4):
        _, ex, out = run(pools, reqs, slots=slots, fixed=5e-3)
        assert all(o.status == serve.LBVH_OK for o in out)
        assert {s for _, _, s in ex.submitted} <= set(range(slots))


def test_budget_is_never_exceeded_and_trees_are_evicted(pools):
    reqs = plan_requests(seed=5)
    big = max(FakeExecutor(None, *pools).footprint([r])[0] for r in reqs)
    budget = 3 * big
    got = {}
    used = []
    clock = serve.VirtualClock()
    ex = FakeExecutor(clock, *pools, slots=2)

    def done(o):
        used.append(srv._used())
        got[o.rid] = tuple(a.copy() for a in o.csr())

    srv = serve.Server(ex, budget, max_batch=64, clock=clock, on_done=done)
    out = srv.run(reqs)
    assert all(o.status == serve.LBVH_OK for o in out)
    assert srv.peak_bytes <= budget and max(used) <= budget
    assert ex.evictions > 0
    assert srv.resident_bytes + srv.inflight_bytes <= budget
    # results handed to on_done are the requests' answers
    r = reqs[0]
    do, di = direct(pools, r)
    assert np.array_equal(got[r.rid][0], do) and np.array_equal(got[r.rid][1], di)


def test_kept_results_count_in_the_budget(pools):
    """Results kept on the device count in the budget, beside the resident
    trees: resident bytes are exactly the resident trees plus the kept
    results, never above the budget.  Trees are evicted before results: with
    room for every result, every tree but few is evicted and every answer
    is still there; with a budget too small for the results too, the oldest
    results go, an evicted answer raises KeyError and a kept one equals the
    oracle.  Without keeping results, only the trees count."""
    reqs = plan_requests(seed=8)
    fx = FakeExecutor(None, *pools)
    big = max(fx.footprint([r])[0] for r in reqs)
    all_results = sum(8 * (r.m + 1) + 4 * len(direct(pools, r)[1]) for r in reqs)
    cases = ((True, True, 2 * big + all_results), (True, True, 2 * big), (True, False, 2 * big),
             (False, True, 2 * big))
    for keep_results, keep_resident, budget in cases:
        srv, ex, out = run(pools, reqs, budget=budget, keep_results=keep_results,
                           keep_resident=keep_resident)
        assert all(o.status == serve.LBVH_OK for o in out)
        assert srv.peak_bytes <= budget
        trees = sum(b.tree_bytes for b, _ in srv.resident.values())
        results = sum(b.result_bytes for b in srv.kept.values())
        assert trees + results == srv.resident_bytes <= budget
        assert all(b.tree_bytes == fx.footprint(b.reqs)[1] for b, _ in srv.resident.values())
        assert all(b.result_bytes == ex.result_bytes(b.handle) > 0 for b in srv.kept.values())
        if not keep_resident:
            assert not srv.resident
        if not keep_results:
            assert not srv.kept
        if srv.kept and srv.resident:
            # trees go first: every kept result is at least as recent as the
            # oldest resident tree's batch... or older ones were kept because
            # trees were evicted instead
            assert min(srv.kept) <= min(srv.resident)
        kept = {r.rid for b in srv.kept.values() for r in b.reqs}
        if keep_results and budget > 2 * big:
            assert len(kept) == len(reqs), "results were dropped although they fit"
            assert ex.evictions > 0, "trees should have been evicted"
        for r, o in zip(reqs, out):
            if r.rid in kept:
                mo, mi = o.csr()
                do, di = direct(pools, r)
                assert np.array_equal(mo, do) and np.array_equal(mi, di)
            else:
                with pytest.raises(KeyError):
                    o.csr()

def test_resident_tree_can_be_queried_again(pools):
    reqs = plan_requests(seed=6)
    srv, ex, out = run(pools, reqs)
    pts, ctr = pools
    for r in reqs[-5:]:
        o, i = srv.query_resident(r.rid, ctr[:50], 0.05)
        t = oracle.build(0, pts[r.p_off:r.p_off + r.n], 63)
        q = np.concatenate([ctr[:50], np.full((50, 1), 0.05, np.float32)], 1)
        eo, ei, _ = oracle.query_traverse(0, q, t)
        assert np.array_equal(o, eo) and np.array_equal(i, ei)
    # with a budget that holds one batch, early trees are gone
    big = max(FakeExecutor(None, *pools).footprint([r])[0] for r in reqs)
    srv, ex, out = run(pools, reqs, budget=2 * big)
    with pytest.raises(KeyError):
        srv.query_resident(reqs[0].rid, ctr[:5], 0.05)


def test_invalid_oversize_and_deadline(pools):
    reqs = plan_requests(seed=7)[:20]
    reqs[1].n = -1                                   # invalid size
    reqs[2].p_off = POOL_P                           # payload outside the pool
    reqs[3].p_off = 2                                # misaligned points
    budget = FakeExecutor(None, *pools).footprint([serve.Request(0, 0.0, POOL_P // 2, 30)])[0]
    reqs[4].n, reqs[4].p_off = POOL_P, 0             # footprint above the whole budget
    # request 5 must be admitted within 1 us of arriving, behind a busy slot
    reqs[5].deadline = reqs[5].arrival + 1e-6
    srv, ex, out = run(pools, reqs, budget=budget, slots=1, fixed=5e-3)
    st = {o.rid: o.status for o in out}
    assert st[1] == st[2] == st[3] == serve.LBVH_EINVAL
    assert st[4] == serve.LBVH_ENOSPACE
    assert st[5] == serve.ERR_DEADLINE
    ok = [o for o in out if o.rid not in (1, 2, 3, 4, 5)]
    assert all(o.status == serve.LBVH_OK for o in ok)


@pytest.mark.parametrize("where", ["fail_submit", "fail_advance"])
def test_failed_batch_is_retried_alone(pools, where):
    reqs = plan_requests(rate=20000, seconds=0.005, seed=8)
    bad = reqs[len(reqs) // 2].rid
    srv, ex, out = run(pools, reqs, slots=1, fixed=2e-3, **{where: [bad]})
    assert max(len(b[1]) for b in ex.submitted) > 1
    for r, o in zip(reqs, out):
        if r.rid == bad:
            assert o.status == serve.ERR_EXECUTOR and "injected" in o.error
        else:
            assert o.status == serve.LBVH_OK, (r.rid, o.error)
            do, di = direct(pools, r)
            mo, mi = o.csr()
            assert np.array_equal(mo, do) and np.array_equal(mi, di)


def test_continuous_batching_beats_fifo_under_load(pools):
    """With a per-batch fixed cost (launch sequence + host) that one request
    at a time cannot amortise, FIFO falls behind the arrival rate and its
    tail grows; continuous batching keeps up."""
    reqs = plan_requests(rate=4000, seconds=0.05, seed=9)
    _, _, fifo = run(pools, reqs, slots=1, max_batch=1, fixed=4e-4)
    _, _, cont = run(pools, reqs, slots=2, max_batch=64, fixed=4e-4)
    sf, sc = serve.summarize(fifo), serve.summarize(cont)
    assert sf["ok"] == sc["ok"] == len(reqs)
    assert sc["p99_ms"] < sf["p99_ms"] and sc["p50_ms"] < sf["p50_ms"]
    for a, b in zip(fifo, cont):
        fo, fi = a.csr()
        co, ci = b.csr()
        assert np.array_equal(fo, co) and np.array_equal(fi, ci)


def test_summary_percentiles():
    out = [serve.Response(k, serve.LBVH_OK, 0.0, done=(k + 1) * 1e-3) for k in range(100)]
    s = serve.summarize(out)
    assert s["ok"] == 100 and s["p50_ms"] == pytest.approx(50.5) and s["p99_ms"] == pytest.approx(99.01)
    assert s["throughput_rps"] == pytest.approx(1000.0)


def test_run_pauses_and_restores_gc(pools):
    import gc
    reqs = plan_requests(seed=10)[:10]
    seen = []

    class Probe(FakeExecutor):
        def submit(self, reqs, slot):
            seen.append(gc.isenabled())
            return super().submit(reqs, slot)

    def go():
        clock = serve.VirtualClock()
        srv = serve.Server(Probe(clock, *pools), 1 << 40, clock=clock, pause_gc=True)
        return srv.run(reqs)

    assert gc.isenabled()
    out = go()
    assert gc.isenabled() and not any(seen) and all(o.status == serve.LBVH_OK for o in out)
    gc.disable()
    try:
        go()
        assert not gc.isenabled()   # left as it was
    finally:
        gc.enable()
