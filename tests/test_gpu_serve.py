"""The serving loop on the GPU: every request's answer must be the same in
the mix (continuous batching over several streams), alone, and through the
plain one-request-at-a-time path, and a sample must equal the oracle."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import say

pytestmark = pytest.mark.gpu

POOL_P, POOL_Q = 1 << 22, 1 << 16


@pytest.fixture(scope="module")
def pools():
    import torch
    p, c = workloads.serving_pools(POOL_P, POOL_Q)
    return p, c, torch.from_numpy(p).cuda(), torch.from_numpy(c).cuda()


def requests(seed=2, rate=20000.0, seconds=0.02, m=1000, lo=1e3, hi=2e5):
    from paper_2402_00665_amd import serve
    p = workloads.serving_plan(rate, seconds, m, lo, hi, pool_points=POOL_P, pool_centres=POOL_Q,
                               seed_stream=seed)
    return [serve.Request(k, float(p["arrival"][k]), int(p["n"][k]), int(p["m"][k]),
                          int(p["p_off"][k]), int(p["q_off"][k]), float(p["radius"][k]))
            for k in range(len(p["n"]))]


def serve_run(pools, reqs, batched=True, budget=64 << 30, slots=3):
    import torch
    from paper_2402_00665_amd import serve
    ex = (serve.GpuExecutor(pools[2], pools[3], slots=slots) if batched
          else serve.PlainExecutor(pools[2], pools[3]))
    srv = serve.Server(ex, budget, max_batch=64 if batched else 1)
    out = srv.run(reqs)
    torch.cuda.synchronize()
    return srv, out


def same(a, b):
    import torch
    ao, ai = a.csr()
    bo, bi = b.csr()
    return bool(torch.equal(ao, bo)) and bool(torch.equal(ai, bi))


def test_mix_alone_plain_and_oracle(pools):
    from paper_2402_00665_amd import serve
    reqs = requests()
    say(f"serving: {len(reqs)} requests, mixed")
    srv, mix = serve_run(pools, reqs)
    assert all(o.status == serve.LBVH_OK for o in mix), [o.error for o in mix if o.status][:3]
    sizes = [b[1] for b in srv.batches]
    say(f"  batches: {len(sizes)}, largest {max(sizes)}, summary {serve.summarize(mix)}")
    assert max(sizes) > 1
    say("serving: plain FIFO")
    _, plain = serve_run(pools, reqs, batched=False)
    bad = [r.rid for r, a, b in zip(reqs, mix, plain) if not same(a, b)]
    assert not bad, f"mix differs from plain for requests {bad[:10]}"
    say("serving: alone")
    for r in reqs[:: max(1, len(reqs) // 25)]:
        _, alone = serve_run(pools, [serve.Request(r.rid, 0.0, r.n, r.m, r.p_off, r.q_off, r.radius)])
        assert same(alone[0], mix[r.rid]), f"request {r.rid}: alone != mix"
    say("serving: oracle sample")
    pts, ctr = pools[0], pools[1]
    for r in sorted(reqs, key=lambda r: r.n)[:: max(1, len(reqs) // 6)]:
        t = oracle.build(0, pts[r.p_off:r.p_off + r.n], 63)
        q = np.concatenate([ctr[r.q_off:r.q_off + r.m], np.full((r.m, 1), r.radius, np.float32)], 1)
        eo, ei, _ = oracle.query_traverse(0, q, t)
        go, gi = mix[r.rid].csr()
        assert np.array_equal(go.cpu().numpy(), eo) and np.array_equal(gi.cpu().numpy(), ei), \
            f"request {r.rid} (n={r.n}) differs from the oracle"
        assert mix[r.rid].hits == len(ei)


def test_tight_budget_and_resident_queries(pools):
    import torch
    from paper_2402_00665_amd import serve
    reqs = requests(seed=3, seconds=0.01)
    _, ref = serve_run(pools, reqs)
    ex = serve.GpuExecutor(pools[2], pools[3], slots=2)
    big = max(ex.footprint([r])[0] for r in reqs)
    got = {}

    def done(o):   # results as they finish (the server may evict its copy)
        off, idx = o.csr()
        got[o.rid] = (off.cpu(), idx.cpu())

    srv = serve.Server(ex, 2 * big, on_done=done)
    out = srv.run(reqs)
    torch.cuda.synchronize()
    say(f"  tight budget {2 * big >> 20} MiB: peak {srv.peak_bytes >> 20} MiB, "
        f"{len(srv.batches)} batches, resident {len(srv.resident)}")
    assert all(o.status == serve.LBVH_OK for o in out)
    assert srv.peak_bytes <= 2 * big
    for a in ref:
        ao, ai = a.csr()
        go, gi = got[a.rid]
        assert torch.equal(ao.cpu(), go) and torch.equal(ai.cpu(), gi), f"request {a.rid}"
    # results kept on the device count in the budget: only the batches the
    # server still keeps results for hold theirs
    kept = {r.rid for b in srv.kept.values() for r in b.reqs}
    for o in out:
        if o.rid not in kept:
            with pytest.raises(KeyError):
                o.csr()
    # the last request's tree is resident: its own queries give its answer again
    r = reqs[-1]
    centres = pools[3][r.q_off:r.q_off + r.m]
    o, i = srv.query_resident(r.rid, centres, r.radius)
    go, gi = got[r.rid]
    assert torch.equal(o.cpu(), go) and torch.equal(i.cpu(), gi)
    with pytest.raises(KeyError):
        srv.query_resident(reqs[0].rid, centres, r.radius)


def test_oracle_sample_across_the_size_range(pools):
    """A seeded set of requests whose sizes span the serving stream's whole
    range (log-uniform in [1e3, 4e6] points, 10^4 spheres with about 8
    expected neighbours each), served together; every answer equals the
    oracle's."""
    import math
    from paper_2402_00665_amd import serve
    rng = np.random.default_rng([5, 77])
    k = 16
    ns = np.floor(np.exp(np.linspace(math.log(1e3), math.log(4e6), k))).astype(np.int64)
    ns = rng.permutation(ns)
    reqs = []
    for j, n in enumerate(ns):
        p_off = int(rng.integers(0, (POOL_P - int(n)) // 4 + 1)) * 4
        q_off = int(rng.integers(0, POOL_Q - 10000 + 1))
        reqs.append(serve.Request(j, 0.0, int(n), 10000, p_off, q_off,
                                  workloads.neighbour_radius(int(n), 8.0)))
    say(f"serving: {k} requests, n from {ns.min()} to {ns.max()}")
    srv, out = serve_run(pools, reqs)
    assert all(o.status == serve.LBVH_OK for o in out), [o.error for o in out if o.status][:3]
    pts, ctr = pools[0], pools[1]
    oracle.threads(16)
    try:
        for r in reqs:
            t = oracle.build(0, pts[r.p_off:r.p_off + r.n], 63)
            q = np.concatenate([ctr[r.q_off:r.q_off + r.m],
                                np.full((r.m, 1), r.radius, np.float32)], 1)
            eo, ei, _ = oracle.query_traverse(0, q, t)
            go, gi = out[r.rid].csr()
            assert np.array_equal(go.cpu().numpy(), eo) and np.array_equal(gi.cpu().numpy(), ei), \
                f"request {r.rid} (n={r.n}) differs from the oracle"
            assert out[r.rid].hits == len(ei)
    finally:
        oracle.threads(1)


def test_hand_over_into_caller_buffers(pools):
    """Answers copied by on_done into caller-owned buffers (nothing kept by
    the server) equal the answers the server keeps."""
    import torch
    from paper_2402_00665_amd import serve
    reqs = requests(seed=4, seconds=0.01)
    _, ref = serve_run(pools, reqs)
    M = sum(r.m for r in reqs)
    offs = torch.empty(M + len(reqs), dtype=torch.int64, device="cuda")
    idx = torch.full((16 * M,), -1, dtype=torch.int32, device="cuda")
    where, pos = {}, [0, 0]

    def done(o):
        r = reqs[o.rid]
        a, b = pos
        where[o.rid] = (a, b, o.hits)
        pos[0], pos[1] = a + r.m + 1, b + o.hits
        assert b + o.hits <= idx.numel()
        got = o.csr(out=(offs[a:a + r.m + 1], idx[b:b + o.hits]))
        assert got[0].data_ptr() == offs[a:].data_ptr()

    ex = serve.GpuExecutor(pools[2], pools[3], slots=3)
    srv = serve.Server(ex, 64 << 30, keep_results=False, on_done=done)
    out = srv.run(reqs)
    torch.cuda.synchronize()
    assert all(o.status == serve.LBVH_OK for o in out)
    assert not srv.kept
    for a in ref:
        ao, ai = a.csr()
        p, q, h = where[a.rid]
        assert torch.equal(ao, offs[p:p + ao.numel()]) and torch.equal(ai, idx[q:q + h]), a.rid
    with pytest.raises(ValueError):   # buffers of the wrong size
        ref[0].csr(out=(offs[:1], idx[:1]))
