"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every build output (sorted Morton codes, leaf permutation, left children,
ropes, node boxes) and every query result (CSR offsets and indices, in
order) must be identical to the oracle's: integers bit for bit, binary32
boxes exactly (tolerance 0).  The oracle's query answers are themselves
pinned to brute force by the CPU tests.
"""

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (assert_query_equal, assert_tree_equal, gpu_build, gpu_query, host_tree,
                      say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    import paper_2402_00665_amd as lb
    return lb.Workspace()


def _parity(w: workloads.Workload, ws, queries=True):
    say(f"case {w.name}: n={w.n} m={w.m} bits={w.code_bits} kind={w.kind}")
    ref = oracle.build(w.kind, w.prims, w.code_bits)
    tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
    assert_tree_equal(tree, ref)
    if queries:
        roff, ridx, _ = oracle.query_traverse(w.qkind, w.queries, ref)
        off, idx = gpu_query(tree, w.queries, w.qkind, ws)
        assert_query_equal(off, idx, roff, ridx)
        return int(roff[-1])
    return None


def test_small_points_full_size(ws):
    hits = _parity(workloads.small_points(), ws)
    assert hits > 0


@pytest.mark.parametrize("name,scale", [("large_points", 1 / 64), ("clustered_boxes", 1 / 64),
                                        ("large_points", 1 / 1000), ("clustered_boxes", 1 / 1000)])
def test_reduced_workloads(name, scale, ws):
    _parity(workloads.by_name(name, scale), ws)


SIZES = [1, 2, 3, 5, 63, 64, 65, 127, 4095, 4096, 4097, 12289, 100003]


@pytest.mark.parametrize("bits", [30, 63])
@pytest.mark.parametrize("kind", [0, 1])
def test_sizes_kinds_bits(kind, bits, ws):
    rng = np.random.default_rng([11, kind, bits])
    for n in SIZES:
        if kind == 0:
            prims = rng.random((n, 3), dtype=np.float32)
        else:
            c = rng.random((n, 3))
            s = rng.random((n, 3)) * 0.02
            prims = np.concatenate([c - s, c + s], 1).astype(np.float32)
        q = workloads.spheres(rng.random((97, 3), dtype=np.float32), np.float32(0.1))
        _parity(workloads.Workload(f"sizes_{n}", kind, prims, bits, 0, q), ws)


@pytest.mark.parametrize("bits", [30, 63])
def test_degenerate_inputs(bits, ws):
    rng = np.random.default_rng([12, bits])
    n = 5000
    cases = {
        "all_equal": np.full((n, 3), 0.25, np.float32),
        "plane": np.concatenate([rng.random((n, 2), dtype=np.float32), np.full((n, 1), 3.0, np.float32)], 1),
        "line": np.stack([rng.random(n, dtype=np.float32)] * 3, 1),
        "grid_dups": (rng.integers(0, 4, size=(n, 3)) / 3.0).astype(np.float32),
        "negative_wide": (rng.normal(size=(n, 3)) * 1e4).astype(np.float32),
        "filled_cube": workloads.filled_cube(n, rng),
        "hollow_cube": workloads.hollow_cube(n, rng),
    }
    for name, p in cases.items():
        lo, hi = p.min(0), p.max(0)
        c = (lo + (hi - lo) * rng.random((64, 3))).astype(np.float32)
        q = workloads.spheres(c, np.float32(0.05 * float(np.max(hi - lo)) + 0.01))
        _parity(workloads.Workload(name, 0, np.ascontiguousarray(p), bits, 0, q), ws)


def test_query_edge_cases(ws):
    rng = np.random.default_rng(13)
    p = rng.random((3000, 3), dtype=np.float32)
    ref = oracle.build(0, p, 30)
    tree, _ = gpu_build(p, 0, 30, ws)
    qs = {
        "r0_on_points": workloads.spheres(p[:50], np.float32(0.0)),
        "huge": workloads.spheres(rng.random((5, 3), dtype=np.float32), np.float32(10.0)),
        "far": workloads.spheres(rng.random((5, 3), dtype=np.float32) + 5, np.float32(0.5)),
        "empty": np.zeros((0, 4), np.float32),
    }
    for name, q in qs.items():
        say(f"query case {name}")
        roff, ridx, _ = oracle.query_traverse(0, q, ref)
        off, idx = gpu_query(tree, q, 0, ws)
        assert_query_equal(off, idx, roff, ridx)
    boxes = np.concatenate([p[:20] - 0.01, p[:20] + 0.01], 1).astype(np.float32)
    roff, ridx, _ = oracle.query_traverse(1, boxes, ref)
    off, idx = gpu_query(tree, boxes, 1, ws)
    assert_query_equal(off, idx, roff, ridx)
    assert off[1] >= 1


def test_empty_tree(ws):
    import torch
    import paper_2402_00665_amd as lb
    tree = lb.build(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 30, workspace=ws)
    assert tree.n == 0
    q = workloads.spheres(np.random.default_rng(1).random((10, 3), dtype=np.float32), np.float32(1))
    off, idx = gpu_query(tree, q, 0, ws)
    assert off.tolist() == [0] * 11 and idx.size == 0


def test_repeated_builds_are_identical(ws):
    """Alg. 4's schedule differs run to run; the tree must not."""
    w = workloads.clustered(1 << 17, 1)
    tree, dev = gpu_build(w.prims, w.kind, w.code_bits, ws)
    first = tree.nodes.clone()
    import paper_2402_00665_amd as lb
    import torch
    for r in range(20):
        tree = lb.build(dev, w.code_bits, kind=w.kind, workspace=ws, tree=tree)
        torch.cuda.synchronize()
        assert torch.equal(tree.nodes, first), f"build {r} differs"
    lb.check_build(tree)


def test_workspace_reuse_across_sizes(ws):
    rng = np.random.default_rng(14)
    for n in (70000, 1000, 33333):
        p = rng.random((n, 3), dtype=np.float32)
        ref = oracle.build(0, p, 63)
        tree, _ = gpu_build(p, 0, 63, ws)
        assert_tree_equal(tree, ref)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["large_points", "clustered_boxes"])
def test_full_size(name, ws):
    """Full-size workloads with the default launch shapes: every build
    output and every query result."""
    say(f"full-size {name}: generating")
    w = workloads.by_name(name)
    _parity(w, ws)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["large_points", "clustered_boxes"])
def test_full_size_autotuned(name, ws):
    """Full-size workloads in the launch configuration the benchmark times:
    the autotuner's picks for this workload (radix tile shape, query split
    levels and leaf schedule), then every build output and query result."""
    import torch
    import paper_2402_00665_amd as lb
    from paper_2402_00665_amd import autotune
    w = workloads.by_name(name)
    knobs = ("sort_variant32", "sort_variant64", "query_split1", "query_split2", "query_leaf_mode",
             "query_order", "radix_bits32", "radix_bits64", "radix_mode")
    old = {k: lb.lbvh_tune(k) for k in knobs}
    try:
        p = torch.from_numpy(w.prims).cuda()
        t = autotune.tune(p, w.code_bits, kind=w.kind, reps=2, save=False)
        for k, v in t["knobs"].items():
            lb.lbvh_tune(k, v)
        tree = lb.build(p, w.code_bits, kind=w.kind)
        tq = autotune.tune_query(tree, torch.from_numpy(w.queries).cuda(), w.qkind, reps=1,
                                 save=False)
        for k, v in zip(knobs[2:6], tq["value"]):
            lb.lbvh_tune(k, v)
        say(f"full-size {name}, tuned: {t['knobs']} query={tq['value']}")
        del tree, p
        _parity(w, ws)
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)


def test_large_queries_all_hit_ranges(ws):
    """Query boxes and spheres big enough to contain whole subtrees spanning
    many 4096- and 128-leaf blocks (the all-hit pieces)."""
    rng = np.random.default_rng(16)
    w = workloads.clustered(1 << 18, 1)
    ref = oracle.build(w.kind, w.prims, w.code_bits)
    tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
    c = rng.random((40, 3))
    s = rng.random((40, 3)) * 0.4
    boxes = np.concatenate([c - s, c + s], 1).astype(np.float32)
    roff, ridx, _ = oracle.query_traverse(1, boxes, ref)
    off, idx = gpu_query(tree, boxes, 1, ws)
    assert_query_equal(off, idx, roff, ridx)
    assert roff[-1] > 1 << 18
    sph = workloads.spheres(rng.random((40, 3), dtype=np.float32), np.float32(0.3))
    roff, ridx, _ = oracle.query_traverse(0, sph, ref)
    off, idx = gpu_query(tree, sph, 0, ws)
    assert_query_equal(off, idx, roff, ridx)


def test_piece_capacity_overflow_passes_through(ws):
    """16 queries that each cover all 2^20 leaves need more pieces than the
    workspace holds at both split levels; the levels pass pieces through
    unsplit and the results stay exact."""
    rng = np.random.default_rng(17)
    p = rng.random((1 << 20, 3), dtype=np.float32)
    ref = oracle.build(0, p, 30)
    tree, _ = gpu_build(p, 0, 30, ws)
    q = workloads.spheres(rng.random((16, 3), dtype=np.float32), np.float32(2.0))
    roff, ridx, _ = oracle.query_traverse(0, q, ref)
    off, idx = gpu_query(tree, q, 0, ws)
    assert_query_equal(off, idx, roff, ridx)
    assert roff[-1] == 16 << 20
    # a mix: most queries light, a few cover everything
    q2 = workloads.spheres(rng.random((600, 3), dtype=np.float32), np.float32(0.01))
    q2[::97, 3] = 2.0
    roff, ridx, _ = oracle.query_traverse(0, q2, ref)
    off, idx = gpu_query(tree, q2, 0, ws)
    assert_query_equal(off, idx, roff, ridx)


@pytest.mark.parametrize("variant", range(9))
def test_sort_tile_variants(variant, ws):
    """Every radix-pass tile shape, with every digit width (8 or 10 bits for
    30-bit codes, 8, 9 or 11 for 63-bit), in both pass forms (onesweep, and
    count + scatter), gives the same tree (tolerance 0).  Sizes span one
    tile, several tiles (and chunks of tiles) with a ragged tail, and odd
    and even pass counts."""
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng([18, variant])
    old = {k: lb.lbvh_tune(k) for k in ("sort_variant32", "sort_variant64", "radix_bits32",
                                        "radix_bits64", "radix_mode")}
    lb.lbvh_tune("sort_variant32", variant)
    lb.lbvh_tune("sort_variant64", variant)
    try:
        cases = [(100003, 30), (100003, 63), (4097, 30), (300, 63), (1 << 18, 30), (40000, 63),
                 (1 << 20, 30)]
        pts = {n: rng.random((n, 3), dtype=np.float32) for n, _ in cases}
        refs = {(n, b): oracle.build(0, pts[n], b) for n, b in cases}
        for mode in (0, 1):
            lb.lbvh_tune("radix_mode", mode)
            for b32, b64 in ((8, 8), (10, 9), (10, 11)):
                lb.lbvh_tune("radix_bits32", b32)
                lb.lbvh_tune("radix_bits64", b64)
                for n, bits in cases:
                    say(f"  mode {mode}, digits {b32 if bits == 30 else b64} bits, n {n}")
                    tree, _ = gpu_build(pts[n], 0, bits, ws)
                    assert_tree_equal(tree, refs[(n, bits)])
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)


def test_sort_digit_widths_duplicates_and_clusters(ws):
    """Clustered boxes with heavy duplicate codes and all-equal codes sort
    stably under every digit width, in both pass forms."""
    import paper_2402_00665_amd as lb
    old = {k: lb.lbvh_tune(k) for k in ("radix_bits32", "radix_bits64", "radix_mode")}
    try:
        rng = workloads._rng(3, 0)
        boxes = workloads.clustered_boxes(150000, rng)
        same = np.repeat(rng.random((1, 3), dtype=np.float32), 9000, axis=0)
        refs = {(k, b): oracle.build(k, p, b) for k, p in ((1, boxes), (0, same)) for b in (30, 63)}
        for mode in (0, 1):
            lb.lbvh_tune("radix_mode", mode)
            for b32, b64 in ((8, 8), (10, 9), (10, 11)):
                lb.lbvh_tune("radix_bits32", b32)
                lb.lbvh_tune("radix_bits64", b64)
                for (k, b), ref in refs.items():
                    tree, _ = gpu_build(boxes if k == 1 else same, k, b, ws)
                    assert_tree_equal(tree, ref)
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)


@pytest.mark.parametrize("split1,split2,leaf_mode,order", [
    (12, 7, 1, 0), (11, 6, 1, 0), (9, 4, 0, 0), (14, 9, 1, 0), (8, 12, 0, 0), (10, 10, 1, 0),
    (6, 3, 0, 0), (12, 7, 0, 1), (12, 6, 1, 1), (8, 12, 0, 1), (6, 3, 0, 1), (24, 24, 0, 1),
    (24, 6, 1, 0)])
def test_query_schedules(split1, split2, leaf_mode, order, ws):
    """Every query schedule (split block sizes, leaf mode, query order) gives
    the oracle's results exactly: dense box queries, sparse spheres, all-hit
    ranges.  Also a second level no finer than the first (one piece per
    item), blocks larger than the tree (one unsplit walk per query), and
    blocks small enough that the levels overflow and pass their items
    through."""
    import paper_2402_00665_amd as lb
    old = [lb.lbvh_tune("query_split1", split1), lb.lbvh_tune("query_split2", split2),
           lb.lbvh_tune("query_leaf_mode", leaf_mode), lb.lbvh_tune("query_order", order)]
    try:
        for name in ("clustered_boxes", "large_points"):
            _parity(workloads.by_name(name, 1 / 64), ws)
        rng = np.random.default_rng([19, split1, split2, leaf_mode, order])
        w = workloads.clustered(1 << 17, 1)
        ref = oracle.build(w.kind, w.prims, w.code_bits)
        tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
        c = rng.random((60, 3))
        s = rng.random((60, 3)) * 0.3
        boxes = np.concatenate([c - s, c + s], 1).astype(np.float32)
        roff, ridx, _ = oracle.query_traverse(1, boxes, ref)
        off, idx = gpu_query(tree, boxes, 1, ws)
        assert_query_equal(off, idx, roff, ridx)
    finally:
        lb.lbvh_tune("query_split1", old[0])
        lb.lbvh_tune("query_split2", old[1])
        lb.lbvh_tune("query_leaf_mode", old[2])
        lb.lbvh_tune("query_order", old[3])


def test_query_order_edge_cases(ws):
    """Queries processed in Morton order ("query_order" = 1) give the
    caller-order CSR of the oracle exactly: query counts around the sort's
    2048-key tile (one tile, a ragged second tile, several tiles), queries
    outside the scene box, a NaN query, a one-leaf tree, split levels that
    overflow, and a fill enqueued after the knob was switched back (the
    fill follows what the count call did)."""
    import torch
    import paper_2402_00665_amd as lb
    old = lb.lbvh_tune("query_order", 1)
    try:
        rng = np.random.default_rng(41)
        for bits in (30, 63):
            p = rng.random((50000, 3), dtype=np.float32)
            ref = oracle.build(0, p, bits)
            tree, _ = gpu_build(p, 0, bits, ws)
            for m in (1, 2, 3, 2047, 2048, 2049, 10007):
                c = (rng.random((m, 3)) * 1.4 - 0.2).astype(np.float32)   # some outside
                q = workloads.spheres(c, np.float32(0.03))
                if m > 2:
                    q[m // 2, 0] = np.nan
                roff, ridx, _ = oracle.query_traverse(0, q, ref)
                off, idx = gpu_query(tree, q, 0, ws)
                assert_query_equal(off, idx, roff, ridx)
            s = rng.random((777, 3)) * 0.1
            boxes = np.concatenate([c[:777] - s, c[:777] + s], 1).astype(np.float32)
            roff, ridx, _ = oracle.query_traverse(1, boxes, ref)
            off, idx = gpu_query(tree, boxes, 1, ws)
            assert_query_equal(off, idx, roff, ridx)
        # one leaf
        p1 = rng.random((1, 3), dtype=np.float32)
        ref1 = oracle.build(0, p1, 30)
        tree1, _ = gpu_build(p1, 0, 30, ws)
        q1 = workloads.spheres(rng.random((300, 3), dtype=np.float32), np.float32(0.5))
        roff, ridx, _ = oracle.query_traverse(0, q1, ref1)
        off, idx = gpu_query(tree1, q1, 0, ws)
        assert_query_equal(off, idx, roff, ridx)
        # split levels overflow: a few queries cover all 2^20 leaves
        p2 = rng.random((1 << 20, 3), dtype=np.float32)
        ref2 = oracle.build(0, p2, 30)
        tree2, _ = gpu_build(p2, 0, 30, ws)
        q2 = workloads.spheres(rng.random((600, 3), dtype=np.float32), np.float32(0.01))
        q2[::97, 3] = 2.0
        roff, ridx, _ = oracle.query_traverse(0, q2, ref2)
        off, idx = gpu_query(tree2, q2, 0, ws)
        assert_query_equal(off, idx, roff, ridx)
        # count reordered, knob switched off, then fill
        dq = torch.from_numpy(q2).cuda()
        qws = lb.Workspace()
        offt = lb.query_count(tree2, dq, 0, qws)
        lb.lbvh_tune("query_order", 0)
        total = int(offt[-1].item())
        idxt = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        lb.query_fill(tree2, dq, 0, idxt, qws)
        torch.cuda.synchronize()
        assert_query_equal(offt.cpu().numpy(), idxt[:total].cpu().numpy(), roff, ridx)
    finally:
        lb.lbvh_tune("query_order", old)


@pytest.mark.parametrize("bits", [30, 63])
@pytest.mark.parametrize("kind", [0, 1])
def test_non_finite_inputs_give_a_well_formed_tree(kind, bits, ws):
    """NaN and infinite coordinates: the tree's structure stays valid (a
    permutation of the leaves, every link a node id, a preorder walk over
    ropes and left children visits every leaf once), and queries run."""
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng([26, kind, bits])
    n = 20000
    p = rng.random((n, 3 if kind == 0 else 6), dtype=np.float32)
    if kind == 1:
        p[:, 3:] = p[:, :3] + 0.01
    bad = rng.choice(n, 300, replace=False)
    p[bad[:100], 0] = np.nan
    p[bad[100:200], 1] = np.inf
    p[bad[200:], 2] = -np.inf
    tree, _ = gpu_build(p, kind, bits, ws)
    lb.check_build(tree)
    _, perm, left, rope, _ = host_tree(tree)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.all((left >= 0) & (left < 2 * n - 1))
    assert np.all((rope >= -1) & (rope < 2 * n - 1))
    # Alg. 1 with every test passing visits each leaf once, in order
    seen, v = [], 0
    while v != -1 and len(seen) <= n:
        if v >= n - 1:
            seen.append(v - (n - 1))
            v = rope[v]
        else:
            v = left[v]
    assert seen == list(range(n))
    q = workloads.spheres(rng.random((500, 3), dtype=np.float32), np.float32(0.05))
    off, idx = gpu_query(tree, q, 0, ws)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and np.all((idx >= 0) & (idx < n))


@pytest.mark.parametrize("order", [0, 1])
def test_graph_capture_single_tree(order, ws):
    """Build, count and fill of one tree enqueue kernels only (no memset, no
    host synchronisation), so they can be captured in a HIP graph; every
    replay, with eager work between replays, reproduces the eager bits.
    Also with the queries walked in Morton order."""
    import paper_2402_00665_amd as lb
    old_order = lb.lbvh_tune("query_order", order)
    try:
        _graph_capture_single_tree()
    finally:
        lb.lbvh_tune("query_order", old_order)


def _graph_capture_single_tree():
    import torch
    import paper_2402_00665_amd as lb
    w = workloads.by_name("clustered_boxes", 1 / 64)
    dp = torch.from_numpy(w.prims).cuda()
    dq = torch.from_numpy(w.queries).cuda()
    bws, qws = lb.Workspace(), lb.Workspace()
    tree = lb.build(dp, w.code_bits, kind=w.kind, workspace=bws)
    off, idx = lb.query(tree, dq, w.qkind, workspace=qws)
    torch.cuda.synchronize()
    total = int(off[-1].item())
    assert total > 0
    eager_nodes, eager_off, eager_idx = tree.nodes.clone(), off.clone(), idx.clone()
    offsets = torch.empty_like(off)
    indices = torch.empty(total, dtype=torch.int32, device="cuda")

    def enqueue():
        lb.build(dp, w.code_bits, kind=w.kind, workspace=bws, tree=tree)
        lb.query_count(tree, dq, w.qkind, qws, offsets=offsets)
        lb.query_fill(tree, dq, w.qkind, indices, qws)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            enqueue()
    torch.cuda.synchronize()
    for r in range(4):
        tree.nodes.zero_()
        offsets.zero_()
        indices.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(tree.nodes, eager_nodes), f"replay {r}: nodes differ"
        assert torch.equal(offsets, eager_off), f"replay {r}: offsets differ"
        assert torch.equal(indices, eager_idx), f"replay {r}: indices differ"
        x = torch.rand(1000, device="cuda").sum()   # eager work between replays
        x.item()
    lb.check_build(tree)


@pytest.mark.parametrize("order", [0, 1])
def test_query_error_word(order, ws):
    """A count call clears its error word (lbvh_query_check is OK after a
    clean call, also after a flagged one); a walk budget capped from the
    host (knob query_walk_budget) is reported as LBVH_EDEVICE, and the fill
    that follows still writes only inside the counted slots."""
    import torch
    import paper_2402_00665_amd as lb
    w = workloads.by_name("clustered_boxes", 1 / 256)
    ref = oracle.build(w.kind, w.prims, w.code_bits)
    tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
    q = torch.from_numpy(w.queries[:20000]).cuda()
    qws = lb.Workspace()
    old = {k: lb.lbvh_tune(k) for k in ("query_order", "query_walk_budget")}
    lb.lbvh_tune("query_order", order)
    try:
        off = lb.query_count(tree, q, w.qkind, qws)
        lb.check_query(qws, q.shape[0])
        say("  capped walk budget: expect the error word")
        lb.lbvh_tune("query_walk_budget", 3)
        off = lb.query_count(tree, q, w.qkind, qws)
        with pytest.raises(lb.LbvhError) as e:
            lb.check_query(qws, q.shape[0])
        assert e.value.status == lb.LBVH_EDEVICE
        total = int(off[-1].item())
        guard = 4096
        buf = torch.full((total + guard,), -7, dtype=torch.int32, device="cuda")
        lb.query_fill(tree, q, w.qkind, buf, qws)
        torch.cuda.synchronize()
        assert bool((buf[total:] == -7).all()), "fill wrote past the counted hits"
        lb.lbvh_tune("query_walk_budget", 0)
        roff, ridx, _ = oracle.query_traverse(w.qkind, w.queries[:20000], ref)
        off2, idx2 = lb.query(tree, q, w.qkind, workspace=qws)
        lb.check_query(qws, q.shape[0])
        assert_query_equal(off2.cpu().numpy(), idx2.cpu().numpy(), roff, ridx)
        # an empty query set clears the word too
        lb.lbvh_tune("query_walk_budget", 3)
        lb.query_count(tree, q, w.qkind, qws)
        lb.lbvh_tune("query_walk_budget", 0)
        lb.query_count(tree, q[:0], w.qkind, qws)
        lb.check_query(qws, 0)
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)
