"""Pins of the oracle's scene box, Morton codes, sort and range queries.

Morton codes have no printed example in the paper (Sec. 3.1 only names the
step), so they are pinned by closed forms: dyadic grids where every float32
operation is exact and the expected code can be spelled out bit by bit as a
string, the scene corners, axis order, flat axes, monotonicity, and agreement
with an exact float64 computation away from cell boundaries.  The sort is
pinned by numpy's stable argsort; queries by brute force, by a stack-based
depth-first walk and by float64 distances away from the sphere surface.
"""

import numpy as np
import pytest

import oracle
import workloads


def string_interleave(qx, qy, qz, b):
    bx, by, bz = (format(q, f"0{b}b") for q in (qx, qy, qz))
    return int("".join(x + y + z for x, y, z in zip(bx, by, bz)), 2)


def deinterleave(code, b):
    q = [0, 0, 0]
    for k in range(b):
        for a in range(3):
            q[a] |= ((int(code) >> (3 * k + 2 - a)) & 1) << k
    return q


# ------------------------------------------------------------ scene / sort

@pytest.mark.parametrize("kind", [0, 1])
def test_scene_box_is_min_max(kind):
    rng = np.random.default_rng(3)
    if kind == 0:
        p = rng.normal(size=(1000, 3)).astype(np.float32)
        ref = np.concatenate([p.min(0), p.max(0)])
    else:
        c = rng.normal(size=(1000, 3))
        p = np.concatenate([c - 0.1, c + 0.3], 1).astype(np.float32)
        ref = np.concatenate([p[:, :3].min(0), p[:, 3:].max(0)])
    assert np.array_equal(oracle.scene_box(kind, p), ref)


def test_sort_is_stable_argsort():
    rng = np.random.default_rng(4)
    codes = rng.integers(0, 50, size=5000).astype(np.uint64)
    s, perm = oracle.sort(codes)
    ref = np.argsort(codes, kind="stable")
    assert np.array_equal(perm, ref) and np.array_equal(s, codes[ref])


# ----------------------------------------------------------------- Morton

@pytest.mark.parametrize("bits", [30, 63])
def test_morton_dyadic_grid_exact(bits):
    """Scene [0,1]^3: scale = 2^b exactly, c = k/2^b gives q = k exactly."""
    b = bits // 3
    rng = np.random.default_rng(bits)
    k = rng.integers(0, 1 << b, size=(500, 3))
    pts = (k / float(1 << b)).astype(np.float32)
    pts = np.concatenate([pts, [[0, 0, 0], [1, 1, 1]]]).astype(np.float32)
    codes = oracle.morton(0, pts, bits)
    for j in range(500):
        assert int(codes[j]) == string_interleave(*map(int, k[j]), b)
    assert int(codes[500]) == 0
    assert int(codes[501]) == (1 << (3 * b)) - 1          # upper corner clamps


@pytest.mark.parametrize("bits", [30, 63])
def test_morton_just_below_cell_boundary(bits):
    b = bits // 3
    k = np.array([1, 7, 1 << (b - 1)], np.float64)
    c = np.nextafter((k / float(1 << b)).astype(np.float32), np.float32(0))
    pts = np.stack([c, np.zeros(3, np.float32), np.zeros(3, np.float32)], 1)
    pts = np.concatenate([pts, [[1, 1, 1], [0, 0, 0]]]).astype(np.float32)
    codes = oracle.morton(0, pts, bits)
    for j in range(3):
        assert deinterleave(codes[j], b)[0] == int(k[j]) - 1


def test_morton_axis_order_and_flat_axis():
    pts = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 0]], np.float32)
    codes = oracle.morton(0, pts, 30)
    x_bits = sum(1 << (3 * k + 2) for k in range(10))
    assert int(codes[0]) == x_bits
    assert int(codes[1]) == x_bits >> 1
    assert int(codes[2]) == x_bits >> 2
    flat = np.array([[0, 0, 5], [1, 1, 5], [0.5, 0.25, 5]], np.float32)
    c = oracle.morton(0, flat, 63)
    assert all(deinterleave(v, 21)[2] == 0 for v in c)


def test_morton_box_centroid():
    lo = np.array([[0.25, 0.5, 0.0]], np.float32)
    hi = np.array([[0.75, 0.5, 0.5]], np.float32)
    boxes = np.concatenate([np.concatenate([lo, hi], 1), [[0, 0, 0, 0, 0, 0], [1, 1, 1, 1, 1, 1]]]).astype(np.float32)
    pts = np.array([[0.5, 0.5, 0.25], [0, 0, 0], [1, 1, 1]], np.float32)
    assert oracle.morton(1, boxes, 30)[0] == oracle.morton(0, pts, 30)[0]


@pytest.mark.parametrize("bits", [30, 63])
def test_morton_monotone_and_range(bits):
    b = bits // 3
    x = np.sort(np.random.default_rng(5).random(3000).astype(np.float32))
    pts = np.stack([x, np.full_like(x, 0.3), np.full_like(x, 0.7)], 1)
    pts = np.concatenate([pts, [[0, 0, 0], [1, 1, 1]]]).astype(np.float32)
    codes = oracle.morton(0, pts, bits)
    qx = [deinterleave(c, b)[0] for c in codes[:-2]]
    assert all(a <= c for a, c in zip(qx, qx[1:]))
    assert int(codes.max()) < (1 << bits)


@pytest.mark.parametrize("bits", [30, 63])
def test_morton_matches_exact_arithmetic_off_boundaries(bits):
    """Away from cell boundaries the float32 quantisation must agree with the
    exact real-number value floor((c - lo) * 2^b / extent).  Three float32
    roundings (subtract, divide, multiply) put t within 3u|t| of the exact
    value, u = 2^-24; samples closer than 4u|t| to an integer are skipped."""
    b = bits // 3
    rng = np.random.default_rng(6)
    p = (rng.random((4000, 3)) * 3.0 - 1.0).astype(np.float32)
    scene = oracle.scene_box(0, p)
    codes = oracle.morton(0, p, bits)
    lo, hi = scene[:3].astype(np.float64), scene[3:].astype(np.float64)
    t = (p.astype(np.float64) - lo) * (1 << b) / (hi - lo)
    frac = t - np.floor(t)
    margin = 4.0 * 2.0 ** -24 * np.abs(t) + 1e-12
    ok = (np.minimum(frac, 1 - frac) > margin) & (t < (1 << b) - 1)
    q = np.array([deinterleave(c, b) for c in codes])
    assert ok.sum() > 3000
    assert np.array_equal(q[ok], np.floor(t[ok]).astype(np.int64))


# ----------------------------------------------------------------- queries

def test_sphere_predicate_special_cases():
    box = np.array([3, 4, 0, 3, 4, 0], np.float32)
    assert oracle.pred_sphere(box, [0, 0, 0, 5])
    assert not oracle.pred_sphere(box, [0, 0, 0, np.nextafter(np.float32(5), np.float32(0))])
    unit = np.array([0, 0, 0, 1, 1, 1], np.float32)
    assert oracle.pred_sphere(unit, [0.5, 0.5, 0.5, 0])          # centre inside
    assert oracle.pred_sphere(unit, [2, 0.5, 0.5, 1])            # touches face
    assert not oracle.pred_sphere(unit, [2, 2, 0.5, 1])          # corner at sqrt 2
    assert oracle.pred_sphere(np.array([1, 1, 1, 1, 1, 1], np.float32), [0, 0, 0, 2])


def test_box_predicate_closed():
    unit = np.array([0, 0, 0, 1, 1, 1], np.float32)
    assert oracle.pred_box(unit, [1, 1, 1, 2, 2, 2])             # corner touch
    assert not oracle.pred_box(unit, [1, 1, np.nextafter(np.float32(1), np.float32(2)), 2, 2, 2])
    assert oracle.pred_box(unit, [0.2, 0.2, 0.2, 0.3, 0.3, 0.3])  # inside
    assert oracle.pred_box(unit, [-1, -1, -1, 2, 2, 2])          # contains


def test_sphere_predicate_matches_exact_distance():
    rng = np.random.default_rng(9)
    boxes = rng.random((3000, 6)).astype(np.float32)
    boxes[:, 3:] = boxes[:, :3] + np.abs(boxes[:, 3:]) * 0.1
    q = np.array([0.5, 0.5, 0.5, 0.3], np.float32)
    b64, q64 = boxes.astype(np.float64), q.astype(np.float64)
    d = np.maximum(np.maximum(b64[:, :3] - q64[:3], q64[:3] - b64[:, 3:]), 0)
    dist = np.sqrt((d * d).sum(1))
    clear = np.abs(dist - q64[3]) > 1e-5
    got = np.array([oracle.pred_sphere(b, q) for b in boxes])
    assert np.array_equal(got[clear], (dist <= q64[3])[clear])


def stack_dfs(t, qkind, q):
    """Classic stack-based traversal with both children (no ropes)."""
    pred = oracle.pred_sphere if qkind == 0 else oracle.pred_box
    out, st, ni = [], [0], t.n - 1
    while st:
        v = st.pop()
        if not pred(t.aabb[v], q):
            continue
        if v >= ni:
            out.append(int(t.perm[v - ni]))
        else:
            st.append(int(t.right[v]))
            st.append(int(t.left[v]))
    return out


def numpy_brute(kind, prims, perm, qkind, q):
    full = prims if kind == 1 else np.concatenate([prims, prims], 1)
    b = full[perm]
    if qkind == 0:
        d = np.maximum(np.maximum(b[:, :3] - q[:3], q[:3] - b[:, 3:]), np.float32(0))
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        hit = d2 <= q[3] * q[3]
    else:
        hit = np.all((q[:3] <= b[:, 3:]) & (b[:, :3] <= q[3:]), axis=1)
    return perm[hit].tolist()


@pytest.mark.parametrize("name,scale", [("small_points", 0.25), ("large_points", 1 / 2048),
                                        ("clustered_boxes", 1 / 256)])
def test_traversal_equals_brute_force(name, scale):
    w = workloads.by_name(name, scale)
    t = oracle.build(w.kind, w.prims, w.code_bits)
    off, idx, visits = oracle.query_traverse(w.qkind, w.queries, t)
    assert visits > 0
    check = range(w.m) if w.m <= 300 else np.random.default_rng(1).choice(w.m, 300, replace=False)
    hits = 0
    for j in check:
        got = idx[off[j]:off[j + 1]].tolist()
        brute = oracle.query_brute(w.qkind, w.queries, int(j), w.kind, w.prims, t.perm).tolist()
        assert got == brute
        assert got == numpy_brute(w.kind, w.prims, t.perm, w.qkind, w.queries[j])
        hits += len(got)
    assert hits > 0
    for j in list(check)[:40]:
        assert idx[off[j]:off[j + 1]].tolist() == stack_dfs(t, w.qkind, w.queries[j])


def test_queries_on_empty_and_single():
    t0 = oracle.build(0, np.zeros((0, 3), np.float32), 30)
    q = np.array([[0, 0, 0, 1]], np.float32)
    off, idx, _ = oracle.query_traverse(0, q, t0)
    assert off.tolist() == [0, 0] and idx.size == 0
    t1 = oracle.build(0, np.array([[0.5, 0.5, 0.5]], np.float32), 30)
    assert t1.rope.tolist() == [-1] and np.array_equal(t1.aabb[0], [0.5] * 6)
    off, idx, _ = oracle.query_traverse(0, np.array([[0.5, 0.5, 0.5, 0], [9, 9, 9, 1]], np.float32), t1)
    assert off.tolist() == [0, 1, 1] and idx.tolist() == [0]


@pytest.mark.parametrize("name,scale,S1,S2", [("clustered_boxes", 1 / 128, 9, 5),
                                              ("large_points", 1 / 512, 8, 3),
                                              ("small_points", 1.0, 12, 7)])
def test_split_walk_equals_plain_walk(name, scale, S1, S2):
    """Cutting Alg. 1 into aligned-block pieces (the GPU query schedule)
    returns the plain walk's hits in the same order."""
    from alg_models import split_walk
    w = workloads.by_name(name, scale)
    t = oracle.build(w.kind, w.prims, w.code_bits)
    off, idx, _ = oracle.query_traverse(w.qkind, w.queries, t)
    pred = oracle.pred_sphere if w.qkind == 0 else oracle.pred_box
    left = np.concatenate([t.left, t.perm]).tolist()
    rope = t.rope.tolist()
    for j in range(min(w.m, 150)):
        q = w.queries[j]
        ref = idx[off[j]:off[j + 1]].tolist()
        got = split_walk(t.n, left, rope, t.perm, lambda v: pred(t.aabb[v], q), S1, S2)
        assert got == ref
        got = split_walk(t.n, left, rope, t.perm, lambda v: pred(t.aabb[v], q), S1, S2,
                         lambda v: contains(w.qkind, t.aabb[v], q))
        assert got == ref
        # the GPU leaf level: pieces no wider than the scan limit test their
        # leaves directly (and a limit below the piece width keeps the walk)
        for scan in (1 << S2, (1 << S2) // 2):
            got = split_walk(t.n, left, rope, t.perm, lambda v: pred(t.aabb[v], q), S1, S2,
                             lambda v: contains(w.qkind, t.aabb[v], q), leaf_scan=scan)
            assert got == ref


def contains(qkind, box, q):
    """The query contains the box (float32 arithmetic as in the kernels)."""
    box = box.astype(np.float32)
    q = q.astype(np.float32)
    if qkind == 1:
        return bool(np.all(q[:3] <= box[:3]) and np.all(box[3:] <= q[3:]))
    f = np.maximum(q[:3] - box[:3], box[3:] - q[:3])
    d2 = np.float32(np.float32(f[0] * f[0]) + np.float32(f[1] * f[1])) + np.float32(f[2] * f[2])
    return bool(d2 <= np.float32(q[3] * q[3]))


@pytest.mark.parametrize("qkind", [0, 1])
def test_containment_implies_every_leaf_passes(qkind):
    """Exactness of the containment shortcut: whenever the float32
    containment test accepts a node, the float32 predicate accepts every
    leaf box below it."""
    w = workloads.clustered(1 << 13, 64) if qkind == 1 else workloads.small_points(1 << 13, 64)
    t = oracle.build(w.kind, w.prims, w.code_bits)
    pred = oracle.pred_sphere if qkind == 0 else oracle.pred_box
    rng = np.random.default_rng(21)
    qs = w.queries.copy()
    if qkind == 0:
        qs[:, 3] = rng.random(len(qs)).astype(np.float32) * 0.3
    else:
        c = rng.random((len(qs), 3)).astype(np.float32)
        s = rng.random((len(qs), 3)).astype(np.float32) * 0.3
        qs = np.concatenate([c - s, c + s], 1).astype(np.float32)
    seen = 0
    for q in qs:
        for v in range(t.n - 1):
            if contains(qkind, t.aabb[v], q):
                seen += 1
                for k in range(t.rlo[v], t.rhi[v] + 1):
                    assert pred(t.aabb[t.n - 1 + k], q)
    assert seen > 0


def test_split_walk_degenerate():
    from alg_models import split_walk
    for n in [1, 2, 3, 5, 40, 300]:
        p = np.full((n, 3), 0.5, np.float32)
        t = oracle.build(0, p, 30)
        left = np.concatenate([t.left, t.perm]).tolist()
        for q in ([0.5, 0.5, 0.5, 0.1], [9, 9, 9, 0.1]):
            q = np.array(q, np.float32)
            off, idx, _ = oracle.query_traverse(0, q[None], t)
            got = split_walk(n, left, t.rope.tolist(), t.perm,
                             lambda v: oracle.pred_sphere(t.aabb[v], q), 3, 1)
            assert got == idx.tolist()


@pytest.mark.parametrize("cap1,cap2,seed", [(10**9, 10**9, 0), (40, 120, 1), (5, 30, 2), (0, 0, 3),
                                            (60, 8, 4)])
def test_split_levels_with_bounded_lists(cap1, cap2, seed):
    """Both split levels over a batch of queries whose pieces exceed the
    append lists: whatever subset of pieces fits (arbitrary append order),
    an item that lost one passes through its level unsplit and every query
    still gets the plain walk's hits in order (the GPU count kernels' rule
    for a full list)."""
    from alg_models import split_levels_capped
    w = workloads.by_name("clustered_boxes", 1 / 256)
    t = oracle.build(w.kind, w.prims, w.code_bits)
    qs = w.queries[:40].copy()
    qs[::5, 3:] += 0.2                                  # some large queries: many pieces
    off, idx, _ = oracle.query_traverse(1, qs, t)
    left = np.concatenate([t.left, t.perm]).tolist()
    rope = t.rope.tolist()
    tests = [(lambda v, q=q: oracle.pred_box(t.aabb[v], q)) for q in qs]
    hits = split_levels_capped(t.n, left, rope, t.perm, tests, 9, 5, cap1, cap2, seed)
    for j in range(len(qs)):
        assert hits[j] == idx[off[j]:off[j + 1]].tolist(), f"query {j}"
