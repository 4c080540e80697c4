"""Pins of the oracle's tree (topology, ropes, boxes) against what the paper
and the mathematics fix, independently of the oracle's own code:

* the paper's worked example (Fig. 1, Fig. 2a, Fig. 2b, Sec. 3.1/3.2);
* the max-Cartesian tree of delta*, an independent O(n) construction of the
  same binary radix tree;
* Alg. 3 (relabelled by range) and Alg. 4 run step by step under
  adversarial schedules;
* the rope definition of Sec. 2 (next node in preorder outside the subtree)
  and the closed form of Alg. 2;
* exhaustive enumeration of every sorted multiset of up to 7 keys over
  3-bit codes.
"""

import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
from alg_models import alg3, alg4, alg4_blocked

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _load_example():
    with open(GOLDEN) as f:
        g = json.load(f)
    keys = np.array([int(b, 2) for b in g["keys_binary"]], np.uint64)
    return g, keys


def _name_to_id(name, n):
    if name == "S":
        return -1
    k = int(name[1:])
    return k if name[0] == "I" else n - 1 + k


# ----------------------------------------------------------- worked example

def test_example_keys_are_sorted_and_distinct():
    g, keys = _load_example()
    assert list(keys) == sorted(keys) and len(set(keys.tolist())) == 8


def test_example_karras_topology():
    g, keys = _load_example()
    n = len(keys)
    t = oracle.tree_from_sorted(keys)
    for name, (a, b) in g["karras"]["children"].items():
        k = int(name[1:])
        assert t.left[k] == _name_to_id(a, n), name
        assert t.right[k] == _name_to_id(b, n), name
    for name, (lo, hi) in g["karras"]["ranges"].items():
        k = int(name[1:])
        assert (t.rlo[k], t.rhi[k]) == (lo, hi), name
    for name, s in g["karras"]["splits"].items():
        k = int(name[1:])
        assert int(np.argmax(t.delta[t.rlo[k]:t.rhi[k]])) + t.rlo[k] == s, name


def test_example_ropes():
    g, keys = _load_example()
    n = len(keys)
    t = oracle.tree_from_sorted(keys)
    for name, target in g["ropes"].items():
        if name.startswith("_"):
            continue
        assert t.rope[_name_to_id(name, n)] == _name_to_id(target, n), name


def test_example_boundary_order():
    g, keys = _load_example()
    t = oracle.tree_from_sorted(keys)
    groups = g["boundary_rank_desc"]["groups"]
    vals = [{int(t.delta[k]) for k in grp} for grp in groups]
    for v in vals:
        assert len(v) == 1            # equal heights -> equal rank
    flat = [next(iter(v)) for v in vals]
    assert flat == sorted(flat, reverse=True) and len(set(flat)) == len(flat)


@pytest.mark.parametrize("policy,seed", [("left", 0), ("right", 0)] + [("random", s) for s in range(20)])
def test_example_alg3_apetrei_order(policy, seed):
    g, keys = _load_example()
    n = len(keys)
    t = oracle.tree_from_sorted(keys)
    children, ranges, root = alg3(t.delta, n, policy, seed)
    assert root == int(g["apetrei"]["root"][1:])
    for name, (a, b) in g["apetrei"]["children"].items():
        p = int(name[1:])
        conv = lambda c: (c[0], int(c[1:]))
        assert tuple(children[p][0]) == conv(a) and tuple(children[p][1]) == conv(b), name


@pytest.mark.parametrize("policy,seed", [("left", 0), ("right", 0)] + [("random", s) for s in range(20)])
def test_example_alg4_matches_figures(policy, seed):
    g, keys = _load_example()
    n = len(keys)
    t = oracle.tree_from_sorted(keys)
    left, rope, _ = alg4(t.delta, n, None, policy, seed)
    for name, (a, _b) in g["karras"]["children"].items():
        assert left[int(name[1:])] == _name_to_id(a, n), name
    for name, target in g["ropes"].items():
        if not name.startswith("_"):
            assert rope[_name_to_id(name, n)] == _name_to_id(target, n), name


def test_example_literal_left_child_line_is_inconsistent():
    """The printed left-child line of Alg. 4 (compare range_left with q, name
    the child by i) does not give Fig. 2a's children; the reading that uses
    the split p does (checked above).  Here: the literal line for the parent
    I1 = [0,1] reached from leaf 1 would test range_left (0) against q (1)
    and pick the internal node of index i = 1, i.e. I1 itself."""
    g, keys = _load_example()
    n = len(keys)
    rl, q, i = 0, 1, 1
    literal = (n - 1 + i) if rl == q else i
    assert literal != _name_to_id(g["karras"]["children"]["I1"][0], n)


# ----------------------------------------------------- independent builders

def cartesian_max(delta):
    """Max-Cartesian tree of delta by the classic stack construction."""
    m = len(delta)
    lc, rc, st = [-1] * m, [-1] * m, []
    for k in range(m):
        last = -1
        while st and delta[st[-1]] < delta[k]:
            last = st.pop()
        lc[k] = last
        if st:
            rc[st[-1]] = k
        st.append(k)
    return (st[0] if st else -1), lc, rc


def _split_of(t, node):
    ni = t.n - 1
    l = int(t.left[node])
    return l - ni if l >= ni else l


def check_against_cartesian(t):
    n, ni = t.n, t.n - 1
    if n < 2:
        return
    root, lc, rc = cartesian_max([int(x) for x in t.delta])
    assert _split_of(t, 0) == root
    for node in range(ni):
        s = _split_of(t, node)
        l, r = int(t.left[node]), int(t.right[node])
        if lc[s] == -1:
            assert l == ni + s
        else:
            assert l < ni and _split_of(t, l) == lc[s]
        if rc[s] == -1:
            assert r == ni + s + 1
        else:
            assert r < ni and _split_of(t, r) == rc[s]


def node_range(t, v):
    ni = t.n - 1
    if v >= ni:
        return (v - ni, v - ni)
    return (int(t.rlo[v]), int(t.rhi[v]))


def check_invariants(t):
    """Contiguous ranges, split = argmax, Karras index rule, ropes."""
    n, ni = t.n, t.n - 1
    D = lambda i: 1 << 30 if (i < 0 or i >= n - 1) else int(t.delta[i])
    seen = np.zeros(2 * n - 1, np.int64)
    seen[0] += 1
    for v in range(ni):
        i, j = node_range(t, v)
        l, r = int(t.left[v]), int(t.right[v])
        seen[l] += 1
        seen[r] += 1
        li, lj = node_range(t, l)
        ri, rj = node_range(t, r)
        assert li == i and rj == j and lj + 1 == ri              # contiguous split
        assert lj == i + int(np.argmax(t.delta[i:j]))            # highest bit
        # Karras index: a left child is named by its right bound, a right
        # child by its left bound (Sec. 3.1)
        assert (l - ni if l >= ni else l) == lj
        assert (r - ni if r >= ni else r) == ri
        # ... which is the bound with the smaller adjacent delta* (Sec. 3.1)
        if l < ni:
            assert (lj if D(lj) < D(li - 1) else li) == l
        if r < ni:
            assert (rj if D(rj) < D(ri - 1) else ri) == r
    assert (seen == 1).all()                                     # a tree
    # ropes: next node in preorder outside the subtree (Sec. 2)
    order, st = [], [0]
    while st:
        v = st.pop()
        order.append(v)
        if v < ni:
            st.append(int(t.right[v]))
            st.append(int(t.left[v]))
    pos = {v: k for k, v in enumerate(order)}
    for v in range(2 * n - 1):
        i, j = node_range(t, v)
        after = pos[v] + 2 * (j - i + 1) - 1
        expect = order[after] if after < len(order) else -1
        assert int(t.rope[v]) == expect, v
        # Alg. 2 closed form from the right bound
        if j == n - 1:
            a2 = -1
        else:
            r = j + 1
            a2 = ni + r if D(r - 1) < D(r) else r
        assert int(t.rope[v]) == a2, v


def check_alg4(t, policies=(("left", 0), ("right", 0), ("random", 1), ("random", 2))):
    n = t.n
    for pol, seed in policies:
        left, rope, _ = alg4(t.delta, n, None, pol, seed)
        assert list(left) == [int(x) for x in t.left]
        assert list(rope) == [int(x) for x in t.rope]


def check_alg3(t, seed=0):
    n, ni = t.n, t.n - 1
    if n < 2:
        return
    children, ranges, root = alg3(t.delta, n, "random", seed)
    assert ranges[root] == (0, n - 1)
    by_split = {_split_of(t, v): v for v in range(ni)}
    assert by_split[root] == 0
    for p, (lo, hi) in ranges.items():
        v = by_split[p]
        assert node_range(t, v) == (lo, hi)
        for side, ch in zip((t.left, t.right), children[p]):
            kind, k = ch
            if kind == "L":
                assert int(side[v]) == ni + k
            else:
                assert int(side[v]) == by_split[k]


def test_exhaustive_small_multisets():
    """Every sorted multiset of n <= 7 keys over 3-bit codes."""
    count = 0
    for n in range(1, 8):
        for keys in itertools.combinations_with_replacement(range(8), n):
            t = oracle.tree_from_sorted(np.array(keys, np.uint64))
            if n >= 2:
                check_invariants(t)
                check_against_cartesian(t)
                check_alg3(t, seed=count)
            check_alg4(t, (("left", 0), ("right", 0), ("random", count)))
            count += 1
    assert count == sum(len(list(itertools.combinations_with_replacement(range(8), n)))
                        for n in range(1, 8))


@pytest.mark.parametrize("seed", range(12))
def test_random_with_duplicates(seed):
    rng = np.random.default_rng([100, seed])
    n = int(rng.integers(2, 3000))
    ncodes = int(rng.integers(1, 64))
    keys = np.sort(rng.integers(0, 1 << int(rng.integers(1, 63)), size=ncodes, dtype=np.uint64))
    keys = np.sort(rng.choice(keys, size=n))
    t = oracle.tree_from_sorted(keys)
    check_invariants(t)
    check_against_cartesian(t)
    check_alg3(t, seed)
    check_alg4(t, (("random", seed), ("left", 0)))


def test_all_equal_codes_is_index_tree():
    """With one repeated code the tree is the radix tree of the indices."""
    n = 37
    t = oracle.tree_from_sorted(np.full(n, 5, np.uint64))
    check_invariants(t)
    # root splits at the highest bit of n-1: leaves [0, 31] and [32, 36]
    assert _split_of(t, 0) == 31


def test_tiny_trees():
    t0 = oracle.tree_from_sorted(np.zeros(0, np.uint64))
    assert t0.n == 0 and t0.rope.size == 0
    t1 = oracle.tree_from_sorted(np.array([3], np.uint64))
    assert t1.rope.tolist() == [-1] and t1.left.size == 0
    t2 = oracle.tree_from_sorted(np.array([3, 3], np.uint64))
    assert t2.left.tolist() == [1] and t2.right.tolist() == [2]
    assert t2.rope.tolist() == [-1, 2, -1]


def test_planted_rope_mistake_is_caught():
    """A rope pointing one node further (a plausible off-by-one) fails the
    preorder pin."""
    g, keys = _load_example()
    t = oracle.tree_from_sorted(keys)
    t.rope = t.rope.copy()
    t.rope[7] = t.rope[8]            # L0 -> I2 instead of L1
    with pytest.raises(AssertionError):
        check_invariants(t)


# ------------------------------------------------------------------- boxes

@pytest.mark.parametrize("kind", [oracle.POINTS, oracle.BOXES])
def test_boxes_union_and_scene(kind):
    rng = np.random.default_rng([7, kind])
    n = 2000
    if kind == oracle.POINTS:
        prims = rng.random((n, 3), dtype=np.float32)
    else:
        c = rng.random((n, 3))
        s = rng.random((n, 3)) * 0.01
        prims = np.concatenate([c - s, c + s], axis=1).astype(np.float32)
    t = oracle.build(kind, prims, 30)
    ni = n - 1
    full = prims if kind == oracle.BOXES else np.concatenate([prims, prims], 1)
    assert np.array_equal(t.aabb[ni:], full[t.perm])
    for v in range(ni):
        a, b = t.aabb[t.left[v]], t.aabb[t.right[v]]
        u = np.concatenate([np.minimum(a[:3], b[:3]), np.maximum(a[3:], b[3:])])
        assert np.array_equal(t.aabb[v], u)
    assert np.array_equal(t.aabb[0], t.scene)
    assert np.array_equal(t.scene[:3], full[:, :3].min(0))
    assert np.array_equal(t.scene[3:], full[:, 3:].max(0))
    check_invariants(t)


@pytest.mark.parametrize("seed", range(3))
def test_alg4_boxes_match_oracle(seed):
    rng = np.random.default_rng([8, seed])
    n = 300
    prims = (rng.integers(0, 4, size=(n, 3)) / 4).astype(np.float32)  # many duplicates
    t = oracle.build(oracle.POINTS, prims, 30)
    leaf_boxes = np.concatenate([prims, prims], 1)[t.perm]
    for pol in ("left", "right", "random"):
        left, rope, boxes = alg4(t.delta, n, leaf_boxes, pol, seed)
        assert np.array_equal(np.array(boxes, np.float32), t.aabb)


# ------------------------------------------------ blocked (level) schedule

@pytest.mark.parametrize("chunk,fanout", [(1, 2), (2, 2), (3, 2), (4, 3), (8, 2), (16, 4)])
def test_alg4_blocked_exhaustive(chunk, fanout):
    """Alg. 4 split into levels of blocks (the GPU kernels' schedule) gives
    the oracle tree for every sorted multiset of <= 6 keys over 3-bit codes."""
    k = 0
    for n in range(1, 7):
        for keys in itertools.combinations_with_replacement(range(8), n):
            t = oracle.tree_from_sorted(np.array(keys, np.uint64))
            for pol in ("left", "right", "random"):
                left, rope, _ = alg4_blocked(t.delta, n, chunk, fanout, None, pol, k)
                assert list(left) == [int(x) for x in t.left]
                assert list(rope) == [int(x) for x in t.rope]
            k += 1


@pytest.mark.parametrize("seed", range(8))
def test_alg4_blocked_random_with_boxes(seed):
    rng = np.random.default_rng([15, seed])
    n = int(rng.integers(2, 1500))
    prims = (rng.integers(0, 6, size=(n, 3)) / 5).astype(np.float32)
    t = oracle.build(oracle.POINTS, prims, 30)
    leaf_boxes = np.concatenate([prims, prims], 1)[t.perm]
    chunk = int(rng.choice([1, 3, 16, 64, 1024]))
    fanout = int(rng.choice([2, 3, 256]))
    left, rope, boxes = alg4_blocked(t.delta, n, chunk, fanout, leaf_boxes, "random", seed)
    assert list(left) == [int(x) for x in t.left]
    assert list(rope) == [int(x) for x in t.rope]
    assert np.array_equal(np.array(boxes, np.float32), t.aabb)
