"""Executable models of the paper's bottom-up constructions (test helpers).

These run the steps of Alg. 3 (Apetrei's original bottom-up pass, Sec. 3.2)
and Alg. 4 (the modified pass that keeps Karras' node order and installs the
skip-connections, Sec. 4) on the CPU, one Python generator per leaf.  Each
generator yields right before its compare-and-swap on ``store``, so a
scheduler can interleave the leaves in any order; the CAS itself and the code
up to the next CAS run without interruption, which is what an atomic CAS
guarantees.  They exist to check, under adversarial schedules, that the
paper's procedure reaches the same tree as the oracle's top-down definition.

Readings used (each one is also listed with the oracle):
  * delta* is the rank of the highest differing bit of the augmented keys,
    with delta*(-1) = delta*(n-1) = +inf;
  * Alg. 4's left-child line is read as: the left child of the parent is leaf
    p if range_left == p, else internal node p, where p is the split (the
    Apetrei index).  Sec. 4 states that the children of a parent with split
    gamma are gamma and gamma+1; the printed condition compares against q and
    names the child by i, which on the worked example gives wrong children;
  * the boxes, omitted from both listings, are merged by the second thread
    to arrive: it reads the sibling's box, written before the sibling's CAS.
"""

from __future__ import annotations

import random

INF = 1 << 30
SENTINEL = -1


class _Delta:
    def __init__(self, delta, n):
        self.d = list(int(x) for x in delta)
        self.n = n

    def __call__(self, i):
        if i < 0 or i >= self.n - 1:
            return INF
        return self.d[i]


def _schedule(gens, policy, rng):
    """Drive generators to completion.  policy: 'random', 'left' (always the
    lowest live leaf first) or 'right' (the highest first)."""
    live = list(range(len(gens)))
    while live:
        if policy == "random":
            k = rng.randrange(len(live))
        elif policy == "left":
            k = 0
        else:
            k = len(live) - 1
        g = live[k]
        try:
            next(gens[g])
        except StopIteration:
            live.pop(k)


def alg4(delta, n, leaf_boxes=None, policy="random", seed=0):
    """Modified Apetrei with ropes (Alg. 4) plus box merging.

    Returns (left[n-1], rope[2n-1], boxes[2n-1] or None) in unified ids
    (internal k -> k, leaf k -> n-1+k, sentinel -1)."""
    D = _Delta(delta, n)
    ni = n - 1
    left = [None] * max(ni, 0)
    rope = [None] * max(2 * n - 1, 0)
    boxes = [None] * max(2 * n - 1, 0) if leaf_boxes is not None else None
    store = [None] * max(ni, 0)   # None plays the 'invalid' marker

    def leaf(k):
        return ni + k

    def union(a, b):
        return tuple(min(a[x], b[x]) for x in range(3)) + tuple(max(a[3 + x], b[3 + x]) for x in range(3))

    def run(i):
        rl = rr = i
        dl, dr = D(i - 1), D(i)
        if i == n - 1:
            rope[leaf(i)] = SENTINEL
        else:
            rope[leaf(i)] = leaf(i + 1) if dr < D(i + 1) else i + 1
        cur = leaf(i)
        if boxes is not None:
            boxes[cur] = tuple(leaf_boxes[i])
        if n == 1:
            return
        while True:
            if dr < dl:                      # left child of its parent
                p = rr
                yield
                old = store[p]
                if old is None:
                    store[p] = rl
                    return
                rr = old
                dr = D(rr)
                sib = leaf(p + 1) if p + 1 == rr else p + 1
            else:                            # right child of its parent
                p = rl - 1
                yield
                old = store[p]
                if old is None:
                    store[p] = rr
                    return
                rl = old
                dl = D(rl - 1)
                sib = leaf(p) if rl == p else p
            q = rr if dr < dl else rl        # Karras index of the parent
            left[q] = leaf(p) if rl == p else p
            if rr == n - 1:
                rope[q] = SENTINEL
            else:
                r = rr + 1
                rope[q] = leaf(r) if dr < D(r) else r
            if boxes is not None:
                boxes[q] = union(boxes[cur], boxes[sib])
            cur = q
            if q == 0:
                return

    rng = random.Random(seed)
    _schedule([run(i) for i in range(n)], policy, rng)
    return left, rope, boxes


def alg4_blocked(delta, n, chunk, fanout, leaf_boxes=None, policy="random", seed=0):
    """Alg. 4 run the way the GPU kernels run it: by levels of blocks.

    Level 0 gives each block `chunk` consecutive leaves; level L >= 1 gives
    each block `fanout` consecutive blocks of level L-1.  A block owns the
    boundaries strictly inside its leaf span [A, B).  Its threads climb as in
    Alg. 4, but a thread whose parent's split p is a boundary of the span
    (p = A-1 or p = B-1) stops and hands its state (node, range) to the
    level above.  Blocks of one level run one after another here (they touch
    disjoint parts of `store`); threads inside a block interleave under the
    given schedule.  Returns (left, rope, boxes) like ``alg4``.

    Level 0 climbs as Alg. 4 does, with delta* looked up.  The levels above
    climb the way the upper-level kernel does: a climb carries delta* at
    its two outer boundaries and its rope; a first arrival parks its far
    end together with delta* at its outer boundary on that side, so the
    second arrival takes the parent's new outer delta* from the parked word
    and looks none up; and a parent's rope is its right child's (Alg. 2
    depends only on the range's right end)."""
    D = _Delta(delta, n)
    ni = n - 1
    left = [None] * max(ni, 0)
    rope = [None] * max(2 * n - 1, 0)
    boxes = [None] * max(2 * n - 1, 0) if leaf_boxes is not None else None
    store = [None] * max(ni, 0)

    def leaf(k):
        return ni + k

    def union(a, b):
        return tuple(min(a[x], b[x]) for x in range(3)) + tuple(max(a[3 + x], b[3 + x]) for x in range(3))

    def climb(cur, rl, rr, A, B, out, carried=None):
        # carried (upper levels): (dl, dr) handed over with the climb
        dl, dr = carried if carried is not None else (D(rl - 1), D(rr))
        upper = carried is not None
        while True:
            if dr < dl:
                p = rr
                if p == B - 1:
                    out[1] = (cur, rl, rr, dl, dr)
                    return
                yield
                old = store[p]
                if old is None:
                    store[p] = (rl, dl)          # far end, delta* beyond it
                    return
                rr, d_far = old
                dr = d_far if upper else D(rr)
                sib = leaf(p + 1) if p + 1 == rr else p + 1
                right = sib
            else:
                p = rl - 1
                if p == A - 1:
                    out[0] = (cur, rl, rr, dl, dr)
                    return
                yield
                old = store[p]
                if old is None:
                    store[p] = (rr, dr)
                    return
                rl, d_far = old
                dl = d_far if upper else D(rl - 1)
                sib = leaf(p) if rl == p else p
                right = cur
            q = rr if dr < dl else rl
            left[q] = leaf(p) if rl == p else p
            if upper:
                rope[q] = rope[right]
            elif rr == n - 1:
                rope[q] = SENTINEL
            else:
                r = rr + 1
                rope[q] = leaf(r) if dr < D(r) else r
            if boxes is not None:
                boxes[q] = union(boxes[cur], boxes[sib])
            cur = q
            if q == 0:
                return

    rng = random.Random(seed)
    for i in range(n):                       # leaf records (Alg. 4 leaf part)
        rope[leaf(i)] = SENTINEL if i == n - 1 else (leaf(i + 1) if D(i) < D(i + 1) else i + 1)
        if boxes is not None:
            boxes[leaf(i)] = tuple(leaf_boxes[i])
    if n == 1:
        return left, rope, boxes

    span = chunk
    nb = (n + span - 1) // span
    pend = []
    for b in range(nb):                      # level 0
        A, B = b * span, min((b + 1) * span, n)
        out = [None, None]
        _schedule([climb(leaf(i), i, i, A, B, out) for i in range(A, B)], policy, rng)
        pend.append(out)
    levels = 0
    while nb > 1:                            # levels >= 1
        levels += 1
        child_span, span = span, span * fanout
        nb_next = (n + span - 1) // span
        nxt = []
        for b in range(nb_next):
            A, B = b * span, min((b + 1) * span, n)
            j0, j1 = A // child_span, (B + child_span - 1) // child_span
            out = [None, None]
            gens = [climb(s[0], s[1], s[2], A, B, out, carried=(s[3], s[4]))
                    for j in range(j0, j1) for s in pend[j] if s is not None]
            _schedule(gens, policy, rng)
            nxt.append(out)
        pend, nb = nxt, nb_next
    assert all(s is None for s in pend[0]), "the top level must finish the tree"
    return left, rope, boxes


def alg3(delta, n, policy="random", seed=0):
    """Apetrei's original bottom-up pass (Alg. 3), nodes indexed by split.

    Returns (children: dict p -> [left, right] with entries ('L', k) or
    ('I', p'), ranges: dict p -> (lo, hi), root p).  The loop stops when a
    thread's range is the whole [0, n-1]."""
    D = _Delta(delta, n)
    children = {}
    ranges = {}
    store = [None] * max(n - 1, 0)
    root = [None]

    def run(i):
        rl = rr = i
        dl, dr = D(i - 1), D(i)
        cur = ("L", i)
        while True:
            if dr < dl:
                p = rr
                children.setdefault(p, [None, None])[0] = cur
                yield
                old = store[p]
                if old is None:
                    store[p] = rl
                    return
                rr = old
                dr = D(rr)
            else:
                p = rl - 1
                children.setdefault(p, [None, None])[1] = cur
                yield
                old = store[p]
                if old is None:
                    store[p] = rr
                    return
                rl = old
                dl = D(rl - 1)
            cur = ("I", p)
            ranges[p] = (rl, rr)
            if rl == 0 and rr == n - 1:
                root[0] = p
                return

    if n == 1:
        return {}, {}, None
    rng = random.Random(seed)
    _schedule([run(i) for i in range(n)], policy, rng)
    return children, ranges, root[0]


def split_walk(n, left, rope, perm, test, S1, S2, contains=None, leaf_scan=None):
    """A query's Alg. 1 walk cut into independent pieces by aligned leaf
    blocks, the way the GPU query kernels run it.

    During a walk the leaf range [i, j] of the current node is known without
    extra data: i is kept (descending left keeps it; a rope leads to the
    node whose Karras index is the new left bound) and j = index(rope) - 1
    (n - 1 at the sentinel).  Level 1 walks from the root and emits one
    piece per aligned block of 2^S1 leaves at the first passing node inside
    that block, then jumps to the largest node starting at the next block
    (internal node r if it is a right child, i.e. its split >= r, else leaf
    r).  Level 2 does the same inside each piece with 2^S2 leaves; the last
    level is the plain walk restricted to the piece's leaf range.  With
    ``contains`` (node -> the query contains its box), a passing multi-block
    node that is contained becomes all-hit ranges split at block bounds, and
    a contained internal node in the last level reports its whole leaf range
    without being walked.  With ``leaf_scan``, a last-level piece [i, hi) no
    wider than leaf_scan is not walked: its hits are the leaves of [i, hi)
    that pass, in index order (the predicates are monotone under box
    inclusion, so every ancestor of a passing leaf passes).  Returns the
    hits in order (must equal the plain walk)."""
    ni = n - 1

    def idx(v):
        return v - ni if v >= ni else v

    def jend(v):
        r = rope[v]
        return n - 1 if r == -1 else idx(r) - 1

    def first_at(r):
        if r <= n - 2 and idx(left[r]) >= r:
            return r
        return ni + r

    ALL = -2

    def ranges(a, b, S):
        out = []
        while a < b:
            e = min(((a >> S) + 1) << S, b)
            out.append((ALL, a, e))
            a = e
        return out

    def split(v, i, hi, S):
        if v == ALL:
            return ranges(i, hi, S)
        out = []
        while v != -1 and i < hi:
            j = jend(v)
            if not test(v):
                v, i = rope[v], j + 1
                continue
            if (i >> S) == (j >> S):
                blk = i >> S
                out.append((v, i, min((blk + 1) << S, hi)))
                r = (blk + 1) << S
                if r >= hi or r > n - 1:
                    break
                v, i = first_at(r), r
                continue
            if contains is not None and contains(v):
                out += ranges(i, min(j + 1, hi), S)
                v, i = rope[v], j + 1
                continue
            v = left[v]
        return out

    def walk(v, i, hi):
        if v == ALL:
            return [int(perm[k]) for k in range(i, hi)]
        if leaf_scan is not None and hi - i <= leaf_scan:
            return [int(perm[k]) for k in range(i, hi) if test(ni + k)]
        out = []
        while v != -1 and i < hi:
            j = jend(v)
            if test(v):
                if v >= ni:
                    out.append(int(perm[v - ni]))
                elif contains is not None and contains(v):
                    out += [int(perm[k]) for k in range(i, min(j + 1, hi))]
                else:
                    v = left[v]
                    continue
            v, i = rope[v], j + 1
        return out

    if n == 0:
        return []
    hits = []
    for (a, i, hi) in split(0, 0, n, S1):
        for (b, i2, hi2) in split(a, i, hi, S2):
            hits += walk(b, i2, hi2)
    return hits


def split_levels_capped(n, left, rope, perm, tests, S1, S2, cap1, cap2, seed=0):
    """Both split levels over a batch of queries with bounded append lists,
    the way the count kernels fill them: every piece of every item is
    appended in an arbitrary interleaving (seeded shuffle); the first
    ``cap`` appended are kept; an item that lost any of its pieces passes
    through its level unsplit, as one piece (a query: the walk from the
    root over [0, n); a level-1 piece: itself).  Returns each query's hits
    in order.  ``tests[q]`` is query q's node predicate."""
    import random as _random
    rng = _random.Random(seed)
    if n == 0:
        return [[] for _ in tests]

    def level(items, S, cap):
        # items: list of (query, v, i, hi); returns the next level's items
        pieces = []
        for t, (q, v, i, hi) in enumerate(items):
            got = _split_pieces(n, left, rope, tests[q], v, i, hi, S)
            pieces.append([(q,) + pc for pc in got])
        order = [(t, r) for t, ps in enumerate(pieces) for r in range(len(ps))]
        rng.shuffle(order)
        kept = set(order[:cap])
        out = []
        for t, ps in enumerate(pieces):
            if all((t, r) in kept for r in range(len(ps))):
                out += ps
            else:
                out.append(items[t])      # unsplit
        return out

    items = [(q, 0, 0, n) for q in range(len(tests))]
    items = level(items, S1, cap1)
    items = level(items, S2, cap2)
    hits = [[] for _ in tests]
    for (q, v, i, hi) in items:
        hits[q] += _walk_range(n, left, rope, perm, tests[q], v, i, hi)
    return hits


def _split_pieces(n, left, rope, test, v, i, hi, S):
    """One split level of one item (no containment): pieces (v, i, hi)."""
    ni = n - 1
    idx = (lambda x: x - ni if x >= ni else x)
    jend = (lambda x: n - 1 if rope[x] == -1 else idx(rope[x]) - 1)

    def first_at(r):
        if r <= n - 2 and idx(left[r]) >= r:
            return r
        return ni + r
    out = []
    while v != -1 and i < hi:
        j = jend(v)
        if not test(v):
            v, i = rope[v], j + 1
            continue
        if (i >> S) == (j >> S):
            blk = i >> S
            out.append((v, i, min((blk + 1) << S, hi)))
            r = (blk + 1) << S
            if r >= hi or r > n - 1:
                break
            v, i = first_at(r), r
            continue
        v = left[v]
    return out


def _walk_range(n, left, rope, perm, test, v, i, hi):
    """Alg. 1 restricted to the leaves [i, hi) from node v."""
    ni = n - 1
    idx = (lambda x: x - ni if x >= ni else x)
    jend = (lambda x: n - 1 if rope[x] == -1 else idx(rope[x]) - 1)
    out = []
    while v != -1 and i < hi:
        j = jend(v)
        if test(v):
            if v >= ni:
                out.append(int(perm[v - ni]))
            else:
                v = left[v]
                continue
        v, i = rope[v], j + 1
    return out
