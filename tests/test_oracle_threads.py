"""The oracle's parallel loops (used only to time it on several host cores)
give bit-identical results for any thread count: each loop iteration is
independent and min/max are exact."""

import numpy as np

import oracle
import workloads


def _all(kind, prims, bits, qkind, queries):
    t = oracle.build(kind, prims, bits)
    off, idx, vis = oracle.query_traverse(qkind, queries, t)
    return t, off, idx, vis


def test_thread_count_does_not_change_results():
    for w in (workloads.by_name("clustered_boxes", 1 / 256), workloads.by_name("large_points", 1 / 128)):
        try:
            oracle.threads(1)
            a = _all(w.kind, w.prims, w.code_bits, w.qkind, w.queries[:4096])
            oracle.threads(4)
            b = _all(w.kind, w.prims, w.code_bits, w.qkind, w.queries[:4096])
        finally:
            oracle.threads(1)
        ta, tb = a[0], b[0]
        for f in ("scene", "codes", "sorted", "perm", "delta", "left", "right", "rlo", "rhi", "rope"):
            assert np.array_equal(getattr(ta, f), getattr(tb, f)), f
        assert np.array_equal(ta.aabb.view(np.uint32), tb.aabb.view(np.uint32))
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and a[3] == b[3]
