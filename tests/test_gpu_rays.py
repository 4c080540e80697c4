"""GPU parity of the ray and segment queries against the CPU oracle.

All hits (the count and fill calls with rays) must give the oracle's CSR
exactly, in order; first hits must give the oracle's primitive and the
bits of its entry parameter.  The oracle's ray answers are pinned to exact
arithmetic and brute force by the CPU tests (test_oracle_rays.py).
"""

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_query_equal, first_mismatch, gpu_build, gpu_query, say

pytestmark = pytest.mark.gpu

RAYS = 2


@pytest.fixture(scope="module")
def ws():
    import paper_2402_00665_amd as lb
    return lb.Workspace()


def gpu_first(tree, rays, ws=None):
    import torch
    import paper_2402_00665_amd as lb
    say(f"  gpu first hit: m={rays.shape[0]} n={tree.n}")
    hit, t = lb.query_first(tree, torch.from_numpy(np.ascontiguousarray(rays)).cuda(), workspace=ws)
    lb.check_query(ws, rays.shape[0]) if ws is not None else torch.cuda.synchronize()
    return hit.cpu().numpy(), t.cpu().numpy()


def assert_first_equal(hit, t, ref_hit, ref_t):
    k = first_mismatch(hit, ref_hit)
    assert k is None, f"hit[{k}]: gpu {hit[k]} oracle {ref_hit[k]}"
    k = first_mismatch(t.view(np.int32), ref_t.view(np.int32))
    assert k is None, f"t[{k}]: gpu {t[k]!r} oracle {ref_t[k]!r}"


def _both(prims, kind, bits, rays, ws):
    """All hits and first hits of `rays` on the tree of `prims`, GPU against
    the oracle; returns the oracle's total hits and rays that hit."""
    ref = oracle.build(kind, prims, bits)
    tree, _ = gpu_build(prims, kind, bits, ws)
    roff, ridx, _ = oracle.query_traverse(RAYS, rays, ref)
    off, idx = gpu_query(tree, rays, RAYS, ws)
    assert_query_equal(off, idx, roff, ridx)
    rhit, rt, _ = oracle.ray_first_traverse(rays, ref)
    hit, t = gpu_first(tree, rays, ws)
    assert_first_equal(hit, t, rhit, rt)
    return int(roff[-1]), int((rhit >= 0).sum())


@pytest.mark.parametrize("segments", [False, True])
def test_reduced_clustered_rays(segments, ws):
    """2^18 clustered boxes: 2^14 rays through them (first hit) or 2^14
    short segments from inside them (all hits), both answered both ways."""
    w = workloads.by_name("clustered_segments" if segments else "clustered_rays", 1 / 64)
    say(f"case {w.name}: n={w.n} m={w.m}")
    hits, firsts = _both(w.prims, w.kind, w.code_bits, w.queries, ws)
    assert hits > w.m and firsts > w.m // 2


@pytest.mark.parametrize("split1,split2,leaf_mode,order", [
    (12, 7, 0, 0), (12, 7, 1, 0), (9, 4, 1, 1), (6, 3, 0, 1), (24, 24, 0, 0), (14, 9, 1, 0)])
def test_ray_query_schedules(split1, split2, leaf_mode, order, ws):
    """Every query schedule gives the oracle's all-hit CSR for rays and
    segments: split block sizes, leaf modes, Morton-ordered queries, unsplit
    walks and levels that overflow (long rays across a dense scene)."""
    import paper_2402_00665_amd as lb
    old = [lb.lbvh_tune("query_split1", split1), lb.lbvh_tune("query_split2", split2),
           lb.lbvh_tune("query_leaf_mode", leaf_mode), lb.lbvh_tune("query_order", order)]
    try:
        w = workloads.by_name("clustered_segments", 1 / 128)
        ref = oracle.build(w.kind, w.prims, w.code_bits)
        tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
        rng = np.random.default_rng([23, split1, split2, leaf_mode, order])
        long = workloads.segments_from(rng.random((500, 3), dtype=np.float32), 1.5, rng)
        rays = workloads.rays_toward(workloads.points_in_boxes(w.prims, 500, rng), rng)
        for q in (w.queries, long, rays):
            roff, ridx, _ = oracle.query_traverse(RAYS, q, ref)
            off, idx = gpu_query(tree, q, RAYS, ws)
            assert_query_equal(off, idx, roff, ridx)
    finally:
        for k, v in zip(("query_split1", "query_split2", "query_leaf_mode", "query_order"), old):
            lb.lbvh_tune(k, v)


def test_ray_edge_cases(ws):
    """Axis-parallel rays (zero direction components), directions whose
    reciprocal overflows, rays that graze faces and pass exactly through
    grid points, empty parameter intervals, tmin = -inf, negative
    directions; on a point grid (exact hits) and on boxes."""
    rng = np.random.default_rng(29)
    g = np.arange(8, dtype=np.float32) / 8
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    grid = np.ascontiguousarray(grid[rng.permutation(grid.shape[0])])
    inf = np.inf
    rays = [
        [0, 0.25, 0.5, 0, 1, 0, 0, inf],          # along a grid line: 8 exact hits
        [0.125, 0, 0.375, 0, 0, 1, 0, inf],
        [0.5, 0.5, 0, -inf, 0, 0, 1, inf],
        [0.5, 0.5, 1, 0, 0, 0, -1, inf],          # negative direction
        [0.5, 0.5, 0.5, 0, 0, 0, 0, inf],         # no direction: the point itself
        [0.51, 0.5, 0.5, 0, 0, 0, 0, inf],        # no direction, off the grid
        [0, 0.25, 0.5, 0, 1e-45, 0, 0, inf],      # reciprocal overflows: parallel
        [0, 0.25, 0.5, 0, -1e-45, 1e-45, 0, inf],
        [0, 0, 0, 0, 1, 1, 1, inf],               # the diagonal: 8 exact hits
        [0, 0, 0, 0.3, 1, 1, 1, 0.6],             # a piece of it
        [0, 0, 0, 0.6, 1, 1, 1, 0.3],             # empty interval
        [0, 0.25, 0.5, 0, 0.875, 0, 0, 1],        # segment ending on a point
        [-1, 0.25, 0.5, 0, 1, 0, 0, 1],           # segment ending on the first point
        [2, 2, 2, 0, 1, 1, 1, inf],               # pointing away
    ]
    rays = np.asarray(rays, np.float32)
    more = workloads.rays_toward(rng.random((300, 3), dtype=np.float32), rng)
    allr = np.concatenate([rays, more, workloads.segments_from(
        rng.random((300, 3), dtype=np.float32), 0.3, rng)])
    for bits in (30, 63):
        _both(grid, 0, bits, allr, ws)
    boxes = workloads.clustered_boxes(20000, rng, components=4, sigma=0.05)
    # rays along the faces of a few boxes (grazing)
    face = np.zeros((50, 8), np.float32)
    face[:, 0:3] = boxes[:50, 0:3]
    face[:, 4] = 1.0
    face[:, 7] = np.inf
    face[:, 0] = -0.5
    _both(boxes, 1, 30, np.concatenate([allr, face]), ws)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_tiny_trees(n, ws):
    """Empty, one-leaf and tiny trees: rays that hit and miss; m = 0."""
    import torch
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng([31, n])
    p = rng.random((n, 3), dtype=np.float32)
    rays = np.concatenate([workloads.rays_toward(p if n else rng.random((1, 3), dtype=np.float32),
                                                 rng),
                           workloads.rays_toward(rng.random((5, 3), dtype=np.float32), rng)])
    if n == 0:
        tree = lb.build(torch.empty((0, 3), dtype=torch.float32, device="cuda"), 30)
        off, idx = gpu_query(tree, rays, RAYS, ws)
        assert not off.any() and idx.size == 0
        hit, t = gpu_first(tree, rays, ws)
        assert (hit == -1).all() and np.isinf(t).all() and (t > 0).all()
    else:
        _both(p, 0, 30, rays, ws)
    tree, _ = gpu_build(p if n else rng.random((1, 3), dtype=np.float32), 0, 30, ws)
    hit, t = lb.query_first(tree, torch.empty((0, 8), dtype=torch.float32, device="cuda"),
                            workspace=ws)
    assert hit.numel() == 0 and t.numel() == 0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("segments", [False, True])
def test_full_size_rays(segments, ws):
    """The 2^24 clustered boxes with 2^20 rays (first hit) or 2^20
    segments (all hits), every result, in the default launch shapes."""
    name = "clustered_segments" if segments else "clustered_rays"
    say(f"full-size {name}: generating")
    w = workloads.by_name(name)
    oracle.threads(16)
    try:
        ref = oracle.build(w.kind, w.prims, w.code_bits)
        tree, _ = gpu_build(w.prims, w.kind, w.code_bits, ws)
        if segments:
            roff, ridx, _ = oracle.query_traverse(RAYS, w.queries, ref)
            off, idx = gpu_query(tree, w.queries, RAYS, ws)
            assert_query_equal(off, idx, roff, ridx)
            say(f"  {int(roff[-1])} hits")
        else:
            rhit, rt, _ = oracle.ray_first_traverse(w.queries, ref)
            hit, t = gpu_first(tree, w.queries, ws)
            assert_first_equal(hit, t, rhit, rt)
            say(f"  {int((rhit >= 0).sum())} rays hit")
    finally:
        oracle.threads(1)


def test_first_hit_error_word(ws):
    """A first-hit walk that spends its node-visit budget is reported by
    lbvh_query_check; the next call clears the word."""
    import torch
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng(37)
    p = rng.random((5000, 3), dtype=np.float32)
    tree, _ = gpu_build(p, 0, 30, ws)
    rays = torch.from_numpy(workloads.rays_toward(p[:64], rng)).cuda()
    qws = lb.Workspace()
    old = lb.lbvh_tune("query_walk_budget", 3)
    try:
        lb.query_first(tree, rays, workspace=qws)
        with pytest.raises(lb.LbvhError):
            lb.check_query(qws, 64)
    finally:
        lb.lbvh_tune("query_walk_budget", old)
    lb.query_first(tree, rays, workspace=qws)
    lb.check_query(qws, 64)
