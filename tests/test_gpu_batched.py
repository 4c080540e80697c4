"""GPU parity of the batched build and batched queries: every scene's tree
and query results must equal the oracle run on that scene alone
(tolerance 0), and a HIP-graph replay must give the same bits each time."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import first_mismatch, say

pytestmark = pytest.mark.gpu


def run_batched(prims, seg_off, bits, kind, max_scene=None, ws=None, shift=0):
    """shift: floats of padding before the primitives in their device
    buffer, so that shift=2 gives an array that is 8- but not 16-byte
    aligned."""
    import torch
    import paper_2402_00665_amd as lb
    sizes = np.diff(seg_off)
    max_scene = int(sizes.max()) if max_scene is None else max_scene
    say(f"  batched build: S={len(sizes)} N={int(seg_off[-1])} bits={bits} kind={kind} "
        f"max_scene={max_scene} shift={shift}")
    host = torch.from_numpy(np.ascontiguousarray(prims))
    flat = torch.zeros(host.numel() + shift, dtype=torch.float32, device="cuda")
    dp = flat[shift:].view(host.shape)
    dp.copy_(host)
    ds = torch.from_numpy(np.ascontiguousarray(seg_off, dtype=np.int64)).cuda()
    b = lb.build_batched(dp, ds, bits, max_scene, kind=kind, workspace=ws)
    return b, dp, ds


def check_scene(b, s, seg_off, ref, nodes_h, codes_h, perm_h):
    a, e = int(seg_off[s]), int(seg_off[s + 1])
    n = e - a
    assert ref.n == n
    if n == 0:
        return
    rec = nodes_h[2 * a: 2 * a + 2 * n - 1]
    f = rec.view(np.float32)
    aabb = np.concatenate([f[:, 0:3], f[:, 4:7]], axis=1)
    codes = codes_h[a:e].astype(np.uint64)
    for name, got, exp in [("codes", codes, ref.sorted), ("leaf_perm", perm_h[a:e], ref.perm),
                           ("perm field", rec[n - 1:, 3], ref.perm), ("left", rec[: n - 1, 3], ref.left),
                           ("rope", rec[:, 7], ref.rope)]:
        k = first_mismatch(got, exp)
        assert k is None, f"scene {s} {name}[{k}]: gpu {got[k]} oracle {exp[k]}"
    bad = np.flatnonzero(~np.all(aabb == ref.aabb, axis=1))
    assert bad.size == 0, f"scene {s} aabb[{bad[0]}]"


def host_arrays(b):
    nodes_h = b.nodes.cpu().numpy()
    c = b.codes.cpu().numpy()
    codes_h = c.view(np.uint32) if b.code_bits == 30 else c.view(np.uint64)
    return nodes_h, codes_h, b.leaf_perm.cpu().numpy()


def batched_parity(prims, seg_off, bits, kind, queries=None, qseg=None, qkind=0, ws=None,
                   check_every=1, shift=0):
    import torch
    import paper_2402_00665_amd as lb
    b, dp, ds = run_batched(prims, seg_off, bits, kind, ws=ws, shift=shift)
    lb.check_batched(b)
    nodes_h, codes_h, perm_h = host_arrays(b)
    S = len(seg_off) - 1
    refs = {}
    for s in range(0, S, check_every):
        a, e = int(seg_off[s]), int(seg_off[s + 1])
        refs[s] = oracle.build(kind, prims[a:e], bits)
        check_scene(b, s, seg_off, refs[s], nodes_h, codes_h, perm_h)
    if queries is None:
        return b
    dq = torch.from_numpy(np.ascontiguousarray(queries)).cuda()
    dqs = torch.from_numpy(np.ascontiguousarray(qseg, dtype=np.int64)).cuda()
    off, idx = lb.query_batched(b, dq, dqs, qkind)
    torch.cuda.synchronize()
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    for s in range(0, S, check_every):
        qa, qe = int(qseg[s]), int(qseg[s + 1])
        roff, ridx, _ = oracle.query_traverse(qkind, queries[qa:qe], refs[s])
        got_off = off[qa:qe + 1] - off[qa]
        k = first_mismatch(got_off, roff)
        assert k is None, f"scene {s} query offsets[{k}]"
        k = first_mismatch(idx[off[qa]:off[qe]], ridx)
        assert k is None, f"scene {s} query indices[{k}]"
    return b


SIZES = [0, 1, 2, 3, 33, 4095, 4096, 4097, 1025, 70000, 0, 5, 8193, 1024, 1023, 300000]


@pytest.mark.parametrize("bits", [30, 63])
@pytest.mark.parametrize("kind", [0, 1])
def test_mixed_scene_sizes(kind, bits):
    rng = np.random.default_rng([20, kind, bits])
    sizes = np.array(SIZES, np.int64)
    seg = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=seg[1:])
    N = int(seg[-1])
    if kind == 0:
        prims = rng.random((N, 3), dtype=np.float32)
    else:
        c = rng.random((N, 3))
        s = rng.random((N, 3)) * 0.01
        prims = np.concatenate([c - s, c + s], 1).astype(np.float32)
    m_per = 7
    q = workloads.spheres(rng.random((len(sizes) * m_per, 3), dtype=np.float32), np.float32(0.05))
    qseg = np.arange(len(sizes) + 1, dtype=np.int64) * m_per
    batched_parity(prims, seg, bits, kind, q, qseg, 0)


@pytest.mark.parametrize("kind", [0, 1])
def test_prims_8_byte_aligned(kind):
    """Primitives 8 bytes past a 16-byte boundary, scenes starting at every
    residue modulo 4: the scene loader's head, 48-byte groups and tail must
    cover each scene exactly once."""
    import torch
    rng = np.random.default_rng([22, kind])
    sizes = np.array([1, 2, 3, 4, 5, 6, 7, 9, 1030, 2, 4099, 3, 20000, 1, 13], np.int64)
    seg = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=seg[1:])
    N = int(seg[-1])
    if kind == 0:
        prims = rng.random((N, 3), dtype=np.float32)
    else:
        c = rng.random((N, 3))
        h = rng.random((N, 3)) * 0.01
        prims = np.concatenate([c - h, c + h], 1).astype(np.float32)
    b = batched_parity(prims, seg, 63, kind, shift=2)
    assert b is not None
    torch.cuda.synchronize()


def test_batched_workload_reduced():
    pts, off, q, qoff = workloads.batched(S=160, m_per=64)
    batched_parity(pts, off, 63, 0, q, qoff, 0)


def test_batched_box_queries_and_duplicates():
    rng = np.random.default_rng(21)
    sizes = np.array([5000, 12000, 3, 64, 9000], np.int64)
    seg = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=seg[1:])
    pts = (rng.integers(0, 5, size=(int(seg[-1]), 3)) / 4).astype(np.float32)   # heavy duplicates
    c = rng.random((50, 3))
    qb = np.concatenate([c - 0.2, c + 0.2], 1).astype(np.float32)
    qseg = np.array([0, 10, 20, 30, 40, 50], np.int64)
    batched_parity(pts, seg, 30, 0, qb, qseg, 1)


def test_max_scene_too_small_is_reported():
    """max_scene = 100 launches no level above the 1024-leaf blocks, so a
    scene of 3000 points cannot be finished: the check call reports it."""
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng(22)
    seg = np.array([0, 3000, 5000], np.int64)
    pts = rng.random((5000, 3), dtype=np.float32)
    b, _, _ = run_batched(pts, seg, 30, 0, max_scene=100)
    with pytest.raises(lb.LbvhError) as e:
        lb.check_batched(b)
    assert e.value.status == lb.LBVH_EDEVICE


def test_max_scene_below_size_within_cover_is_exact():
    """max_scene = 1500 launches one level above the 1024-leaf blocks
    (covering 262144 leaves), so a 3000-point scene is still built exactly."""
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng(24)
    seg = np.array([0, 3000, 5000], np.int64)
    pts = rng.random((5000, 3), dtype=np.float32)
    b, _, _ = run_batched(pts, seg, 30, 0, max_scene=1500)
    lb.check_batched(b)
    nodes_h, codes_h, perm_h = host_arrays(b)
    for s in range(2):
        ref = oracle.build(0, pts[seg[s]:seg[s + 1]], 30)
        check_scene(b, s, seg, ref, nodes_h, codes_h, perm_h)


@pytest.fixture(params=[0, 1], ids=["segmented", "per_scene"])
def sort_mode(request):
    """Both sort schedules of the batched build: segmented onesweep passes
    over all scenes, and one block per scene."""
    import paper_2402_00665_amd as lb
    old = lb.lbvh_tune("batch_sort_mode", request.param)
    yield request.param
    lb.lbvh_tune("batch_sort_mode", old)


def test_graph_capture_replays_identically(sort_mode):
    """The batched build and count enqueue kernels only, so they can be
    captured in a HIP graph; every replay must reproduce the eager bits."""
    import torch
    import paper_2402_00665_amd as lb
    pts, off, q, qoff = workloads.batched(S=64, m_per=64)
    max_scene = int(np.diff(off).max())
    dp = torch.from_numpy(pts).cuda()
    ds = torch.from_numpy(off).cuda()
    dq = torch.from_numpy(q).cuda()
    dqs = torch.from_numpy(qoff).cuda()
    ws, qws = lb.Workspace(), lb.Workspace()
    b = lb.build_batched(dp, ds, 63, max_scene, workspace=ws)
    offsets = torch.empty(q.shape[0] + 1, dtype=torch.int64, device="cuda")
    qbuf = qws.get(lb.lbvh_query_batched_workspace_bytes(q.shape[0]))

    def enqueue():
        lb._check(lb.lbvh_build_batched(0, dp.data_ptr(), b.desc, b.workspace.data_ptr(),
                                        b.workspace.numel(), lb._stream()), "build")
        lb._check(lb.lbvh_query_batched_spheres_count(b.desc, dq.data_ptr(), dqs.data_ptr(),
                                                      q.shape[0], offsets.data_ptr(), qbuf.data_ptr(),
                                                      qbuf.numel(), lb._stream()), "count")

    # records the build owns: scene s has 2n_s-1 of its 2n_s slots
    used = np.zeros(b.nodes.shape[0], bool)
    for a, e in zip(off[:-1], off[1:]):
        used[2 * a: 2 * a + max(2 * (e - a) - 1, 0)] = True
    used = torch.from_numpy(used).cuda()
    enqueue()
    torch.cuda.synchronize()
    eager_nodes, eager_off = b.nodes[used].clone(), offsets.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            enqueue()
    torch.cuda.synchronize()
    for r in range(4):
        b.nodes.zero_()
        offsets.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.nodes[used], eager_nodes), f"replay {r}: nodes differ"
        assert torch.equal(offsets, eager_off), f"replay {r}: offsets differ"
        x = torch.rand(1000, device="cuda").sum()   # eager work between replays
        x.item()
    lb.check_batched(b)


@pytest.mark.timeout(900)
def test_batched_workload_full_size(sort_mode):
    """4096 scenes, sizes log-uniform in [32, 65536] (35M points), 63-bit
    codes, 64 spheres per scene: every scene's tree and query results
    checked against the oracle run on that scene alone."""
    say(f"full batched workload (sort mode {sort_mode}): generating")
    pts, off, q, qoff = workloads.batched()
    oracle.threads(16)
    try:
        batched_parity(pts, off, 63, 0, q, qoff, 0, check_every=1)
    finally:
        oracle.threads(1)


@pytest.mark.parametrize("shape", range(4))
@pytest.mark.parametrize("bits", [30, 63])
def test_scene_sort_widths_and_sizes(bits, shape):
    """The one-block-per-scene sort with every block shape and digit
    width: empty and one-point scenes, scenes around the 4096- and
    8192-key tiles, a 65536-point scene, scenes whose top digit value
    holds exactly 4096 keys and 4097 keys (runs of whole digit values on
    chip, and the pass-per-digit form), duplicate codes; every tree equals
    the oracle's.  A batch with a scene above 262144 points, asked for in
    this mode, is built by the segmented passes and is checked too."""
    import paper_2402_00665_amd as lb
    old = {k: lb.lbvh_tune(k) for k in ("batch_sort_mode", "batch_sort_variant", "radix_bits32",
                                        "radix_bits64")}
    lb.lbvh_tune("batch_sort_mode", 1)
    lb.lbvh_tune("batch_sort_variant", shape)
    try:
        rng = np.random.default_rng([29, bits])
        sizes = np.array([4097, 1, 4096, 0, 65536, 6000, 4095, 16384, 8193, 2, 0, 3, 8191, 8192,
                          28000, 28001], np.int64)
        seg = np.zeros(len(sizes) + 1, np.int64)
        np.cumsum(sizes, out=seg[1:])
        pts = rng.random((int(seg[-1]), 3), dtype=np.float32)
        pts[seg[5]:seg[6]] = pts[seg[5]]                     # one scene of equal points
        pts[seg[7]:seg[8]:3] = pts[seg[7]]                    # duplicates in another
        for j, zeros in ((14, 4096), (15, 4097)):
            # the origin's top digit value holds exactly `zeros` keys: the
            # other points lie in [0.3, 1]^3, away from every axis' first
            # quarter, and one at (1, 1, 1) fixes the scene box
            a, e = int(seg[j]), int(seg[j + 1])
            pts[a:e] = (np.float32(0.3) + np.float32(0.7) * pts[a:e]).astype(np.float32)
            pts[a:a + zeros] = 0.0
            pts[e - 1] = 1.0
        for width in ((8, 10) if bits == 30 else (8, 9, 11)):
            lb.lbvh_tune("radix_bits32" if bits == 30 else "radix_bits64", width)
            say(f"  per-scene sort, {width}-bit digits, {bits}-bit codes")
            batched_parity(pts, seg, bits, 0)
            boxes = np.concatenate([pts, pts + 1e-3], 1).astype(np.float32)
            batched_parity(boxes, seg, bits, 1)
        if shape == 0:
            big = np.concatenate([pts[:20000], rng.random((270000, 3), dtype=np.float32)])
            bseg = np.array([0, 20000, 290000], np.int64)
            say("  per-scene sort asked for with a 270000-point scene")
            batched_parity(big, bseg, bits, 0)
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)


@pytest.mark.parametrize("variant", range(4))
def test_batched_tile_variants(variant):
    """Every segmented radix tile shape, with every digit width, gives the
    same trees (tolerance 0)."""
    import paper_2402_00665_amd as lb
    old = {k: lb.lbvh_tune(k) for k in ("batch_sort_variant", "radix_bits32", "radix_bits64")}
    lb.lbvh_tune("batch_sort_variant", variant)
    try:
        rng = np.random.default_rng([23, variant])
        sizes = np.array([4097, 1, 2048, 0, 100003, 6000, 2047, 16384, 8193, 4095], np.int64)
        seg = np.zeros(len(sizes) + 1, np.int64)
        np.cumsum(sizes, out=seg[1:])
        pts = rng.random((int(seg[-1]), 3), dtype=np.float32)
        for b32, b64 in ((8, 8), (10, 9), (10, 11)):
            lb.lbvh_tune("radix_bits32", b32)
            lb.lbvh_tune("radix_bits64", b64)
            for bits in (30, 63):
                say(f"  batched digits {b32 if bits == 30 else b64} bits")
                batched_parity(pts, seg, bits, 0)
    finally:
        for k, v in old.items():
            lb.lbvh_tune(k, v)


def test_batched_query_error_word():
    """The batched count call clears its error word; a capped walk budget is
    reported, and the fill stays inside the counted slots."""
    import torch
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng(77)
    sizes = np.array([5000, 300, 70000, 1], np.int64)
    seg = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=seg[1:])
    pts = torch.from_numpy(rng.random((int(seg[-1]), 3), dtype=np.float32)).cuda()
    dseg = torch.from_numpy(seg).cuda()
    b = lb.build_batched(pts, dseg, 63, int(sizes.max()))
    lb.check_batched(b)
    qn = np.array([100, 100, 100, 100], np.int64)
    qseg = np.zeros(5, np.int64)
    np.cumsum(qn, out=qseg[1:])
    q = np.empty((400, 4), np.float32)
    q[:, :3] = rng.random((400, 3), dtype=np.float32)
    q[:, 3] = 0.2
    dq, dqs = torch.from_numpy(q).cuda(), torch.from_numpy(qseg).cuda()
    qws = lb.Workspace()
    old = lb.lbvh_tune("query_walk_budget")
    try:
        off, idx = lb.query_batched(b, dq, dqs, 0, workspace=qws)
        lb.check_query(qws, 400, batched=True)
        lb.lbvh_tune("query_walk_budget", 5)
        off = lb.query_batched_count(b, dq, dqs, 0, qws)
        with pytest.raises(lb.LbvhError) as e:
            lb.check_query(qws, 400, batched=True)
        assert e.value.status == lb.LBVH_EDEVICE
        total = int(off[-1].item())
        buf = torch.full((total + 4096,), -7, dtype=torch.int32, device="cuda")
        lb.query_batched_fill(b, dq, dqs, 0, off, buf, qws)
        torch.cuda.synchronize()
        assert bool((buf[total:] == -7).all()), "fill wrote past the counted hits"
        lb.lbvh_tune("query_walk_budget", 0)
        off2, idx2 = lb.query_batched(b, dq, dqs, 0, workspace=qws)
        lb.check_query(qws, 400, batched=True)
        # uncapped again: the same answers as the first clean call
        first_off, first_idx = lb.query_batched(b, dq, dqs, 0)
        assert torch.equal(off2, first_off) and torch.equal(idx2, first_idx)
        assert torch.equal(idx2, idx)
    finally:
        lb.lbvh_tune("query_walk_budget", old)
