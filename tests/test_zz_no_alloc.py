"""The allocation-free build (lbvh_build_noalloc) through the C ABI: its
trees are bit-identical to lbvh_build's with a workspace, on consecutive
calls that reuse the one fixed scratch (a large call, then a smaller one of
another kind and code width, then the large one again), and to the
oracle's; sizes above its limit are refused before anything is enqueued."""

import numpy as np
import pytest

import oracle
from gpu_util import assert_tree_equal, say

pytestmark = pytest.mark.gpu


def _noalloc(prims, kind, bits, err):
    import torch
    import paper_2402_00665_amd as lb
    n = prims.shape[0]
    tree = lb.alloc_tree(n, bits)
    err.fill_(-1)
    rc = lb.lbvh_build_noalloc(kind, prims.data_ptr(), n, bits, tree.desc, err.data_ptr(),
                               int(torch.cuda.current_stream().cuda_stream))
    assert rc == lb.LBVH_OK, lb.lbvh_strerror(rc)
    tree.kind = kind
    torch.cuda.synchronize()
    assert int(err.item()) == 0, "the build flagged a device error"
    return tree


def _with_workspace(prims, kind, bits):
    import torch
    import paper_2402_00665_amd as lb
    n = prims.shape[0]
    tree = lb.alloc_tree(n, bits)
    wsb = lb.lbvh_build_workspace_bytes(n, bits, kind)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    rc = lb.lbvh_build(kind, prims.data_ptr(), n, bits, tree.desc, ws.data_ptr(), wsb,
                       int(torch.cuda.current_stream().cuda_stream))
    assert rc == lb.LBVH_OK, lb.lbvh_strerror(rc)
    assert lb.lbvh_build_check(ws.data_ptr(), n, bits, kind,
                               int(torch.cuda.current_stream().cuda_stream)) == lb.LBVH_OK
    return tree


def test_noalloc_matches_the_workspace_build():
    import torch
    import paper_2402_00665_amd as lb
    rng = np.random.default_rng(97)
    err = torch.empty(1, dtype=torch.int32, device="cuda")
    big = lb.LBVH_NOALLOC_MAX_PRIMS
    c = rng.random((big, 3), dtype=np.float32)
    s = (rng.random((big, 3), dtype=np.float32) * 1e-3).astype(np.float32)
    boxes = np.concatenate([c - s, c + s], 1).astype(np.float32)
    pts = rng.random((77777, 3), dtype=np.float32)
    pts[::7] = pts[3]                                   # duplicate codes
    cases = [(boxes, 1, 63), (pts, 0, 30), (boxes, 1, 63)]
    for prims, kind, bits in cases:
        say(f"noalloc build: n={prims.shape[0]} kind={kind} bits={bits}")
        dev = torch.from_numpy(prims).cuda()
        got = _noalloc(dev, kind, bits, err)
        ref = _with_workspace(dev, kind, bits)
        for name in ("nodes", "codes", "leaf_perm"):
            a, b = getattr(got, name), getattr(ref, name)
            assert torch.equal(a, b), f"{name} differs from the workspace build"
    # and the smaller tree against the oracle, element by element
    dev = torch.from_numpy(pts).cuda()
    assert_tree_equal(_noalloc(dev, 0, 30, err), oracle.build(0, pts, 30))


def test_noalloc_limits_and_arguments():
    import torch
    import paper_2402_00665_amd as lb
    stream = int(torch.cuda.current_stream().cuda_stream)
    t = lb.lbvh_tree(0, 0, 0, None, None, None)
    n = lb.LBVH_NOALLOC_MAX_PRIMS + 1
    assert lb.lbvh_build_noalloc(0, 16, n, 30, t, None, stream) == lb.LBVH_ELIMIT
    assert lb.lbvh_build_noalloc(0, None, 10, 31, t, None, stream) == lb.LBVH_EINVAL
    assert lb.lbvh_build_noalloc(0, None, 10, 30, t, None, stream) == lb.LBVH_EINVAL
    assert lb.lbvh_build_noalloc(0, 16, 10, 30, t, 2, stream) == lb.LBVH_EINVAL   # misaligned flag
    assert lb.lbvh_build_noalloc(0, None, 0, 30, t, None, stream) == lb.LBVH_OK and t.n == 0
    assert "scratch" in lb.lbvh_strerror(lb.LBVH_ELIMIT)
    # one point: a one-leaf tree
    p = torch.rand(1, 3, device="cuda")
    tree = lb.build_noalloc(p, 63)
    torch.cuda.synchronize()
    assert tree.n == 1 and int(tree.rope[0]) == -1 and int(tree.perm[0]) == 0
