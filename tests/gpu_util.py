"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare every output with the oracle, element by element, tolerance 0."""

from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_build(prims: np.ndarray, kind: int, bits: int, ws=None):
    import torch
    import paper_2402_00665_amd as lb
    say(f"  gpu build: kind={kind} n={prims.shape[0]} bits={bits}")
    dev = torch.from_numpy(np.ascontiguousarray(prims)).cuda()
    tree = lb.build(dev, bits, kind=kind, workspace=ws)
    lb.check_build(tree)
    torch.cuda.synchronize()
    return tree, dev


def host_tree(tree):
    """numpy views of a GPU tree: (codes u64, perm, left, rope, aabb[2n-1,6])."""
    n = tree.n
    if n == 0:
        z = np.zeros(0, np.int32)
        return np.zeros(0, np.uint64), z, z, z, np.zeros((0, 6), np.float32)
    nodes = tree.nodes.cpu().numpy()
    codes = tree.codes.cpu().numpy()[:n]
    codes = codes.view(np.uint32 if tree.code_bits == 30 else np.uint64).astype(np.uint64)
    f = nodes.view(np.float32)
    aabb = np.concatenate([f[:, 0:3], f[:, 4:7]], axis=1)
    perm = nodes[n - 1:, 3].copy()
    assert np.array_equal(tree.leaf_perm.cpu().numpy()[:n], perm), "leaf_perm != leaf records"
    return codes, perm, nodes[: n - 1, 3].copy(), nodes[:, 7].copy(), aabb


def first_mismatch(a, b):
    idx = np.flatnonzero(np.asarray(a) != np.asarray(b))
    return None if idx.size == 0 else int(idx[0])


def assert_tree_equal(tree, ref: oracle.Tree):
    codes, perm, left, rope, aabb = host_tree(tree)
    assert tree.n == ref.n
    for name, got, exp in [("codes", codes, ref.sorted), ("perm", perm, ref.perm),
                           ("left", left, ref.left), ("rope", rope, ref.rope)]:
        assert got.shape == exp.shape, (name, got.shape, exp.shape)
        k = first_mismatch(got, exp)
        assert k is None, f"{name}[{k}]: gpu {got[k]} oracle {exp[k]}"
    # binary32 equality (signed zeros compare equal)
    bad = np.flatnonzero(~np.all(aabb == ref.aabb, axis=1))
    assert bad.size == 0, f"aabb[{bad[0]}]: gpu {aabb[bad[0]]} oracle {ref.aabb[bad[0]]}"


def gpu_query(tree, queries: np.ndarray, qkind: int, ws=None):
    import torch
    import paper_2402_00665_amd as lb
    say(f"  gpu query: qkind={qkind} m={queries.shape[0]} n={tree.n}")
    q = torch.from_numpy(np.ascontiguousarray(queries)).cuda()
    off, idx = lb.query(tree, q, qkind, workspace=ws)
    torch.cuda.synchronize()
    return off.cpu().numpy(), idx.cpu().numpy()


def assert_query_equal(off, idx, ref_off, ref_idx):
    k = first_mismatch(off, ref_off)
    assert k is None, f"offsets[{k}]: gpu {off[k]} oracle {ref_off[k]}"
    k = first_mismatch(idx, ref_idx)
    assert k is None, f"indices[{k}]: gpu {idx[k]} oracle {ref_idx[k]}"
