"""CPU oracle for the rope-LBVH build and its range queries.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``; the library
(``paper_2402_00665_amd``) never imports it.

Thin ctypes wrapper over ``lbvh_oracle.c`` (plain, single-threaded C built by
``oracle/make_lib.py``).  Each function states the definition it follows; the C
file's header lists the readings taken where the paper is silent.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbvh_oracle.so")

POINTS, BOXES = 0, 1
SPHERES, QBOXES, RAYS = 0, 1, 2

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import make_lib
            make_lib.build()
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int
        lib.orc_scene_box.argtypes = [i32, P, i64, P]
        lib.orc_scales.argtypes = [P, i32, P]
        lib.orc_scales.restype = None
        lib.orc_morton.argtypes = [i32, P, i64, i32, P, P]
        lib.orc_sort.argtypes = [P, i64, P, P]
        lib.orc_delta.argtypes = [P, i64, P]
        lib.orc_topdown.argtypes = [P, i64, P, P, P, P]
        lib.orc_ropes.argtypes = [P, P, i64, P]
        lib.orc_aabbs.argtypes = [i32, P, P, P, P, i64, P]
        lib.orc_build.argtypes = [i32, P, i64, i32] + [P] * 11
        lib.orc_pred_sphere.argtypes = [P, P]
        lib.orc_pred_box.argtypes = [P, P]
        lib.orc_query_brute.argtypes = [i32, P, i64, i32, P, P, i64, P, i64]
        lib.orc_query_brute.restype = i64
        lib.orc_query_traverse.argtypes = [i32, P, i64, i64, P, P, P, P, P, P]
        lib.orc_query_traverse.restype = i64
        lib.orc_query_fill.argtypes = [i32, P, i64, i64, P, P, P, P, P, P]
        lib.orc_pred_ray.argtypes = [P, P, P]
        lib.orc_ray_first_brute.argtypes = [P, i64, i32, P, P, i64, P]
        lib.orc_ray_first_brute.restype = C.c_int32
        lib.orc_ray_first_traverse.argtypes = [P, i64, i64, P, P, P, P, P, P, P]
        lib.orc_threads.argtypes = [i32]
        lib.orc_threads.restype = None
        lib.orc_threads(1)
        _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _f32(a, width):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == width, a.shape
    return a


def _kind_width(kind):
    return 3 if kind == POINTS else 6


def scene_box(kind: int, prims: np.ndarray) -> np.ndarray:
    """Componentwise min of lower corners and max of upper corners."""
    prims = _f32(prims, _kind_width(kind))
    out = np.zeros(6, np.float32)
    _check(_load().orc_scene_box(kind, _p(prims), prims.shape[0], _p(out)), "scene_box")
    return out


def scales(scene: np.ndarray, bits: int) -> np.ndarray:
    scene = np.ascontiguousarray(scene, dtype=np.float32)
    out = np.zeros(3, np.float32)
    _load().orc_scales(_p(scene), bits, _p(out))
    return out


def morton(kind: int, prims: np.ndarray, bits: int, scene: np.ndarray | None = None) -> np.ndarray:
    """Morton code (uint64) of each primitive's centroid, input order."""
    prims = _f32(prims, _kind_width(kind))
    if scene is None:
        scene = scene_box(kind, prims)
    scene = np.ascontiguousarray(scene, dtype=np.float32)
    codes = np.zeros(prims.shape[0], np.uint64)
    _check(_load().orc_morton(kind, _p(prims), prims.shape[0], bits, _p(scene), _p(codes)), "morton")
    return codes


def sort(codes: np.ndarray):
    """Stable ascending sort: (sorted codes, permutation of input indices)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    n = codes.shape[0]
    s = np.zeros(n, np.uint64)
    perm = np.zeros(n, np.int32)
    _check(_load().orc_sort(_p(codes), n, _p(s), _p(perm)), "sort")
    return s, perm


def delta(sorted_codes: np.ndarray) -> np.ndarray:
    """delta*(i), i in [0, n-2], as the rank of the highest differing bit of
    the augmented keys (255 would be +inf and never appears inside)."""
    sc = np.ascontiguousarray(sorted_codes, dtype=np.uint64)
    n = sc.shape[0]
    d = np.zeros(max(n - 1, 0), np.uint8)
    if n > 1:
        _check(_load().orc_delta(_p(sc), n, _p(d)), "delta")
    return d


def topdown(delta_arr: np.ndarray, n: int):
    """Top-down Karras tree: (left, right, range_lo, range_hi), each [n-1]."""
    d = np.ascontiguousarray(delta_arr, dtype=np.uint8)
    ni = max(n - 1, 0)
    left = np.zeros(ni, np.int32); right = np.zeros(ni, np.int32)
    rlo = np.zeros(ni, np.int32); rhi = np.zeros(ni, np.int32)
    _check(_load().orc_topdown(_p(d), n, _p(left), _p(right), _p(rlo), _p(rhi)), "topdown")
    return left, right, rlo, rhi


def ropes(left: np.ndarray, right: np.ndarray, n: int) -> np.ndarray:
    """Skip-connections by an explicit depth-first walk, [2n-1]."""
    rope = np.zeros(max(2 * n - 1, 0), np.int32)
    if n > 0:
        _check(_load().orc_ropes(_p(np.ascontiguousarray(left, np.int32)),
                                 _p(np.ascontiguousarray(right, np.int32)), n, _p(rope)), "ropes")
    return rope


@dataclass
class Tree:
    n: int
    bits: int
    kind: int
    scene: np.ndarray      # [6]
    codes: np.ndarray      # [n] uint64, input order
    sorted: np.ndarray     # [n] uint64
    perm: np.ndarray       # [n] int32: leaf k -> primitive index
    delta: np.ndarray      # [n-1] uint8
    left: np.ndarray       # [n-1] unified ids
    right: np.ndarray      # [n-1] unified ids
    rlo: np.ndarray        # [n-1]
    rhi: np.ndarray        # [n-1]
    rope: np.ndarray       # [2n-1] unified ids or -1
    aabb: np.ndarray       # [2n-1, 6]


def build(kind: int, prims: np.ndarray, bits: int) -> Tree:
    """Whole build: scene box, Morton codes, stable sort, delta*, top-down
    tree, DFS ropes and range-union boxes."""
    prims = _f32(prims, _kind_width(kind))
    n = prims.shape[0]
    ni, nt = max(n - 1, 0), max(2 * n - 1, 0)
    t = Tree(n, bits, kind, np.zeros(6, np.float32), np.zeros(n, np.uint64),
             np.zeros(n, np.uint64), np.zeros(n, np.int32), np.zeros(ni, np.uint8),
             np.zeros(ni, np.int32), np.zeros(ni, np.int32), np.zeros(ni, np.int32),
             np.zeros(ni, np.int32), np.zeros(nt, np.int32), np.zeros((nt, 6), np.float32))
    if n == 0:
        return t
    rc = _load().orc_build(kind, _p(prims), n, bits, _p(t.scene), _p(t.codes), _p(t.sorted),
                           _p(t.perm), _p(t.delta), _p(t.left), _p(t.right), _p(t.rlo),
                           _p(t.rhi), _p(t.rope), _p(t.aabb))
    _check(rc, "build")
    return t


def tree_from_sorted(sorted_codes: np.ndarray) -> Tree:
    """Topology and ropes for already-sorted codes (no primitives: boxes and
    permutation are left empty).  Used for the paper's worked example."""
    sc = np.ascontiguousarray(sorted_codes, dtype=np.uint64)
    n = sc.shape[0]
    d = delta(sc)
    left, right, rlo, rhi = topdown(d, n)
    rope = ropes(left, right, n)
    return Tree(n, 0, -1, np.zeros(6, np.float32), sc.copy(), sc, np.arange(n, dtype=np.int32),
                d, left, right, rlo, rhi, rope, np.zeros((max(2 * n - 1, 0), 6), np.float32))


def pred_sphere(box, q) -> bool:
    box = np.ascontiguousarray(box, np.float32); q = np.ascontiguousarray(q, np.float32)
    return bool(_load().orc_pred_sphere(_p(box), _p(q)))


def pred_box(box, q) -> bool:
    box = np.ascontiguousarray(box, np.float32); q = np.ascontiguousarray(q, np.float32)
    return bool(_load().orc_pred_box(_p(box), _p(q)))


def _qwidth(qkind: int) -> int:
    return {SPHERES: 4, QBOXES: 6, RAYS: 8}[qkind]


def pred_ray(box, q):
    """Ray / segment q = (o.xyz, tmin, d.xyz, tmax) against a box:
    (hit, entry parameter or None)."""
    box = np.ascontiguousarray(box, np.float32); q = np.ascontiguousarray(q, np.float32)
    e = np.zeros(1, np.float32)
    hit = bool(_load().orc_pred_ray(_p(box), _p(q), _p(e)))
    return hit, (float(e[0]) if hit else None)


def query_brute(qkind: int, queries: np.ndarray, j: int, kind: int, prims: np.ndarray,
                perm: np.ndarray) -> np.ndarray:
    """All primitives satisfying query j's predicate, in ascending leaf order."""
    queries = _f32(queries, _qwidth(qkind))
    prims = _f32(prims, _kind_width(kind))
    perm = np.ascontiguousarray(perm, np.int32)
    n = prims.shape[0]
    out = np.zeros(max(n, 1), np.int32)
    h = _load().orc_query_brute(qkind, _p(queries), j, kind, _p(prims), _p(perm), n, _p(out), n)
    return out[:h].copy()


def query_traverse(qkind: int, queries: np.ndarray, tree: Tree):
    """Alg. 1 on the oracle tree for every query: (offsets[m+1] int64,
    indices int32 in traversal order, total node visits)."""
    queries = _f32(queries, _qwidth(qkind))
    m = queries.shape[0]
    lib = _load()
    offsets = np.zeros(m + 1, np.int64)
    vis = np.zeros(1, np.int64)
    total = lib.orc_query_traverse(qkind, _p(queries), m, tree.n, _p(tree.left), _p(tree.rope),
                                   _p(tree.aabb), _p(tree.perm), _p(offsets), _p(vis))
    idx = np.zeros(max(total, 1), np.int32)
    lib.orc_query_fill(qkind, _p(queries), m, tree.n, _p(tree.left), _p(tree.rope),
                       _p(tree.aabb), _p(tree.perm), _p(offsets), _p(idx))
    return offsets, idx[:total].copy(), int(vis[0])


def ray_first_brute(rays: np.ndarray, j: int, kind: int, prims: np.ndarray, perm: np.ndarray):
    """First hit of ray j by brute force over all primitives in leaf order:
    (primitive id or -1, entry parameter; +inf if none)."""
    rays = _f32(rays, 8)
    prims = _f32(prims, _kind_width(kind))
    perm = np.ascontiguousarray(perm, np.int32)
    t = np.zeros(1, np.float32)
    h = _load().orc_ray_first_brute(_p(rays), j, kind, _p(prims), _p(perm), prims.shape[0], _p(t))
    return int(h), float(t[0])


def ray_first_traverse(rays: np.ndarray, tree: Tree):
    """First hit of every ray by Alg. 1 with pruning on the oracle tree:
    (hit int32 [m] primitive or -1, t float32 [m], total node visits)."""
    rays = _f32(rays, 8)
    m = rays.shape[0]
    hit = np.zeros(m, np.int32)
    t = np.zeros(m, np.float32)
    vis = np.zeros(1, np.int64)
    _load().orc_ray_first_traverse(_p(rays), m, tree.n, _p(tree.left), _p(tree.rope),
                                   _p(tree.aabb), _p(tree.perm), _p(hit), _p(t), _p(vis))
    return hit, t, int(vis[0])


def threads(t: int):
    """Host threads of the oracle's independent loops (1 = sequential); the
    results are the same for every count."""
    _load().orc_threads(int(t))
