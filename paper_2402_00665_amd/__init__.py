"""Python binding of the MI355X rope-LBVH library (``liblbvh.so``).

Two layers, both argument marshalling only (every step of the build and of
the queries runs in the library's HIP kernels):

* ``lbvh_*`` functions with the names and arguments of the C ABI in
  ``include/lbvh.h`` (device pointers as ints, the tree descriptor as a
  ctypes structure, the stream as a hipStream_t int);
* ``build`` / ``query`` / ``Tree``: the same calls with torch tensors for
  device memory and torch's current stream.

The shared library must have been built (``python -m
paper_2402_00665_amd.build_lib`` or ``__graft_entry__.build()``); there is
no fallback of any kind.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbvh.so")

LBVH_OK, LBVH_EINVAL, LBVH_ENOSPACE, LBVH_EHIP, LBVH_EDEVICE, LBVH_ELIMIT = 0, -1, -2, -3, -4, -5
LBVH_NOALLOC_MAX_PRIMS = 1 << 20
LBVH_NOALLOC_SCRATCH_BYTES = 25 << 20
LBVH_POINTS, LBVH_BOXES = 0, 1
SPHERES, QBOXES, RAYS = 0, 1, 2
QUERY_WIDTH = {SPHERES: 4, QBOXES: 6, RAYS: 8}
LBVH_MAX_PRIMS = (1 << 30) - 1
NODE_BYTES = 32


class LbvhError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = f"{what}: {lbvh_strerror(status)} ({status})"
        if status == LBVH_EHIP:
            msg += f": {lbvh_last_hip_error()}"
        super().__init__(msg)
        self.status = status


class lbvh_tree(C.Structure):
    _fields_ = [("n", C.c_int64), ("code_bits", C.c_int32), ("kind", C.c_int32),
                ("nodes", C.c_void_p), ("codes", C.c_void_p), ("leaf_perm", C.c_void_p)]


class lbvh_batch(C.Structure):
    _fields_ = [("num_scenes", C.c_int32), ("code_bits", C.c_int32), ("kind", C.c_int32),
                ("reserved", C.c_int32), ("total_n", C.c_int64), ("max_scene", C.c_int64),
                ("seg_off", C.c_void_p), ("nodes", C.c_void_p), ("codes", C.c_void_p),
                ("leaf_perm", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2402_00665_amd.build_lib`")
        # torch ships its own HIP runtime under the same soname
        # (libamdhip64.so.7); importing torch first makes liblbvh bind to
        # that runtime, so device pointers and streams from torch belong to
        # the runtime the library launches on (one runtime per process).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        T = C.POINTER(lbvh_tree)
        Bt = C.POINTER(lbvh_batch)
        sig = {
            "lbvh_build_batched_workspace_bytes": (i64, [i64, i32, i64, i32, i32]),
            "lbvh_build_batched": (C.c_int, [i32, P, Bt, P, i64, P]),
            "lbvh_build_batched_check": (C.c_int, [P, Bt, P]),
            "lbvh_build_batched_status_async": (C.c_int, [P, Bt, P, P]),
            "lbvh_query_batched_workspace_bytes": (i64, [i64]),
            "lbvh_query_check": (C.c_int, [P, i64, P]),
            "lbvh_query_batched_check": (C.c_int, [P, i64, P]),
            "lbvh_query_batched_spheres_count": (C.c_int, [Bt, P, P, i64, P, P, i64, P]),
            "lbvh_query_batched_boxes_count": (C.c_int, [Bt, P, P, i64, P, P, i64, P]),
            "lbvh_query_batched_spheres_fill": (C.c_int, [Bt, P, P, i64, P, P, P, i64, P]),
            "lbvh_query_batched_boxes_fill": (C.c_int, [Bt, P, P, i64, P, P, P, i64, P]),
            "lbvh_build_workspace_bytes": (i64, [i64, i32, i32]),
            "lbvh_build": (C.c_int, [i32, P, i64, i32, T, P, i64, P]),
            "lbvh_build_points": (C.c_int, [P, i64, i32, T, P, i64, P]),
            "lbvh_build_boxes": (C.c_int, [P, i64, i32, T, P, i64, P]),
            "lbvh_build_check": (C.c_int, [P, i64, i32, i32, P]),
            "lbvh_build_noalloc": (C.c_int, [i32, P, i64, i32, T, P, P]),
            "lbvh_query_workspace_bytes": (i64, [i64]),
            "lbvh_query_spheres_count": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_boxes_count": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_spheres_fill": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_boxes_fill": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_rays_count": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_rays_fill": (C.c_int, [T, P, i64, P, P, i64, P]),
            "lbvh_query_rays_first": (C.c_int, [T, P, i64, P, P, P, i64, P]),
            "lbvh_strerror": (C.c_char_p, [C.c_int]),
            "lbvh_last_hip_error": (C.c_char_p, []),
            "lbvh_tune": (i64, [C.c_char_p, i64]),
            "lbvh_profile_enable": (C.c_int, [i32]),
            "lbvh_profile_reset": (C.c_int, []),
            "lbvh_profile_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(i64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


# --------------------------------------------------------- C-ABI names

def lbvh_strerror(status: int) -> str:
    return lib().lbvh_strerror(status).decode()


def lbvh_last_hip_error() -> str:
    return lib().lbvh_last_hip_error().decode()


def lbvh_build_workspace_bytes(n: int, code_bits: int, kind: int) -> int:
    return lib().lbvh_build_workspace_bytes(n, code_bits, kind)


def lbvh_build(kind, prims_ptr, n, code_bits, tree: lbvh_tree, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_build(kind, prims_ptr, n, code_bits, C.byref(tree), ws_ptr, ws_bytes, stream)


def lbvh_build_points(xyz_ptr, n, code_bits, tree: lbvh_tree, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_build_points(xyz_ptr, n, code_bits, C.byref(tree), ws_ptr, ws_bytes, stream)


def lbvh_build_boxes(lohi_ptr, n, code_bits, tree: lbvh_tree, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_build_boxes(lohi_ptr, n, code_bits, C.byref(tree), ws_ptr, ws_bytes, stream)


def lbvh_build_noalloc(kind, prims_ptr, n, code_bits, tree: lbvh_tree, err_ptr, stream) -> int:
    return lib().lbvh_build_noalloc(kind, prims_ptr, n, code_bits, C.byref(tree), err_ptr, stream)


def lbvh_build_check(ws_ptr, n, code_bits, kind, stream) -> int:
    return lib().lbvh_build_check(ws_ptr, n, code_bits, kind, stream)


def lbvh_query_workspace_bytes(m: int) -> int:
    return lib().lbvh_query_workspace_bytes(m)


def lbvh_query_spheres_count(tree, q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_spheres_count(C.byref(tree), q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_boxes_count(tree, q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_boxes_count(C.byref(tree), q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_spheres_fill(tree, q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_spheres_fill(C.byref(tree), q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_boxes_fill(tree, q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_boxes_fill(C.byref(tree), q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_rays_count(tree, q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_rays_count(C.byref(tree), q_ptr, m, offsets_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_rays_fill(tree, q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_rays_fill(C.byref(tree), q_ptr, m, idx_ptr, ws_ptr, ws_bytes, stream)


def lbvh_query_rays_first(tree, q_ptr, m, hit_ptr, t_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_rays_first(C.byref(tree), q_ptr, m, hit_ptr, t_ptr, ws_ptr, ws_bytes,
                                       stream)


def lbvh_query_check(ws_ptr, m, stream) -> int:
    return lib().lbvh_query_check(ws_ptr, m, stream)


def lbvh_query_batched_check(ws_ptr, m, stream) -> int:
    return lib().lbvh_query_batched_check(ws_ptr, m, stream)


def lbvh_tune(name: str, value: int = -1) -> int:
    return lib().lbvh_tune(name.encode(), value)


def lbvh_build_batched_workspace_bytes(total_n, num_scenes, max_scene, code_bits, kind) -> int:
    return lib().lbvh_build_batched_workspace_bytes(total_n, num_scenes, max_scene, code_bits, kind)


def lbvh_build_batched(kind, prims_ptr, batch: lbvh_batch, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_build_batched(kind, prims_ptr, C.byref(batch), ws_ptr, ws_bytes, stream)


def lbvh_build_batched_check(ws_ptr, batch: lbvh_batch, stream) -> int:
    return lib().lbvh_build_batched_check(ws_ptr, C.byref(batch), stream)


def lbvh_build_batched_status_async(ws_ptr, batch: lbvh_batch, flag_ptr, stream) -> int:
    return lib().lbvh_build_batched_status_async(ws_ptr, C.byref(batch), flag_ptr, stream)


def lbvh_query_batched_workspace_bytes(m) -> int:
    return lib().lbvh_query_batched_workspace_bytes(m)


def lbvh_query_batched_spheres_count(batch, q_ptr, qseg_ptr, m, off_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_batched_spheres_count(C.byref(batch), q_ptr, qseg_ptr, m, off_ptr, ws_ptr,
                                                 ws_bytes, stream)


def lbvh_query_batched_boxes_count(batch, q_ptr, qseg_ptr, m, off_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib().lbvh_query_batched_boxes_count(C.byref(batch), q_ptr, qseg_ptr, m, off_ptr, ws_ptr,
                                               ws_bytes, stream)


def lbvh_query_batched_spheres_fill(batch, q_ptr, qseg_ptr, m, off_ptr, idx_ptr, ws_ptr, ws_bytes,
                                    stream) -> int:
    return lib().lbvh_query_batched_spheres_fill(C.byref(batch), q_ptr, qseg_ptr, m, off_ptr, idx_ptr,
                                                ws_ptr, ws_bytes, stream)


def lbvh_query_batched_boxes_fill(batch, q_ptr, qseg_ptr, m, off_ptr, idx_ptr, ws_ptr, ws_bytes,
                                  stream) -> int:
    return lib().lbvh_query_batched_boxes_fill(C.byref(batch), q_ptr, qseg_ptr, m, off_ptr, idx_ptr,
                                              ws_ptr, ws_bytes, stream)


def lbvh_profile_enable(on: bool) -> int:
    return lib().lbvh_profile_enable(1 if on else 0)


def lbvh_profile_reset() -> int:
    return lib().lbvh_profile_reset()


def lbvh_profile_read(kernel: str):
    ms, cnt = C.c_double(0.0), C.c_int64(0)
    rc = lib().lbvh_profile_read(kernel.encode(), C.byref(ms), C.byref(cnt))
    if rc != LBVH_OK:
        raise LbvhError(rc, f"lbvh_profile_read({kernel})")
    return ms.value, cnt.value


# ------------------------------------------------------- torch layer

def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != LBVH_OK:
        raise LbvhError(rc, what)


def _dev_f32(t, width, what):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{what} must be a float32 CUDA tensor")
    if t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous [n, {width}] tensor")
    return t


@dataclass
class Tree:
    """A built tree: ``nodes`` is int32 [2n-1, 8] (lo.xyz, left, hi.xyz,
    rope; the float fields are stored by bit pattern), ``codes`` the sorted
    Morton codes (int32 storage for 30-bit codes, int64 for 63-bit),
    ``leaf_perm`` int32 [n] (leaf k -> input index)."""
    n: int
    code_bits: int
    kind: int
    nodes: object
    codes: object
    leaf_perm: object
    desc: lbvh_tree

    @property
    def lo(self):
        return self.nodes[:, 0:3].view(_torch().float32)

    @property
    def hi(self):
        return self.nodes[:, 4:7].view(_torch().float32)

    @property
    def left(self):
        """Left-child ids of the internal nodes, [n-1]."""
        return self.nodes[: max(self.n - 1, 0), 3]

    @property
    def rope(self):
        return self.nodes[:, 7]

    @property
    def perm(self):
        """Leaf k -> input index of its primitive, [n] (the leaves' `left`
        fields; ``leaf_perm`` holds the same values contiguously)."""
        return self.nodes[max(self.n - 1, 0):, 3]


class Workspace:
    """Grow-only device scratch buffer (a torch uint8 tensor)."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device or "cuda")
        return self.buf


def alloc_tree(n: int, code_bits: int, device="cuda") -> Tree:
    torch = _torch()
    nodes = torch.empty((max(2 * n - 1, 0), 8), dtype=torch.int32, device=device)
    codes = torch.empty(max(n, 1), dtype=torch.int32 if code_bits == 30 else torch.int64, device=device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    desc = lbvh_tree(n, code_bits, 0, nodes.data_ptr() if n > 0 else None, codes.data_ptr(),
                     perm.data_ptr())
    return Tree(n, code_bits, 0, nodes, codes, perm, desc)


def build(prims, code_bits: int, kind: int | None = None, workspace: Workspace | None = None,
          tree: Tree | None = None, stream=None) -> Tree:
    """Build the rope-LBVH of ``prims`` (float32 CUDA [n,3] points or [n,6]
    boxes) on the current stream; asynchronous."""
    if kind is None:
        kind = LBVH_POINTS if prims.shape[1] == 3 else LBVH_BOXES
    prims = _dev_f32(prims, 3 if kind == LBVH_POINTS else 6, "prims")
    n = int(prims.shape[0])
    if tree is None or tree.n != n or tree.code_bits != code_bits:
        tree = alloc_tree(n, code_bits, prims.device)
    ws_bytes = lbvh_build_workspace_bytes(n, code_bits, kind)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_build_workspace_bytes")
    ws = (workspace or Workspace(prims.device)).get(ws_bytes)
    rc = lbvh_build(kind, prims.data_ptr() if n else None, n, code_bits, tree.desc,
                    ws.data_ptr(), ws.numel(), _stream(stream))
    _check(rc, "lbvh_build")
    tree.kind = kind
    tree.last_workspace = ws
    return tree


def build_noalloc(prims, code_bits: int, kind: int | None = None, tree: Tree | None = None,
                  error=None, stream=None) -> Tree:
    """``build`` through lbvh_build_noalloc: no workspace, the library's
    fixed per-GPU scratch (n <= LBVH_NOALLOC_MAX_PRIMS).  ``error``: an
    optional int32 CUDA tensor of one element that receives the build's
    error word.  Pass a preallocated ``tree`` for a call that allocates
    nothing at all."""
    if kind is None:
        kind = LBVH_POINTS if prims.shape[1] == 3 else LBVH_BOXES
    prims = _dev_f32(prims, 3 if kind == LBVH_POINTS else 6, "prims")
    n = int(prims.shape[0])
    if tree is None or tree.n != n or tree.code_bits != code_bits:
        tree = alloc_tree(n, code_bits, prims.device)
    rc = lbvh_build_noalloc(kind, prims.data_ptr() if n else None, n, code_bits, tree.desc,
                            error.data_ptr() if error is not None else None, _stream(stream))
    _check(rc, "lbvh_build_noalloc")
    tree.kind = kind
    tree.last_workspace = None
    return tree


def check_build(tree: Tree, stream=None):
    """Synchronise and raise if the last build on this tree flagged an error."""
    ws = getattr(tree, "last_workspace", None)
    if ws is None or tree.n == 0:
        return
    _check(lbvh_build_check(ws.data_ptr(), tree.n, tree.code_bits, tree.kind, _stream(stream)),
           "lbvh_build_check")


def query_count(tree: Tree, queries, qkind: int, workspace: Workspace, offsets=None, stream=None):
    """First call: CSR offsets (int64 [m+1]) on the device; the workspace
    keeps what the fill call needs."""
    torch = _torch()
    q = _dev_f32(queries, QUERY_WIDTH[qkind], "queries")
    m = int(q.shape[0])
    if offsets is None:
        offsets = torch.empty(m + 1, dtype=torch.int64, device=q.device)
    ws_bytes = lbvh_query_workspace_bytes(m)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_query_workspace_bytes")
    ws = workspace.get(ws_bytes)
    f = {SPHERES: lbvh_query_spheres_count, QBOXES: lbvh_query_boxes_count,
         RAYS: lbvh_query_rays_count}[qkind]
    _check(f(tree.desc, q.data_ptr() if m else None, m, offsets.data_ptr(), ws.data_ptr(),
             ws.numel(), _stream(stream)), "query count")
    return offsets


def check_query(workspace: Workspace, m: int, batched: bool = False, stream=None):
    """Synchronise and raise if the last count call on this workspace (m
    queries) flagged an error."""
    f = lbvh_query_batched_check if batched else lbvh_query_check
    _check(f(workspace.buf.data_ptr(), m, _stream(stream)), "lbvh_query_check")


def query_fill(tree: Tree, queries, qkind: int, indices, workspace: Workspace, stream=None):
    """Second call, with the count call's workspace."""
    q = _dev_f32(queries, QUERY_WIDTH[qkind], "queries")
    m = int(q.shape[0])
    ws = workspace.buf
    f = {SPHERES: lbvh_query_spheres_fill, QBOXES: lbvh_query_boxes_fill,
         RAYS: lbvh_query_rays_fill}[qkind]
    _check(f(tree.desc, q.data_ptr() if m else None, m, indices.data_ptr(), ws.data_ptr(),
             ws.numel(), _stream(stream)), "query fill")
    return indices


def query(tree: Tree, queries, qkind: int, workspace: Workspace | None = None, stream=None):
    """Count, read the total (one 8-byte device-to-host copy), fill.
    Returns (offsets int64 [m+1], indices int32 [total]) on the device."""
    torch = _torch()
    workspace = workspace or Workspace(queries.device)
    offsets = query_count(tree, queries, qkind, workspace, stream=stream)
    total = int(offsets[-1].item())
    # at least one element so the device pointer is never null
    buf = torch.empty(max(total, 1), dtype=torch.int32, device=queries.device)
    query_fill(tree, queries, qkind, buf, workspace, stream=stream)
    return offsets, buf[:total]


def query_first(tree: Tree, rays, workspace: Workspace | None = None, hit=None, t=None,
                stream=None):
    """First hit of each ray (float32 CUDA [m, 8] = o.xyz, tmin, d.xyz,
    tmax): (hit int32 [m], input index or -1; t float32 [m], entry
    parameter or +inf) on the device; asynchronous."""
    torch = _torch()
    q = _dev_f32(rays, 8, "rays")
    m = int(q.shape[0])
    if hit is None:
        hit = torch.empty(max(m, 1), dtype=torch.int32, device=q.device)[:m]
    if t is None:
        t = torch.empty(max(m, 1), dtype=torch.float32, device=q.device)[:m]
    workspace = workspace or Workspace(q.device)
    ws_bytes = lbvh_query_workspace_bytes(m)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_query_workspace_bytes")
    ws = workspace.get(ws_bytes)
    _check(lbvh_query_rays_first(tree.desc, q.data_ptr() if m else None, m,
                                 hit.data_ptr() if m else None, t.data_ptr() if m else None,
                                 ws.data_ptr(), ws.numel(), _stream(stream)), "lbvh_query_rays_first")
    return hit, t


# ------------------------------------------------------------- batched

def _batched_width(qkind: int) -> int:
    if qkind not in (SPHERES, QBOXES):
        raise ValueError("batched queries are spheres or boxes")
    return QUERY_WIDTH[qkind]


@dataclass
class Batch:
    """Trees of many scenes built together.  Scene s's 2n_s-1 node records
    start at record 2*seg_off[s] of ``nodes`` (int32 [2N, 8]); ``codes`` and
    ``leaf_perm`` hold its sorted codes and local primitive ids at
    [seg_off[s], seg_off[s+1])."""
    num_scenes: int
    total_n: int
    code_bits: int
    kind: int
    max_scene: int
    seg_off: object
    nodes: object
    codes: object
    leaf_perm: object
    desc: lbvh_batch
    workspace: object = None

    def scene_nodes(self, s: int, seg_off_host):
        a, b = int(seg_off_host[s]), int(seg_off_host[s + 1])
        return self.nodes[2 * a: 2 * a + max(2 * (b - a) - 1, 0)]


def alloc_batch(seg_off, code_bits: int, max_scene: int, device="cuda", total_n: int | None = None) -> Batch:
    """seg_off: int64 CUDA tensor [S+1]; pass ``total_n`` (= seg_off[S]) when
    it is known on the host, to avoid reading it back from the device."""
    torch = _torch()
    S = int(seg_off.numel()) - 1
    if total_n is not None:
        N = int(total_n)
    else:
        N = int(seg_off[-1].item()) if S >= 0 else 0
    nodes = torch.empty((max(2 * N, 1), 8), dtype=torch.int32, device=device)
    codes = torch.empty(max(N, 1), dtype=torch.int32 if code_bits == 30 else torch.int64, device=device)
    perm = torch.empty(max(N, 1), dtype=torch.int32, device=device)
    desc = lbvh_batch(S, code_bits, 0, 0, N, max_scene, seg_off.data_ptr(), nodes.data_ptr(),
                      codes.data_ptr(), perm.data_ptr())
    return Batch(S, N, code_bits, 0, max_scene, seg_off, nodes, codes, perm, desc)


def build_batched(prims, seg_off, code_bits: int, max_scene: int, kind: int | None = None,
                  workspace: Workspace | None = None, batch: Batch | None = None, stream=None) -> Batch:
    """Build the trees of all scenes; prims float32 CUDA [N,3] or [N,6],
    seg_off int64 CUDA [S+1]; max_scene >= every scene size (host value)."""
    torch = _torch()
    if kind is None:
        kind = LBVH_POINTS if prims.shape[1] == 3 else LBVH_BOXES
    prims = _dev_f32(prims, 3 if kind == LBVH_POINTS else 6, "prims")
    if not (seg_off.is_cuda and seg_off.dtype == torch.int64 and seg_off.is_contiguous()):
        raise TypeError("seg_off must be a contiguous int64 CUDA tensor")
    if batch is None:
        batch = alloc_batch(seg_off, code_bits, max_scene, prims.device)
    ws_bytes = lbvh_build_batched_workspace_bytes(batch.total_n, batch.num_scenes, max_scene,
                                                  code_bits, kind)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_build_batched_workspace_bytes")
    ws = (workspace or Workspace(prims.device)).get(ws_bytes)
    _check(lbvh_build_batched(kind, prims.data_ptr() if batch.total_n else None, batch.desc,
                              ws.data_ptr(), ws.numel(), _stream(stream)), "lbvh_build_batched")
    batch.kind = kind
    batch.workspace = ws
    return batch


def check_batched(batch: Batch, stream=None):
    if batch.workspace is None:
        return
    _check(lbvh_build_batched_check(batch.workspace.data_ptr(), batch.desc, _stream(stream)),
           "lbvh_build_batched_check")


def query_batched_count(batch: Batch, queries, qseg_off, qkind: int, workspace: Workspace,
                        offsets=None, stream=None):
    """First batched call, asynchronous: CSR offsets int64 [m+1]."""
    torch = _torch()
    q = _dev_f32(queries, _batched_width(qkind), "queries")
    m = int(q.shape[0])
    if offsets is None:
        offsets = torch.empty(m + 1, dtype=torch.int64, device=q.device)
    ws_bytes = lbvh_query_batched_workspace_bytes(m)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_query_batched_workspace_bytes")
    ws = workspace.get(ws_bytes)
    cnt = lbvh_query_batched_spheres_count if qkind == SPHERES else lbvh_query_batched_boxes_count
    _check(cnt(batch.desc, q.data_ptr() if m else None, qseg_off.data_ptr(), m, offsets.data_ptr(),
               ws.data_ptr(), ws.numel(), _stream(stream)), "batched query count")
    return offsets


def query_batched_fill(batch: Batch, queries, qseg_off, qkind: int, offsets, indices,
                       workspace: Workspace, stream=None):
    """Second batched call, asynchronous, with the count call's workspace:
    indices int32 [offsets[m]] (the tensor must hold at least one element)."""
    q = _dev_f32(queries, _batched_width(qkind), "queries")
    m = int(q.shape[0])
    ws = workspace.buf
    fill = lbvh_query_batched_spheres_fill if qkind == SPHERES else lbvh_query_batched_boxes_fill
    _check(fill(batch.desc, q.data_ptr() if m else None, qseg_off.data_ptr(), m, offsets.data_ptr(),
                indices.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)), "batched query fill")
    return indices


def query_batched(batch: Batch, queries, qseg_off, qkind: int, workspace: Workspace | None = None,
                  stream=None):
    """Count, read the total, fill.  Returns (offsets int64 [m+1], indices
    int32 [total]) with scene-local primitive ids."""
    torch = _torch()
    q = _dev_f32(queries, _batched_width(qkind), "queries")
    m = int(q.shape[0])
    offsets = torch.empty(m + 1, dtype=torch.int64, device=q.device)
    ws_bytes = lbvh_query_batched_workspace_bytes(m)
    _check(ws_bytes if ws_bytes < 0 else 0, "lbvh_query_batched_workspace_bytes")
    ws = (workspace or Workspace(q.device)).get(ws_bytes)
    cnt = lbvh_query_batched_spheres_count if qkind == SPHERES else lbvh_query_batched_boxes_count
    _check(cnt(batch.desc, q.data_ptr() if m else None, qseg_off.data_ptr(), m, offsets.data_ptr(),
               ws.data_ptr(), ws.numel(), _stream(stream)), "batched query count")
    total = int(offsets[-1].item())
    buf = torch.empty(max(total, 1), dtype=torch.int32, device=q.device)
    fill = lbvh_query_batched_spheres_fill if qkind == SPHERES else lbvh_query_batched_boxes_fill
    _check(fill(batch.desc, q.data_ptr() if m else None, qseg_off.data_ptr(), m, offsets.data_ptr(),
                buf.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)), "batched query fill")
    return offsets, buf[:total]
