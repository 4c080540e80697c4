"""CPU checks of the C-ABI library: it loads, exports every function that
include/lbvh.h declares, sizes workspaces sensibly and rejects bad arguments
before touching the GPU.  No compute call is made here."""

import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2402_00665_amd as lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbvh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbvh_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["lbvh_build", "lbvh_build_points", "lbvh_build_boxes", "lbvh_build_workspace_bytes",
                 "lbvh_query_spheres_count", "lbvh_query_boxes_count", "lbvh_query_spheres_fill",
                 "lbvh_query_boxes_fill", "lbvh_query_workspace_bytes", "lbvh_strerror"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = lb.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lbvh_\w+)", out))
    assert set(declared_functions()) <= exported


def test_binding_mirrors_c_names():
    for name in declared_functions():
        assert callable(getattr(lb, name)), name


def test_node_record_layout():
    class Node(C.Structure):
        _fields_ = [("lo", C.c_float * 3), ("left", C.c_int32), ("hi", C.c_float * 3), ("rope", C.c_int32)]
    assert C.sizeof(Node) == lb.NODE_BYTES == 32
    assert C.sizeof(lb.lbvh_tree) == 40


def test_strerror():
    assert lb.lbvh_strerror(0) == "ok"
    assert "workspace" in lb.lbvh_strerror(lb.LBVH_ENOSPACE)
    assert lb.lbvh_strerror(-99) == "unknown status"


@pytest.mark.parametrize("bits,kb", [(30, 4), (63, 8)])
def test_workspace_bytes(bits, kb):
    for kind in (0, 1):
        w0 = lb.lbvh_build_workspace_bytes(0, bits, kind)
        w = lb.lbvh_build_workspace_bytes(1 << 20, bits, kind)
        assert 0 < w0 < w
        # keys ping-pong + two value buffers + Alg. 4 flags dominate
        assert w >= (1 << 20) * (kb + 12)
        assert w % 256 == 0
    assert lb.lbvh_build_workspace_bytes(-1, bits, 0) == lb.LBVH_EINVAL
    assert lb.lbvh_build_workspace_bytes(1 << 30, bits, 0) == lb.LBVH_EINVAL
    assert lb.lbvh_query_workspace_bytes(1000) >= 4000
    assert lb.lbvh_query_workspace_bytes(-1) == lb.LBVH_EINVAL


def test_invalid_arguments_are_rejected_without_side_effects():
    t = lb.lbvh_tree(0, 0, 0, None, None, None)
    assert lb.lbvh_build(0, None, 10, 31, t, None, 0, None) == lb.LBVH_EINVAL   # code_bits
    assert lb.lbvh_build(2, None, 10, 30, t, None, 0, None) == lb.LBVH_EINVAL   # kind
    assert lb.lbvh_build(0, None, -1, 30, t, None, 0, None) == lb.LBVH_EINVAL   # n < 0
    assert lb.lbvh_build(0, None, 10, 30, t, None, 0, None) == lb.LBVH_EINVAL   # null pointers
    # misaligned pointers (never dereferenced: rejected up front)
    t2 = lb.lbvh_tree(0, 0, 0, 4096, 4096, 4096)
    assert lb.lbvh_build(0, 4100, 10, 30, t2, 4096, 1 << 30, None) == lb.LBVH_EINVAL
    assert lb.lbvh_build(0, 4096, 10, 30, t2, 4096 + 16, 1 << 30, None) == lb.LBVH_EINVAL
    # too small a workspace
    assert lb.lbvh_build(0, 4096, 10, 30, t2, 4096, 16, None) == lb.LBVH_ENOSPACE
    # empty build needs nothing and touches nothing
    t3 = lb.lbvh_tree(5, 0, 0, None, None, None)
    assert lb.lbvh_build(1, None, 0, 63, t3, None, 0, None) == lb.LBVH_OK
    assert (t3.n, t3.code_bits, t3.kind) == (0, 63, 1)
    # queries
    assert lb.lbvh_query_spheres_count(t3, None, -1, 4096, 4096, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_boxes_count(t3, None, 4, None, 4096, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_boxes_count(t3, 4096, 4, 4096, 4096, 8, None) == lb.LBVH_ENOSPACE
    assert lb.lbvh_query_spheres_fill(t3, 4100, 4, 4096, 4096, 1 << 30, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_spheres_fill(t3, 4096, 4, 4096, 4096, 8, None) == lb.LBVH_ENOSPACE


def test_profile_names():
    for name in ["bounds", "bounds_final", "morton", "sort_pass", "bottomup", "bottomup_up",
                 "query_split", "query_count", "query_fill", "scan", "query_order", "batch_prep"]:
        assert lb.lbvh_profile_read(name)[1] >= 0
    with pytest.raises(lb.LbvhError):
        lb.lbvh_profile_read("nope")


def test_tune_knobs():
    """Every knob reads back, takes a value in range and refuses one out of
    range (no GPU needed: knobs are host state)."""
    ranges = {"sort_variant32": 8, "sort_variant64": 8, "batch_sort_variant": 3, "morton_order": 1,
              "radix_mode": 1, "batch_sort_mode": 1,
              "query_split1": 24, "query_split2": 24, "query_leaf_mode": 1, "query_order": 1}
    for name, hi in ranges.items():
        old = lb.lbvh_tune(name)
        assert old >= 0
        assert lb.lbvh_tune(name, hi) == old
        assert lb.lbvh_tune(name) == hi
        assert lb.lbvh_tune(name, old) == hi
        assert lb.lbvh_tune(name, hi + 1) == lb.LBVH_EINVAL
    # digit widths: only the widths each code width allows
    for name, ok in (("radix_bits32", (8, 10)), ("radix_bits64", (8, 9, 11))):
        old = lb.lbvh_tune(name)
        assert old in ok
        for v in range(7, 13):
            rc = lb.lbvh_tune(name, v)
            if v in ok:
                assert rc in ok
            else:
                assert rc == lb.LBVH_EINVAL
        lb.lbvh_tune(name, old)
        assert lb.lbvh_tune(name) == old
    assert lb.lbvh_tune("no_such_knob", 0) == lb.LBVH_EINVAL


def test_product_path_does_not_import_the_oracle():
    import sys
    src_dir = os.path.join(ROOT, "paper_2402_00665_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lbvh_oracle" not in text, f


def test_one_hip_runtime_per_process():
    """The library binds to the HIP runtime torch loaded (same soname), so
    torch's pointers and streams are the library's own."""
    lb.lib()
    maps = open("/proc/self/maps").read()
    runtimes = {ln.split()[-1] for ln in maps.splitlines() if "libamdhip64" in ln}
    assert len(runtimes) == 1, runtimes


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with status 2 and
    says so (before touching any GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_ray_calls_reject_bad_arguments_up_front():
    """The ray entry points validate before enqueuing anything (no pointer
    here is ever dereferenced)."""
    t = lb.lbvh_tree(0, 30, 0, None, None, None)
    assert lb.lbvh_query_rays_first(t, None, -1, None, None, None, 0, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_rays_first(t, None, 0, None, None, None, 0, None) == lb.LBVH_OK   # m = 0
    assert lb.lbvh_query_rays_first(t, None, 10, 16, 16, 256, 0, None) == lb.LBVH_EINVAL  # no rays
    assert lb.lbvh_query_rays_first(t, 8, 10, 16, 16, 256, 1 << 20, None) == lb.LBVH_EINVAL  # align
    assert lb.lbvh_query_rays_first(t, 16, 10, None, 16, 256, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_rays_first(t, 16, 10, 16, 16, 256, 0, None) == lb.LBVH_ENOSPACE
    assert lb.lbvh_query_rays_first(t, 16, 10, 16, 16, 128, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_rays_count(t, None, -1, 16, 256, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_rays_count(t, 8, 10, 16, 256, 1 << 20, None) == lb.LBVH_EINVAL
    assert lb.lbvh_query_rays_fill(t, 16, 10, None, 256, 0, None) == lb.LBVH_ENOSPACE
