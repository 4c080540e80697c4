"""Self-written autotuner for the library's launch-shape knobs.

A knob (see ``lbvh_tune`` in include/lbvh.h) picks a digit width, a tile
shape or a query piece size; results never depend on it, only speed does.
``tune`` (radix digit width and tile shape of a build) and ``tune_query``
(the query schedule) time every candidate on the caller's own workload with
HIP events,
check once per candidate that its output is bit-identical to the default's,
keep the fastest and record it in a JSON cache keyed by GPU arch, knob and
workload shape (code bits / query kind, size buckets floor(log2 n) and
floor(log2 m)).  ``apply`` and ``apply_query`` set the cached winners.

Cache path: $LBVH_TUNING_CACHE, else ~/.cache/paper_2402_00665_amd/tuning.json.
"""

from __future__ import annotations

import json
import math
import os

from . import (LBVH_POINTS, Workspace, alloc_tree, build, build_batched, check_batched,
               check_build, lbvh_profile_enable, lbvh_profile_read, lbvh_profile_reset,
               lbvh_tune, query_count, query_fill)

KNOB_CANDIDATES = {
    "sort_variant32": list(range(9)),
    "sort_variant64": list(range(9)),
    "batch_sort_variant": list(range(4)),
    "batch_sort_mode": [0, 1],
    "radix_bits32": [8, 10],
    "radix_mode": [0, 1],
    "radix_bits64": [8, 9, 11],
}
# (query_split1, query_split2, query_leaf_mode, query_order): each split
# schedule with the queries as given and in Morton order
# Coarse blocks suit thin queries (rays, segments), whose hits fall in few
# Morton ranges but whose finer pieces would exceed the split levels'
# capacity; (24, 24): blocks larger than the tree, each query one plain
# Alg. 1 walk by one lane.
_SPLITS = [(12, 7, 0), (13, 8, 0), (12, 8, 0), (12, 6, 0), (13, 7, 0), (11, 6, 0),
           (12, 7, 1), (11, 6, 1), (13, 7, 1), (11, 5, 1), (14, 10, 1), (16, 10, 1),
           (14, 9, 1), (15, 10, 0), (24, 24, 0)]
QUERY_CANDIDATES = [s + (o,) for o in (0, 1) for s in _SPLITS]
_QUERY_KNOBS = ("query_split1", "query_split2", "query_leaf_mode", "query_order")


def cache_path() -> str:
    return os.environ.get("LBVH_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2402_00665_amd",
                                       "tuning.json"))


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(knob: str, code_bits: int, kind: int, n: int) -> str:
    return f"{_arch()}/{knob}/{code_bits}/{kind}/{int(math.log2(max(n, 1)))}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _sort_ms(prep: str):
    """ms of the codes kernel and all radix passes since the last reset."""
    t0, _ = lbvh_profile_read(prep)
    t1, _ = lbvh_profile_read("sort_pass")
    return t0 + t1


def _time_single(prims, code_bits, kind, ws, tree, reps):
    import torch
    for _ in range(2):
        build(prims, code_bits, kind=kind, workspace=ws, tree=tree)
    torch.cuda.synchronize()
    lbvh_profile_reset()
    lbvh_profile_enable(True)
    for _ in range(reps):
        build(prims, code_bits, kind=kind, workspace=ws, tree=tree)
    torch.cuda.synchronize()
    lbvh_profile_enable(False)
    ms = _sort_ms("morton")
    check_build(tree)
    return ms / reps


def _time_batched(prims, seg_off, code_bits, kind, max_scene, ws, batch, reps):
    import torch
    for _ in range(2):
        build_batched(prims, seg_off, code_bits, max_scene, kind=kind, workspace=ws, batch=batch)
    torch.cuda.synchronize()
    lbvh_profile_reset()
    lbvh_profile_enable(True)
    for _ in range(reps):
        build_batched(prims, seg_off, code_bits, max_scene, kind=kind, workspace=ws, batch=batch)
    torch.cuda.synchronize()
    lbvh_profile_enable(False)
    ms = _sort_ms("batch_prep")
    check_batched(batch)
    return ms / reps


def sort_knobs(code_bits: int, batched: bool):
    """(digit-width knob, tile-shape knob) of a build."""
    width = f"radix_bits{32 if code_bits == 30 else 64}"
    shape = "batch_sort_variant" if batched else f"sort_variant{32 if code_bits == 30 else 64}"
    return width, shape


def tune(prims, code_bits: int, kind: int | None = None, seg_off=None, max_scene: int | None = None,
         reps: int = 5, save: bool = True, verbose: bool = False) -> dict:
    """Tune the radix digit width and tile shape for this workload (a single
    tree, or a batch when ``seg_off`` is given), and for a single tree the
    pass form ("radix_mode"): each candidate is timed as the codes kernel
    plus all radix passes of a build.  Returns {"knobs": {knob: value},
    "times_ms": {"bits/shape[/mode]": ms per build}}; every candidate is
    checked to give the same tree, bit for bit, as the first (current) one."""
    import torch
    if kind is None:
        kind = LBVH_POINTS if prims.shape[1] == 3 else 1
    batched = seg_off is not None
    wk, sk = sort_knobs(code_bits, batched)
    # batched builds also choose between the segmented passes (mode 0, each
    # tile shape) and one block per scene (mode 1, each block shape): a
    # mode-1 candidate's shape slot holds -1 - shape
    mode0 = lbvh_tune("batch_sort_mode") if batched else 0
    rmode0 = 0 if batched else lbvh_tune("radix_mode")
    default = (lbvh_tune(wk), lbvh_tune(sk) if mode0 == 0 else -1 - lbvh_tune(sk), rmode0)
    if batched:
        cands = [(b, v, 0) for b in KNOB_CANDIDATES[wk] for v in KNOB_CANDIDATES[sk]]
        cands += [(b, -1 - v, 0) for b in KNOB_CANDIDATES[wk] for v in KNOB_CANDIDATES[sk]]
    else:
        cands = [(b, v, m) for m in KNOB_CANDIDATES["radix_mode"] for b in KNOB_CANDIDATES[wk]
                 for v in KNOB_CANDIDATES[sk]]
    order = [default] + [c for c in cands if c != default]
    shape0 = lbvh_tune(sk)
    ws = Workspace(prims.device)
    n = int(prims.shape[0])
    if batched:
        from . import alloc_batch
        obj = alloc_batch(seg_off, code_bits, max_scene, prims.device)
    else:
        obj = alloc_tree(n, code_bits, prims.device)
    times, ref = {}, None
    try:
        for b, v, m in order:
            lbvh_tune(wk, b)
            if batched:
                lbvh_tune("batch_sort_mode", 1 if v < 0 else 0)
            else:
                lbvh_tune("radix_mode", m)
            lbvh_tune(sk, v if v >= 0 else -1 - v)
            t = (_time_batched(prims, seg_off, code_bits, kind, max_scene, ws, obj, reps) if batched
                 else _time_single(prims, code_bits, kind, ws, obj, reps))
            out = torch.cat([obj.nodes.flatten(), obj.leaf_perm]).clone()
            if ref is None:
                ref = out
            elif not torch.equal(out, ref):
                raise RuntimeError(f"{wk}={b}, {sk}={v} changed the tree; refusing to tune with it")
            times[f"{b}/{v}" if batched else f"{b}/{v}/{m}"] = t
            if verbose:
                print(f"[autotune] {wk}={b} {sk}={v}" + ("" if batched else f" radix_mode={m}")
                      + f": {t * 1e3:.1f} us per build", flush=True)
    finally:
        lbvh_tune(wk, default[0])
        lbvh_tune(sk, shape0)
        if batched:
            lbvh_tune("batch_sort_mode", mode0)
        else:
            lbvh_tune("radix_mode", rmode0)
    best = min(times, key=times.get)
    got = [int(x) for x in best.split("/")]
    b_best, v_best = got[0], got[1]
    if batched:
        knobs = {wk: b_best, "batch_sort_mode": 1 if v_best < 0 else 0,
                 sk: v_best if v_best >= 0 else -1 - v_best}
    else:
        knobs = {wk: b_best, sk: v_best, "radix_mode": got[2]}
    if save:
        cache = _load()
        cache[_key(sk, code_bits, kind, n)] = {"knobs": knobs, "times_ms": times}
        _save(cache)
    return {"knobs": knobs, "times_ms": times}


def apply(n: int, code_bits: int, kind: int, batched: bool = False) -> dict:
    """Set the cached best digit width and tile shape for this shape, if
    any; returns {knob: value} for what was set."""
    _, sk = sort_knobs(code_bits, batched)
    hit = _load().get(_key(sk, code_bits, kind, n))
    if hit is None or "knobs" not in hit:
        return {}
    for k, v in hit["knobs"].items():
        lbvh_tune(k, int(v))
    return {k: int(v) for k, v in hit["knobs"].items()}


def _query_key(qkind: int, n: int, m: int) -> str:
    return (f"{_arch()}/query_schedule/{qkind}/{int(math.log2(max(n, 1)))}/"
            f"{int(math.log2(max(m, 1)))}")


def tune_query(tree, queries, qkind: int, candidates=None, reps: int = 5, save: bool = True,
               verbose: bool = False) -> dict:
    """Tune the query schedule for this tree and query set: times the count
    call plus the fill call per (split1, split2, leaf mode, query order)
    candidate, checks each gives the default's offsets and indices bit for
    bit, keeps the fastest.  Returns {"value": (s1, s2, mode, order),
    "times_ms": {...}}."""
    import torch
    cands = [tuple(c) for c in (candidates or QUERY_CANDIDATES)]
    default = tuple(lbvh_tune(k) for k in _QUERY_KNOBS)
    order = [default] + [c for c in cands if c != default]
    ws = Workspace(queries.device)
    m = int(queries.shape[0])
    times, ref = {}, None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    try:
        for cand in order:
            for k, v in zip(_QUERY_KNOBS, cand):
                lbvh_tune(k, v)
            best = None
            for r in range(reps + 1):
                e0.record()
                off = query_count(tree, queries, qkind, ws)
                total = int(off[-1].item())
                idx = torch.empty(max(total, 1), dtype=torch.int32, device=queries.device)
                query_fill(tree, queries, qkind, idx, ws)
                e1.record()
                torch.cuda.synchronize()
                if r > 0:
                    ms = e0.elapsed_time(e1)
                    best = ms if best is None else min(best, ms)
            out = (off.clone(), idx[:total].clone())
            if ref is None:
                ref = out
            elif not (torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])):
                raise RuntimeError(f"query schedule {cand} changed the results; refusing to tune")
            times["/".join(map(str, cand))] = best
            if verbose:
                print(f"[autotune] query schedule {cand}: {best * 1e3:.1f} us", flush=True)
    finally:
        for k, v in zip(_QUERY_KNOBS, default):
            lbvh_tune(k, v)
    key = min(times, key=times.get)
    value = tuple(int(x) for x in key.split("/"))
    if save:
        cache = _load()
        cache[_query_key(qkind, tree.n, m)] = {"value": list(value), "times_ms": times}
        _save(cache)
    return {"value": value, "times_ms": times}


def apply_query(n: int, m: int, qkind: int) -> dict:
    """Set the cached best query schedule for this shape, if any."""
    hit = _load().get(_query_key(qkind, n, m))
    if hit is None:
        return {}
    vals = [int(x) for x in hit["value"]]
    for k, v in zip(_QUERY_KNOBS, vals):
        lbvh_tune(k, v)
    return dict(zip(_QUERY_KNOBS, vals))
