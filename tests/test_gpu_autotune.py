"""GPU test of the self-written autotuner: it times every tile shape on a
workload, checks each one gives the default's tree bit for bit, caches the
winner and re-applies it."""

import json

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_tune_single_and_batched(tmp_path, monkeypatch):
    import torch
    import paper_2402_00665_amd as lb
    from paper_2402_00665_amd import autotune
    monkeypatch.setenv("LBVH_TUNING_CACHE", str(tmp_path / "tuning.json"))
    rng = np.random.default_rng(30)
    p = torch.from_numpy(rng.random((1 << 18, 3), dtype=np.float32)).cuda()
    defaults = {k: lb.lbvh_tune(k) for k in autotune.KNOB_CANDIDATES}
    r = autotune.tune(p, 63, reps=3, verbose=True)
    say(f"single: {r}")
    assert set(r["knobs"]) == {"radix_bits64", "sort_variant64", "radix_mode"}
    assert set(r["times_ms"]) == {f"{b}/{v}/{m}" for b in (8, 9, 11) for v in range(9) for m in (0, 1)}
    assert {k: lb.lbvh_tune(k) for k in defaults} == defaults   # tuning restores the defaults
    sizes = np.array([3000, 70000, 1, 0, 40000], np.int64)
    seg = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=seg[1:])
    pb = torch.from_numpy(rng.random((int(seg[-1]), 3), dtype=np.float32)).cuda()
    rb = autotune.tune(pb, 30, seg_off=torch.from_numpy(seg).cuda(), max_scene=70000, reps=3)
    say(f"batched: {rb}")
    assert set(rb["knobs"]) == {"radix_bits32", "batch_sort_mode", "batch_sort_variant"}
    assert set(rb["times_ms"]) == {f"{b}/{v}" for b in (8, 10) for v in range(-4, 4)}
    cache = json.loads((tmp_path / "tuning.json").read_text())
    assert len(cache) == 2
    try:
        assert autotune.apply(1 << 18, 63, 0) == r["knobs"]
        assert lb.lbvh_tune("sort_variant64") == r["knobs"]["sort_variant64"]
        assert lb.lbvh_tune("radix_bits64") == r["knobs"]["radix_bits64"]
        assert lb.lbvh_tune("radix_mode") == r["knobs"]["radix_mode"]
        assert autotune.apply(int(seg[-1]), 30, 0, batched=True) == rb["knobs"]
        assert autotune.apply(1 << 10, 63, 0) == {}   # other size bucket: nothing cached
    finally:
        for k, v in defaults.items():
            lb.lbvh_tune(k, v)


def test_tune_query_schedule(tmp_path, monkeypatch):
    import torch
    import paper_2402_00665_amd as lb
    import workloads
    from paper_2402_00665_amd import autotune
    monkeypatch.setenv("LBVH_TUNING_CACHE", str(tmp_path / "tuning.json"))
    w = workloads.by_name("clustered_boxes", 1 / 16)
    tree = lb.build(torch.from_numpy(w.prims).cuda(), w.code_bits, kind=w.kind)
    q = torch.from_numpy(w.queries).cuda()
    knobs = ("query_split1", "query_split2", "query_leaf_mode", "query_order")
    before = tuple(lb.lbvh_tune(k) for k in knobs)
    r = autotune.tune_query(tree, q, w.qkind, reps=2, verbose=True)
    say(f"query schedule: {r}")
    assert r["value"] in [tuple(c) for c in autotune.QUERY_CANDIDATES] + [before]
    assert tuple(lb.lbvh_tune(k) for k in knobs) == before
    try:
        assert autotune.apply_query(tree.n, q.shape[0], w.qkind) == dict(zip(knobs, r["value"]))
    finally:
        for k, v in zip(knobs, before):
            lb.lbvh_tune(k, v)
