"""Benchmark of the rope-LBVH hot path on one MI355X.

One step = one full pass of the path over resident inputs: build (scene box,
Morton codes, radix sort, Alg. 4 bottom-up pass) followed by the stackless
range queries (count pass, offset scan, read of the total, fill pass).

Prints one JSON line:
  value        build throughput, Mprims/s (n / mean build time of a step)
  ms_per_step  mean wall time of a whole step (build + queries)
  queries      query throughput of the same steps
  roofline     the dominant kernel's algorithmic bytes per launch over its
               mean launch time (HIP events the library records on the
               launch stream), against the 8 TB/s HBM peak
  cpu_baseline the plain single-threaded C oracle on a bounded sample

Default workload: 2^24 clustered boxes with 30-bit codes and 2^20 box
queries of side 0.01 (the 2^24-primitive configuration).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# Algorithmic bytes per primitive of each build kernel (P = primitive bytes,
# K = code bytes, d = radix passes), counting each array element once per
# kernel that must touch it:
#   bounds    read P
#   morton    read P, write code K, write the Alg. 4 flag 4
#   sort pass read key K (+ value 4 after the first pass), write K + 4
#   bottomup  read code K, perm 4, primitive P, flag CAS 8, sibling box 24,
#             write leaf node 32 and internal node 32
def build_bytes_per_prim(P: int, K: int, d: int) -> dict:
    return {
        "bounds": P,
        "morton": P + K + 4,
        "sort_pass": ((2 * K + 4) + (d - 1) * (2 * K + 8)) / d,
        "bottomup": K + 4 + P + 8 + 24 + 32 + 32,
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered_boxes",
                    choices=["clustered_boxes", "large_points", "small_points"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--build-only", action="store_true",
                    help="time the build alone (no queries in the step)")
    ap.add_argument("--cpu-sample", type=float, default=0.5,
                    help="fraction of the workload the oracle baseline runs on")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this path has no multi-GPU form)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2402_00665_amd as lb
    import workloads

    torch.cuda.set_device(0)
    t0 = time.time()
    w = workloads.by_name(args.workload)
    log(f"[bench] workload {w.name}: n={w.n} m={w.m} bits={w.code_bits} "
        f"(generated in {time.time() - t0:.1f}s)")
    prims = torch.from_numpy(w.prims).cuda()
    queries = torch.from_numpy(w.queries).cuda()
    ws = lb.Workspace()
    qws = lb.Workspace()
    tree = lb.alloc_tree(w.n, w.code_bits)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        lb.build(prims, w.code_bits, kind=w.kind, workspace=ws, tree=tree)
        if ev:
            ev[1].record(stream)
        off, idx = (None, None) if args.build_only else lb.query(tree, queries, w.qkind, workspace=qws)
        if ev:
            ev[2].record(stream)
        return off, idx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lb.check_build(tree)
    log(f"[bench] warmup {args.warmup} done")

    lb.lbvh_profile_reset()
    lb.lbvh_profile_enable(True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    hits = 0
    for k in range(args.steps):
        off, idx = step(evs[k])
        hits = int(idx.numel()) if idx is not None else 0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lb.lbvh_profile_enable(False)
    log(f"[bench] timed {args.steps} steps in {wall:.3f}s")

    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    query_ms = [e[1].elapsed_time(e[2]) for e in evs]
    mean_build = float(np.mean(build_ms))
    mean_query = float(np.mean(query_ms))
    ms_per_step = wall * 1e3 / args.steps

    kernels = {}
    for name in ["bounds", "bounds_final", "morton", "sort_pass", "bottomup", "query_split",
                 "query_count", "scan", "query_fill"]:
        tot, cnt = lb.lbvh_profile_read(name)
        if cnt:
            kernels[name] = {"ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps,
                             "ms_per_launch": tot / cnt}

    P = 12 if w.kind == 0 else 24
    K = 4 if w.code_bits == 30 else 8
    d = (w.code_bits + 7) // 8
    bpp = build_bytes_per_prim(P, K, d)
    for name, b in bpp.items():
        if name in kernels:
            gbps = b * w.n / (kernels[name]["ms_per_launch"] * 1e-3) / 1e9
            kernels[name]["alg_bytes_per_launch"] = b * w.n
            kernels[name]["achieved_gbps"] = gbps
    build_kernels = {k: v for k, v in kernels.items() if k in bpp}
    dom = max(build_kernels, key=lambda k: build_kernels[k]["ms_per_step"])
    dk = kernels[dom]
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(dk["achieved_gbps"], 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(dk["achieved_gbps"] / HBM_PEAK_GBPS, 4),
        "traffic": None,
        "alg_bytes_per_launch": int(dk["alg_bytes_per_launch"]),
        "ms_per_launch": round(dk["ms_per_launch"], 4),
    }
    model_bytes = (bpp["bounds"] + bpp["morton"] + d * bpp["sort_pass"] + bpp["bottomup"]) * w.n

    # stream-copy bandwidth in the same run, for context
    buf = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(buf)
    for _ in range(3):
        dst.copy_(buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(buf)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * buf.numel() * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del buf, dst

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = max(1, int(w.n * args.cpu_sample))
        ms_ = max(1, int(w.m * args.cpu_sample))
        sub_p = np.ascontiguousarray(w.prims[:ns])
        sub_q = np.ascontiguousarray(w.queries[:ms_])
        log(f"[bench] cpu baseline: oracle on {ns} primitives, {ms_} queries")
        c0 = time.perf_counter()
        ref = oracle.build(w.kind, sub_p, w.code_bits)
        c1 = time.perf_counter()
        oracle.query_traverse(w.qkind, sub_q, ref)
        c2 = time.perf_counter()
        cpu = {"value": round(ns / (c1 - c0) / 1e6, 3), "unit": "Mprims/s", "cores": 1,
               "kind": "oracle",
               "sample": f"first {ns} of the {w.n} primitives (build) and first {ms_} of the "
                         f"{w.m} queries (Alg. 1 on the oracle tree); single-threaded C",
               "build_s": round(c1 - c0, 3), "query_s": round(c2 - c1, 3),
               "queries_mqps": round(ms_ / (c2 - c1) / 1e6, 3)}
        log(f"[bench] cpu baseline done in {c2 - c0:.1f}s")

    out = {
        "metric": "rope-LBVH build Mprims/s + stackless Mqueries/s",
        "value": round(w.n / (mean_build * 1e-3) / 1e6, 2),
        "unit": "Mprims/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "kind": "points" if w.kind == 0 else "boxes",
                   "code_bits": w.code_bits, "m": w.m,
                   "queries": "spheres" if w.qkind == 0 else "boxes"},
        "build_ms": round(mean_build, 4),
        "queries": None if args.build_only else {
            "mqueries_per_s": round(w.m / (mean_query * 1e-3) / 1e6, 2),
            "ms": round(mean_query, 4), "hits": hits},
        "build_model_bytes": int(model_bytes),
        "build_model_gbps": round(model_bytes / (mean_build * 1e-3) / 1e9, 1),
        "copy_gbps": round(copy_gbps, 1),
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
