"""Benchmark of the rope-LBVH hot path on one MI355X.

One step = one full pass of the path over resident inputs: build (scene box,
Morton codes, radix sort, Alg. 4 bottom-up pass) followed by the stackless
range queries (count pass, offset scan, read of the total, fill pass).

The timed steps launch the library's kernels directly (--graph replays the
build from a HIP graph captured once: same kernels, same buffers, measured
the same); the queries include the read of the hit total between count and
fill.  Per-kernel times come from a second, untimed pass of the same steps
with the library's per-launch events on, which cost about 65 us of host
time per build when left in the timed loop.

Prints one JSON line:
  value        build throughput, Mprims/s (n / median build time of the
               timed steps: 3 warmups, then the median of 10 by default)
  ms_per_step  mean wall time of a whole step (build + queries)
  queries      query throughput of the same steps (median), and their
               roofline: bytes per query from the oracle's exact Alg. 1 visit
               counts on the identical tree
  roofline     the dominant build kernel (level 0 of the bottom-up pass):
               its stage bytes in the fixed byte model, K + P + 100 per
               primitive for all n leaves one launch processes, over its mean
               launch time (HIP events the library records on the launch
               stream), against the 8 TB/s HBM peak
  cpu_baseline the plain C oracle on the host's cores (all of them, with
               OpenMP over its independent loops), and on one core

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
# K = code bytes, d = radix passes): each array element a kernel must move
# between HBM and the chip, counted once per kernel:
#   bounds    read the primitive (P)
#   morton    read the primitive, write its code (P + K)
#   sort pass read key (+ 4-byte value after the first pass), write key and
#             value (averaged over the d passes)
#   bottomup  level 0 of the bottom-up pass: read the code (K), leaf_perm (4)
#             and the primitive (P, a gather), write the leaf record (32),
#             the internal record (32) and the store slot (4); sibling boxes
#             and arrival flags stay in LDS
def build_bytes_per_prim(P: int, K: int, d: int) -> dict:
    return {
        "bounds": P,
        "morton": P + K,
        "sort_pass": ((2 * K + 4) + (d - 1) * (2 * K + 8)) / d,
        "bottomup": K + 4 + P + 32 + 32 + 4,
    }


# The fixed whole-build byte model used for the roofline target, with
# 8-bit digits (d8 = ceil(bits / 8) passes):
#   bounds P, Morton P + K, sort 2K + (2 d8 - 1)(K + 4), bottom-up K + P + 100
# (the bottom-up stage: codes K, leaf_perm 4, primitive gather P, store init
# 4, store CAS 8, sibling box 24, leaf record 28, internal record 32).
def model_stage_bytes_per_prim(P: int, K: int, d8: int) -> dict:
    return {"bounds": P, "morton": P + K, "sort": 2 * K + (2 * d8 - 1) * (K + 4),
            "bottomup": K + P + 100}


def build_model_bytes_per_prim(P: int, K: int, d8: int) -> float:
    return float(sum(model_stage_bytes_per_prim(P, K, d8).values()))


def host_info() -> dict:
    """Host cores this process may use (its CPU affinity, capped by
    OMP_NUM_THREADS when that is set) and the CPU model."""
    affinity = len(os.sched_getaffinity(0))
    cores = affinity
    try:
        cores = max(1, min(affinity, int(os.environ.get("OMP_NUM_THREADS", affinity))))
    except ValueError:
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cores": cores, "affinity_cores": affinity, "cpu_model": model}


KERNEL_SOURCES = ["paper_2402_00665_amd/csrc/build_kernels.hip",
                  "paper_2402_00665_amd/csrc/batch_kernels.hip",
                  "paper_2402_00665_amd/csrc/query_kernels.hip",
                  "paper_2402_00665_amd/csrc/bottomup.hpp",
                  "paper_2402_00665_amd/csrc/radix_sort.hpp",
                  "paper_2402_00665_amd/csrc/query_common.hpp",
                  "paper_2402_00665_amd/csrc/device_common.hpp",
                  "paper_2402_00665_amd/csrc/lbvh_internal.hpp"]


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps (the reported build and query times are their medians)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered_boxes",
                    choices=["clustered_boxes", "large_points", "small_points"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain comparison (4096 scenes)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--no-rays", action="store_true",
                    help="skip the ray leg (clustered boxes only: first hits of 2^20 rays, all "
                         "hits of 2^20 segments, on the same tree)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default launch shapes instead of autotuned ones")
    ap.add_argument("--knobs", default="",
                    help="set tuning knobs (name=value,...) instead of autotuning")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the Poisson arrival trace")
    ap.add_argument("--serve-slots", type=int, default=3, help="streams of the batching server")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="HBM budget for in-flight batches and resident trees")
    ap.add_argument("--graph", action="store_true",
                    help="replay the timed builds from a HIP graph captured once instead of "
                         "launching them one kernel at a time (measured the same)")
    ap.add_argument("--build-only", action="store_true",
                    help="time the build alone (no queries in the step)")
    ap.add_argument("--cpu-sample", type=float, default=1.0,
                    help="fraction of the workload the oracle baseline runs on")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="repeat each oracle baseline leg until this much time is spent (max 8 runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched build + queries (no plain per-scene leg, no "
                         "single-tree or serving legs); for profiling the batched kernels")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="turn rocprofv3 outputs (kernel-trace --stats run, --pmc FETCH_SIZE "
                         "run, --pmc WRITE_SIZE run) into profiles/ summaries and exit")
    ap.add_argument("--command", default="", help="with --summarize: the profiled command")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_bandwidth() -> float:
    """GB/s of a 256 MiB device-to-device copy (read + write), for context;
    it is also the copy of known size the traffic counters are scaled by."""
    import torch
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
    gbps = 2 * buf.numel() * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del buf, dst
    return gbps


def main():
    args = parse()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this path has no multi-GPU form)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2402_00665_amd as lb
    import workloads

    torch.cuda.set_device(0)
    # the library's knob values before any leg tunes them: each later leg
    # starts from these (the batched leg tunes its own; serving runs on them)
    knob_defaults = {k: lb.lbvh_tune(k) for k in KNOBS}

    def reset_knobs():
        for k, v in knob_defaults.items():
            lb.lbvh_tune(k, v)

    if args.batched_only:
        for kv in filter(None, args.knobs.split(",")):
            k, v = kv.split("=")
            lb.lbvh_tune(k.strip(), int(v))
        batched = bench_batched(args, plain=False)
        print(json.dumps({"batched": batched, "copy_gbps": round(copy_bandwidth(), 1)}), flush=True)
        return
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

    tuning = None
    if args.knobs:
        tuning = {}
        for kv in args.knobs.split(","):
            k, v = kv.split("=")
            lb.lbvh_tune(k.strip(), int(v))
            tuning[k.strip()] = int(v)
        log(f"[bench] knobs set: {tuning}")
    elif not args.no_autotune:
        # the library's own autotuner, run once on this workload before any
        # timing (as a user would): radix tile shape and query schedule
        from paper_2402_00665_amd import autotune
        a0 = time.time()
        ts = autotune.tune(prims, w.code_bits, kind=w.kind, reps=3, save=False)
        for k, v in ts["knobs"].items():
            lb.lbvh_tune(k, v)
        tuning = dict(ts["knobs"])
        if not args.build_only:
            lb.build(prims, w.code_bits, kind=w.kind, workspace=ws, tree=tree)
            tq = autotune.tune_query(tree, queries, w.qkind, reps=3, save=False)
            for k, v in zip(("query_split1", "query_split2", "query_leaf_mode", "query_order"),
                            tq["value"]):
                lb.lbvh_tune(k, v)
                tuning[k] = v
        log(f"[bench] autotuned in {time.time() - a0:.1f}s: {tuning}")

    def build_eager():
        lb.build(prims, w.code_bits, kind=w.kind, workspace=ws, tree=tree)

    run_build = build_eager
    if args.graph:
        # the build's launches captured once in a HIP graph and replayed:
        # the same kernels on the same buffers, one launch call per build
        build_eager()
        torch.cuda.synchronize()
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(graph, stream=gs):
                build_eager()
        torch.cuda.synchronize()
        run_build = graph.replay

    def step(ev=None, build=None):
        if ev:
            ev[0].record(stream)
        (build or run_build)()
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

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    hits = 0
    for k in range(args.steps):
        off, idx = step(evs[k])
        hits = int(idx.numel()) if idx is not None else 0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lb.check_build(tree)
    log(f"[bench] timed {args.steps} steps in {wall:.3f}s")

    # per-kernel times: the same steps again, eager, with the library's
    # per-launch events on (kept out of the timed loop above)
    lb.lbvh_profile_reset()
    lb.lbvh_profile_enable(True)
    for _ in range(args.steps):
        step(build=build_eager)
    torch.cuda.synchronize()
    lb.lbvh_profile_enable(False)

    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    query_ms = [e[1].elapsed_time(e[2]) for e in evs]
    med_build = float(np.median(build_ms))
    med_query = float(np.median(query_ms))
    ms_per_step = wall * 1e3 / args.steps

    kernels = {}
    for name in ["bounds", "bounds_final", "morton", "sort_pass", "bottomup", "bottomup_up",
                 "query_order", "query_split", "query_count", "scan", "query_fill"]:
        tot, cnt = lb.lbvh_profile_read(name)
        if cnt:
            kernels[name] = {"ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps,
                             "ms_per_launch": tot / cnt}

    P = 12 if w.kind == 0 else 24
    K = 4 if w.code_bits == 30 else 8
    d8 = (w.code_bits + 7) // 8
    radix_bits = lb.lbvh_tune(f"radix_bits{32 if w.code_bits == 30 else 64}")
    d = (w.code_bits + radix_bits - 1) // radix_bits
    bpp = build_bytes_per_prim(P, K, d)
    for name, b in bpp.items():
        if name in kernels:
            gbps = b * w.n / (kernels[name]["ms_per_launch"] * 1e-3) / 1e9
            kernels[name]["alg_bytes_per_launch"] = b * w.n
            kernels[name]["achieved_gbps"] = gbps
    build_kernels = {k: v for k, v in kernels.items() if k in bpp}
    dom = max(build_kernels, key=lambda k: build_kernels[k]["ms_per_step"])
    dk = kernels[dom]
    traffic = measured_traffic(w.name, dom)
    # the dominant kernel's stage bytes in the fixed model: the bottom-up
    # stage for level 0 (it takes all n leaves), else the kernel's own bytes
    stage = model_stage_bytes_per_prim(P, K, d8)
    unit_bytes = stage["bottomup"] if dom == "bottomup" else bpp[dom]
    roof_bytes = unit_bytes * w.n
    achieved = roof_bytes / (dk["ms_per_launch"] * 1e-3) / 1e9
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": None if traffic is None else int(traffic),
        "bytes_per_unit": unit_bytes,
        "units_per_launch": w.n,
        "alg_bytes_per_launch": int(roof_bytes),
        "ms_per_launch": round(dk["ms_per_launch"], 4),
        # the bytes the kernel itself must move (LDS-resident sibling boxes
        # and arrival flags not counted), over the same time
        "kernel_bytes_per_launch": int(dk["alg_bytes_per_launch"]),
        "kernel_frac": round(dk["achieved_gbps"] / HBM_PEAK_GBPS, 4),
        # the measured HBM bytes over the same launch time: how close the
        # kernel runs to the memory system, whatever its algorithmic bytes
        "traffic_gbps": None if traffic is None else round(traffic / (dk["ms_per_launch"] * 1e-3) / 1e9, 1),
        "traffic_frac": None if traffic is None else
        round(traffic / (dk["ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
    }
    model_bytes = build_model_bytes_per_prim(P, K, d8) * w.n

    copy_gbps = copy_bandwidth()

    cpu = None
    visits = None
    if not args.no_cpu_baseline:
        import oracle
        host = host_info()
        ns = max(1, int(w.n * args.cpu_sample))
        ms_ = max(1, int(w.m * args.cpu_sample))
        sub_p = np.ascontiguousarray(w.prims[:ns])
        sub_q = np.ascontiguousarray(w.queries[:ms_])
        legs = {}
        for threads in (host["cores"], 1):
            log(f"[bench] cpu baseline: oracle on {ns} primitives, {ms_} queries, {threads} thread(s)")
            oracle.threads(threads)
            tb = tq = 0.0
            runs = 0
            try:
                while runs == 0 or (tb + tq < args.cpu_seconds and runs < 8):
                    c0 = time.perf_counter()
                    ref = oracle.build(w.kind, sub_p, w.code_bits)
                    c1 = time.perf_counter()
                    _, _, vis = oracle.query_traverse(w.qkind, sub_q, ref)
                    c2 = time.perf_counter()
                    tb, tq, runs = tb + (c1 - c0), tq + (c2 - c1), runs + 1
                    del ref
            finally:
                oracle.threads(1)
            if ns == w.n and ms_ == w.m:
                visits = vis
            legs[threads] = {"value": round(runs * ns / tb / 1e6, 3), "cores": threads,
                             "runs": runs, "build_s": round(tb / runs, 3),
                             "query_s": round(tq / runs, 3),
                             "queries_mqps": round(runs * ms_ / tq / 1e6, 3)}
            log(f"[bench] cpu baseline, {threads} thread(s): {runs} run(s) in {tb + tq:.1f}s")
        T = host["cores"]
        cpu = {"value": legs[T]["value"], "unit": "Mprims/s", "cores": T, "kind": "oracle",
               "sample": f"build over the first {ns} of the {w.n} primitives (scene box, Morton "
                         "codes, qsort, top-down tree, DFS ropes, range-union boxes), then Alg. 1 "
                         f"for the first {ms_} of the {w.m} queries on the oracle tree; C with "
                         f"OpenMP over its independent loops on {T} thread(s) (sort, top-down "
                         "split and rope walk sequential)",
               "host": host, "build_s": legs[T]["build_s"], "query_s": legs[T]["query_s"],
               "queries_mqps": legs[T]["queries_mqps"], "runs": legs[T]["runs"],
               "single_thread": legs[1]}

    qroof = None
    if visits is not None and not args.build_only:
        # bytes per query call: the query (16 or 24 B) and its offset (8 B),
        # one 32-byte node record per Alg. 1 visit, 4 B per hit written
        qbytes = w.m * ((16 if w.qkind == 0 else 24) + 8) + 32 * visits + 4 * hits
        qgbps = qbytes / (med_query * 1e-3) / 1e9
        qroof = {"bound": "hbm", "achieved": round(qgbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": round(qgbps / HBM_PEAK_GBPS, 4), "bytes": int(qbytes),
                 "visits": int(visits), "visits_per_query": round(visits / w.m, 2),
                 "note": "node bytes counted once per visit; upper tree levels stay in cache, "
                         "so this can exceed what HBM alone would allow"}

    rays = None
    if not args.no_rays and w.name == "clustered_boxes" and not args.build_only:
        rays = bench_rays(args, w, tree)

    tuned_here = {k: lb.lbvh_tune(k) for k in KNOBS}
    reset_knobs()
    batched = None if args.no_batched else bench_batched(args)
    reset_knobs()
    serving = None if args.no_serving else bench_serving(args)
    for k, v in tuned_here.items():   # the single-tree workload's knobs again, for what follows
        lb.lbvh_tune(k, v)

    out = {
        "metric": "rope-LBVH build Mprims/s + stackless Mqueries/s",
        "value": round(w.n / (med_build * 1e-3) / 1e6, 2),
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
                   "code_bits": w.code_bits, "radix_bits": radix_bits, "m": w.m,
                   "queries": "spheres" if w.qkind == 0 else "boxes",
                   "build_launch": "hip_graph" if args.graph else "eager"},
        "build_ms": round(med_build, 4),
        "build_ms_mean": round(float(np.mean(build_ms)), 4),
        "queries": None if args.build_only else {
            "mqueries_per_s": round(w.m / (med_query * 1e-3) / 1e6, 2),
            "ms": round(med_query, 4), "ms_mean": round(float(np.mean(query_ms)), 4),
            "hits": hits, "roofline": qroof},
        "build_model_bytes": int(model_bytes),
        "build_model_gbps": round(model_bytes / (med_build * 1e-3) / 1e9, 1),
        "build_model_frac": round(model_bytes / (med_build * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "copy_gbps": round(copy_gbps, 1),
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "tuning": tuning,
        "cpu_baseline": cpu,
        "rays": rays,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------- rays

def bench_rays(args, w, tree, reps: int = 10):
    """Rays and segments on the built tree (the clustered boxes): first
    hits of 2^20 rays through random points of random boxes, and all hits
    of 2^20 segments of length 0.002 from such points (the clustered_rays /
    clustered_segments workloads).  Median of ``reps`` timed calls after
    two warm-ups (their parity with the oracle is the GPU tests' job)."""
    import torch
    import paper_2402_00665_amd as lb
    import workloads
    t0 = time.time()
    rays = workloads.clustered_ray_queries(w.prims, w.m, segments=False)
    segs = workloads.clustered_ray_queries(w.prims, w.m, segments=True)
    log(f"[bench] rays: {w.m} rays, {w.m} segments (generated in {time.time() - t0:.1f}s)")
    dr, dsg = torch.from_numpy(rays).cuda(), torch.from_numpy(segs).cuda()
    ws = lb.Workspace()
    # the segments' own query schedule (thin queries: walks beat scans)
    qknobs = ("query_split1", "query_split2", "query_leaf_mode", "query_order")
    saved = {k: lb.lbvh_tune(k) for k in qknobs}
    tuned = None
    if not args.no_autotune and not args.knobs:
        from paper_2402_00665_amd import autotune
        tq = autotune.tune_query(tree, dsg, lb.RAYS, reps=2, save=False)
        tuned = dict(zip(qknobs, tq["value"]))
        for k, v in tuned.items():
            lb.lbvh_tune(k, v)
        log(f"[bench] rays: segment schedule {tuned}")
    hit = torch.empty(w.m, dtype=torch.int32, device="cuda")
    tt = torch.empty(w.m, dtype=torch.float32, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    first_ms, all_ms = [], []
    for r in range(reps + 2):
        e[0].record()
        lb.query_first(tree, dr, workspace=ws, hit=hit, t=tt)
        e[1].record()
        torch.cuda.synchronize()
        if r >= 2:
            first_ms.append(e[0].elapsed_time(e[1]))
    lb.check_query(ws, w.m)
    for r in range(reps + 2):
        e[0].record()
        off, idx = lb.query(tree, dsg, lb.RAYS, workspace=ws)
        e[1].record()
        torch.cuda.synchronize()
        if r >= 2:
            all_ms.append(e[0].elapsed_time(e[1]))
    lb.check_query(ws, w.m)
    for k, v in saved.items():
        lb.lbvh_tune(k, v)
    hit_h = hit.cpu().numpy()
    off_h = off.cpu().numpy()
    fm, am = float(np.median(first_ms)), float(np.median(all_ms))
    return {"workload": "clustered_rays / clustered_segments", "m": w.m,
            "first_hit_ms": round(fm, 4), "first_hit_mrays_per_s": round(w.m / (fm * 1e-3) / 1e6, 1),
            "rays_hit": int((hit_h >= 0).sum()),
            "segments_ms": round(am, 4),
            "segments_mqueries_per_s": round(w.m / (am * 1e-3) / 1e6, 1),
            "segment_hits": int(off_h[-1]), "segment_tuning": tuned}


# ---------------------------------------------------------------- batched

def bench_batched(args, reps: int = 5, plain: bool = True):
    """4096 uniform point sets (sizes log-uniform in [32, 65536], 63-bit
    codes, 64 spheres of radius 0.05 each): one batched launch sequence for
    all scenes (the build replayed from a HIP graph captured once) against
    one plain build + query per scene, same GPU, same stream.  Both produce every scene's tree; they are compared bit for bit
    on the device."""
    import torch
    import paper_2402_00665_amd as lb
    import workloads
    t0 = time.time()
    pts, off, q, qoff = workloads.batched()
    S, N, m = len(off) - 1, int(off[-1]), q.shape[0]
    max_scene = int(np.diff(off).max())
    log(f"[bench] batched workload: S={S} N={N} m={m} (generated in {time.time() - t0:.1f}s)")
    dp, ds = torch.from_numpy(pts).cuda(), torch.from_numpy(off).cuda()
    dq, dqs = torch.from_numpy(q).cuda(), torch.from_numpy(qoff).cuda()
    ws, qws = lb.Workspace(), lb.Workspace()
    tuned = None
    if not args.no_autotune and not args.knobs:
        from paper_2402_00665_amd import autotune
        t = autotune.tune(dp, 63, kind=lb.LBVH_POINTS, seg_off=ds, max_scene=max_scene, reps=2,
                          save=False)
        for k, v in t["knobs"].items():
            lb.lbvh_tune(k, v)
        tuned = dict(t["knobs"])
        log(f"[bench] batched: autotuned {tuned}")
    b = lb.build_batched(dp, ds, 63, max_scene, workspace=ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    # the batched build's launches captured once in a HIP graph and
    # replayed for every batch (same kernels, same buffers)
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            lb.build_batched(dp, ds, 63, max_scene, workspace=ws, batch=b)
    torch.cuda.synchronize()

    def batched_step():
        graph.replay()
        ev[1].record()
        return lb.query_batched(b, dq, dqs, 0, workspace=qws)

    for _ in range(2):
        batched_step()
    torch.cuda.synchronize()
    lb.check_batched(b)
    bt, qt, wt = [], [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev[0].record()
        boff, bidx = batched_step()
        ev[2].record()
        torch.cuda.synchronize()
        wt.append(time.perf_counter() - w0)
        bt.append(ev[0].elapsed_time(ev[1]))
        qt.append(ev[1].elapsed_time(ev[2]))

    bb, bq, bw = float(np.median(bt)), float(np.median(qt)), float(np.median(wt))
    res = {
        "workload": "batched_scenes", "scenes": S, "n": N, "m": m, "code_bits": 63,
        "batched_build_ms": round(bb, 4), "batched_query_ms": round(bq, 4),
        "batched_wall_ms": round(bw * 1e3, 3),
        "batched_mprims_per_s": round(N / (bb * 1e-3) / 1e6, 1),
        "build_launch": "hip_graph",
        "tuning": tuned,
    }
    if not plain:
        return res

    # plain: one single-scene build and one query call per scene
    off_h, qoff_h = off.tolist(), qoff.tolist()
    trees = [lb.alloc_tree(off_h[s + 1] - off_h[s], 63) for s in range(S)]
    # each scene in its own allocation, as a caller of the single-tree entry
    # point holds it (a slice of the packed array is not 16-byte aligned)
    scene_p = [dp[off_h[s]:off_h[s + 1]].clone() for s in range(S)]
    pws, pqws = lb.Workspace(), lb.Workspace()

    def plain_pass(with_queries):
        res = []
        for s in range(S):
            t = lb.build(scene_p[s], 63, kind=0, workspace=pws, tree=trees[s])
            if with_queries:
                res.append(lb.query(t, dq[qoff_h[s]:qoff_h[s + 1]], 0, workspace=pqws))
        return res

    plain_pass(True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    plain_pass(False)
    torch.cuda.synchronize()
    plain_build_s = time.perf_counter() - w0
    w0 = time.perf_counter()
    pres = plain_pass(True)
    torch.cuda.synchronize()
    plain_all_s = time.perf_counter() - w0

    # same trees and results, scene by scene
    same = True
    for s in range(S):
        a, e = off_h[s], off_h[s + 1]
        if e > a:
            same &= bool(torch.equal(b.nodes[2 * a:2 * a + 2 * (e - a) - 1], trees[s].nodes))
        qa, qe = qoff_h[s], qoff_h[s + 1]
        po, pi = pres[s]
        same &= bool(torch.equal(boff[qa:qe + 1] - boff[qa], po))
        same &= bool(torch.equal(bidx[int(boff[qa]):int(boff[qe])], pi))
    res.update({
        "plain_build_ms": round(plain_build_s * 1e3, 3),
        "plain_wall_ms": round(plain_all_s * 1e3, 3),
        "plain_mprims_per_s": round(N / plain_build_s / 1e6, 1),
        "build_speedup": round(plain_build_s * 1e3 / bb, 2),
        "wall_speedup": round(plain_all_s / bw, 2),
        "identical": same,
    })
    return res


# ---------------------------------------------------------------- serving

def bench_serving(args):
    """The serving stream (Poisson arrivals at 2000 requests/s; each request
    builds the tree of n uniform points, n log-uniform in [1e3, 4e6], 63-bit
    codes, and answers 10^4 spheres with about 8 expected neighbours),
    served twice on the same trace in real time: FIFO one request at a time
    through the single-tree entry points, and continuous batching through
    the batched ones on 3 streams.  Latency = completion - arrival.  Each
    finished request's answer is handed to the client: copied, on the
    batch's stream, into a client-owned device buffer (one per run,
    allocated before the runs, request k at the same place in both), after
    which the server drops it.  After the two runs the two buffers are
    compared whole, so every request's answer is checked.  Both servers run
    with the library's default knobs (not the single-tree workload's tuned
    ones)."""
    import torch
    import workloads
    from paper_2402_00665_amd import serve
    t0 = time.time()
    plan = workloads.serving_plan(seconds=args.serve_seconds)
    pts, ctr = workloads.serving_pools()
    dp, dc = torch.from_numpy(pts).cuda(), torch.from_numpy(ctr).cuda()
    R = len(plan["n"])

    def reqs(lo, hi, shift=0.0):
        return [serve.Request(k, float(plan["arrival"][k]) - shift, int(plan["n"][k]),
                              int(plan["m"][k]), int(plan["p_off"][k]), int(plan["q_off"][k]),
                              float(plan["radius"][k])) for k in range(lo, hi)]

    log(f"[bench] serving: {R} requests over {args.serve_seconds:.0f}s "
        f"(generated in {time.time() - t0:.1f}s)")
    budget = int(args.serve_budget_gib * (1 << 30))
    # the clients' buffers: offsets of request k at its prefix of (m + 1),
    # indices placed by the first run as they come (10 hits per sphere of
    # room; about 8 are expected) and at the same places in the second
    m_all = plan["m"].astype(np.int64)
    off_pos = np.concatenate([[0], np.cumsum(m_all + 1)])
    idx_cap = int(10 * m_all.sum())
    arena = {mode: (torch.empty(int(off_pos[-1]), dtype=torch.int64, device="cuda"),
                    torch.empty(idx_cap, dtype=torch.int32, device="cuda"))
             for mode in ("fifo", "continuous")}
    idx_pos = {}          # rid -> (start, hits) in the indices buffers
    state = {"next": 0, "mismatch": 0, "skipped": 0}

    def hand_over(mode):
        a_off, a_idx = arena[mode]

        def done(o):   # runs with the batch's stream current
            k = o.rid
            if mode == "fifo":
                if state["next"] + o.hits > idx_cap:
                    state["skipped"] += 1
                    return
                idx_pos[k] = (state["next"], o.hits)
                state["next"] += o.hits
            elif k not in idx_pos:
                return
            elif idx_pos[k][1] != o.hits:
                state["mismatch"] += 1
                return
            p0, h = idx_pos[k]
            o.csr(out=(a_off[int(off_pos[k]):int(off_pos[k + 1])], a_idx[p0:p0 + h]))
        return done

    res = {}
    for mode in ("fifo", "continuous"):
        ex = (serve.PlainExecutor(dp, dc) if mode == "fifo"
              else serve.GpuExecutor(dp, dc, slots=args.serve_slots))
        warm = reqs(0, min(R, 400))
        wsrv = serve.Server(ex, budget, max_batch=1 if mode == "fifo" else 64, keep_results=False)
        wsrv.run(warm)
        wsrv.evict_all()
        del wsrv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()   # both modes start from the same allocator state
        srv = serve.Server(ex, budget, max_batch=1 if mode == "fifo" else 64, keep_results=False,
                           on_done=hand_over(mode))
        w0 = time.perf_counter()
        out = srv.run(reqs(0, R))
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        s = serve.summarize(out)
        if not s["ok"]:
            raise RuntimeError(f"serving {mode}: no request succeeded: {s}")
        ok = [o for o in out if o.status == serve.LBVH_OK]
        npts = sum(int(plan["n"][o.rid]) for o in ok)
        nq = sum(int(plan["m"][o.rid]) for o in ok)
        s.update({"wall_s": round(wall, 3),
                  "mprims_per_s": round(npts / s["makespan_s"] / 1e6, 1),
                  "mqueries_per_s": round(nq / s["makespan_s"] / 1e6, 2),
                  "batches": len(srv.batches),
                  "mean_batch": round(float(np.mean([b[1] for b in srv.batches])), 2),
                  "peak_gib": round(srv.peak_bytes / (1 << 30), 2)})
        if mode == "continuous":
            s["slots"] = args.serve_slots
        res[mode] = s
        log(f"[bench] serving {mode}: {s}")
        srv.evict_all()
        del srv
    # both buffers hold every handed-over answer at the same places
    used = state["next"]
    compared = len(idx_pos) if state["mismatch"] == 0 else 0
    same = (state["mismatch"] == 0 and state["skipped"] == 0 and compared == R
            and bool(torch.equal(arena["fifo"][0], arena["continuous"][0]))
            and bool(torch.equal(arena["fifo"][1][:used], arena["continuous"][1][:used])))
    del arena
    torch.cuda.empty_cache()
    f, c = res["fifo"], res["continuous"]
    return {"workload": "serving_stream", "rate_per_s": 2000, "seconds": args.serve_seconds,
            "requests": R, "budget_gib": args.serve_budget_gib, "fifo": f, "continuous": c,
            "p99_speedup": round(f["p99_ms"] / c["p99_ms"], 2),
            "throughput_ratio": round(c["throughput_rps"] / f["throughput_rps"], 3),
            "identical": same, "compared": compared}


# --------------------------------------------------------------- profiles

KNOBS = ("sort_variant32", "sort_variant64", "batch_sort_variant", "query_split1", "query_split2",
         "query_leaf_mode", "query_order", "radix_bits32", "radix_bits64", "morton_order",
         "batch_sort_mode", "radix_mode")

KERNEL_GROUPS = {  # rocprofv3 kernel-name fragment -> bench kernel name (first match wins)
    "k_onesweep<unsigned int, 512, 4>": "query_order", "k_qorder": "query_order",
    "k_bounds<": "bounds", "k_bounds_final": "bounds_final", "k_morton": "morton",
    "k_onesweep": "sort_pass", "k_bottomup_l0": "bottomup", "k_bottomup_up": "bottomup_up",
    "k_split": "query_split", "k_leaf_scan_count": "query_count", "k_leaf_count_wide": "query_count",
    "k_leaf_mixed_count": "query_count", "k_leaf_fill": "query_fill", "copyBuffer": "copy",
    "k_batch_plan": "batch_plan", "k_batch_morton": "morton", "k_batch_count": "query_count",
    "k_batch_fill": "query_fill", "k_scene_sort": "scene_sort", "k_ray_first": "ray_first",
    "k_radix_count": "sort_count",
}


def _group(name: str):
    for frag, g in KERNEL_GROUPS.items():
        if frag in name:
            return g
    return None


def summarize(args):
    """Write profiles/<workload> summaries from rocprofv3 CSV outputs: the
    --kernel-trace --stats table, and per-kernel HBM bytes from the two
    --pmc runs, each counter scaled by what it reads for the 256 MiB device
    copy the bench itself runs (a copy of known size)."""
    import csv
    import collections
    import glob
    stats_dir, fetch_dir, write_dir = args.summarize
    name = "batched_scenes" if args.batched_only else args.workload

    def one(pattern):
        got = glob.glob(os.path.join(pattern, "**", "*"), recursive=True)
        return got

    stats = [f for f in one(stats_dir) if f.endswith("kernel_stats.csv")][0]
    rows = list(csv.DictReader(open(stats)))
    lines = [f"# Kernel time: {name}", "",
             f"Command: `{args.command}`", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        nm = r["Name"].replace("lbvh::(anonymous namespace)::", "")
        nm = nm.split("(")[0].replace("void ", "")
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"kernels_{name}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_dispatch(d, counter):
        f = [x for x in one(d) if x.endswith("counter_collection.csv")][0]
        agg = collections.OrderedDict()
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]))
            agg[key] = agg.get(key, 0.0) + float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
        return agg

    fetch, write = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    copy_bytes = 1 << 28
    def calib(agg):
        vals = [v for (d, nm, g), v in agg.items() if "copyBuffer" in nm and v > copy_bytes / 8]
        return copy_bytes / (sum(vals) / len(vals))
    # the copy reads 256 MiB and writes 256 MiB
    cf, cw = calib(fetch), calib(write)
    out = collections.defaultdict(lambda: {"fetch": [], "write": []})
    for (d, nm, g), v in fetch.items():
        grp = _group(nm)
        if grp and grp != "copy":
            out[grp]["fetch"].append(v * cf)
    for (d, nm, g), v in write.items():
        grp = _group(nm)
        if grp and grp != "copy":
            out[grp]["write"].append(v * cw)
    kernels = {}
    for grp, dv in out.items():
        fb = sum(dv["fetch"]) / max(len(dv["fetch"]), 1)
        wb = sum(dv["write"]) / max(len(dv["write"]), 1)
        kernels[grp] = {"fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
                        "hbm_bytes_per_launch": int(fb + wb), "launches": len(dv["fetch"])}
    doc = {"workload": name, "command": args.command,
           "calibration": {"fetch_scale": cf, "write_scale": cw,
                           "copy_kernel": "__amd_rocclr_copyBuffer, 256 MiB device copy"},
           "source_sha256": source_hash(), "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", f"traffic_{name}.json"), "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc, indent=1))


if __name__ == "__main__":
    main()
