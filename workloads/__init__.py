"""Seeded synthetic inputs for the rope-LBVH build and range queries.

This module only draws numbers: it holds none of the method's arithmetic
(no Morton codes, no sorting, no tree logic), so both the CPU oracle and the
HIP path can take their inputs from it.

Every array is float32 and C-contiguous:
  points  : [n, 3]  (x, y, z)
  boxes   : [n, 6]  (lo.x, lo.y, lo.z, hi.x, hi.y, hi.z)
  spheres : [m, 4]  (c.x, c.y, c.z, r)
  qboxes  : [m, 6]  same layout as boxes
  rays    : [m, 8]  (o.x, o.y, o.z, tmin, d.x, d.y, d.z, tmax): the points
            o + t*d for tmin <= t <= tmax (a segment is [0, 1] with d its
            end minus its start; a ray has tmax = +inf)

Random streams come from ``numpy.random.default_rng([cfg_id, stream])`` with
stream 0 for primitives and stream 1 for queries, so a reduced-size variant of
a workload draws the same distribution from the same seed.

The paper's experiments use "filled cube" and "hollow cube" point clouds
(Performance results section); ``filled_cube`` / ``hollow_cube`` follow that
description with the half-width a = n^(1/3).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

POINTS = 0
BOXES = 1
SPHERES = 0
QBOXES = 1
RAYS = 2


def _rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cfg_id, stream])


def uniform_points(n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in [0,1)^3, drawn directly in float32."""
    return np.ascontiguousarray(rng.random((n, 3), dtype=np.float32))


def spheres(centers: np.ndarray, radius) -> np.ndarray:
    m = centers.shape[0]
    out = np.empty((m, 4), dtype=np.float32)
    out[:, :3] = centers
    out[:, 3] = radius
    return out


def neighbour_radius(n: int, k: float) -> float:
    """Radius whose ball holds k expected neighbours among n uniform points
    in the unit cube: r = (k / (n * 4*pi/3))^(1/3), rounded to float32."""
    return float(np.float32((k / (n * 4.0 * math.pi / 3.0)) ** (1.0 / 3.0)))


def clustered_boxes(n: int, rng: np.random.Generator, components: int = 64,
                    sigma: float = 0.005, mu: float = -7.0,
                    s: float = 0.5) -> np.ndarray:
    """Boxes whose centres come from an equal-weight Gaussian mixture.

    Means uniform in [0,1)^3, isotropic sigma, centres clamped to
    [0, 1 - 2^-24]; per-axis side lengths lognormal(mu, s); lo/hi computed in
    float64 as c -/+ side/2 and then rounded to float32 (so lo <= hi).
    """
    means = rng.random((components, 3))
    comp = rng.integers(0, components, size=n)
    c = means[comp] + rng.normal(0.0, sigma, size=(n, 3))
    np.clip(c, 0.0, 1.0 - 2.0 ** -24, out=c)
    side = rng.lognormal(mean=mu, sigma=s, size=(n, 3))
    out = np.empty((n, 6), dtype=np.float32)
    out[:, :3] = c - 0.5 * side
    out[:, 3:] = c + 0.5 * side
    return out


def query_boxes(m: int, side: float, rng: np.random.Generator) -> np.ndarray:
    """Axis-aligned query boxes of a fixed side, centres uniform in [0,1)^3."""
    c = rng.random((m, 3))
    out = np.empty((m, 6), dtype=np.float32)
    out[:, :3] = c - 0.5 * side
    out[:, 3:] = c + 0.5 * side
    return out


def points_in_boxes(boxes: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    """m points, each uniform inside a box drawn uniformly from ``boxes``
    (float64 lo + u * (hi - lo), then rounded to float32)."""
    pick = rng.integers(0, boxes.shape[0], size=m)
    lo = boxes[pick, :3].astype(np.float64)
    hi = boxes[pick, 3:].astype(np.float64)
    return (lo + rng.random((m, 3)) * (hi - lo)).astype(np.float32)


def rays_toward(targets: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Rays [0, +inf) from origins uniform in [0,1)^3 through the given
    targets (d = target - origin, so t = 1 reaches the target)."""
    m = targets.shape[0]
    o = rng.random((m, 3))
    out = np.empty((m, 8), dtype=np.float32)
    out[:, :3] = o
    out[:, 3] = 0.0
    out[:, 4:7] = targets.astype(np.float64) - o
    out[:, 7] = np.inf
    return out


def segments_from(starts: np.ndarray, length: float, rng: np.random.Generator) -> np.ndarray:
    """Segments of a fixed length from the given starts in directions
    uniform on the sphere (o = start, d = length * unit direction, [0, 1])."""
    m = starts.shape[0]
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    out = np.empty((m, 8), dtype=np.float32)
    out[:, :3] = starts
    out[:, 3] = 0.0
    out[:, 4:7] = length * u
    out[:, 7] = 1.0
    return out


def filled_cube(n: int, rng: np.random.Generator) -> np.ndarray:
    """Points uniform in [-a, a]^3 with a = n^(1/3)."""
    a = n ** (1.0 / 3.0)
    return np.ascontiguousarray(
        (rng.random((n, 3)) * 2.0 * a - a).astype(np.float32))


def hollow_cube(n: int, rng: np.random.Generator) -> np.ndarray:
    """Points on the faces of [-a, a]^3, a = n^(1/3); point k goes on face
    k mod 6, uniformly placed on it."""
    a = n ** (1.0 / 3.0)
    p = rng.random((n, 3)) * 2.0 * a - a
    face = np.arange(n) % 6
    axis = face // 2
    sign = np.where(face % 2 == 0, -a, a)
    p[np.arange(n), axis] = sign
    return np.ascontiguousarray(p.astype(np.float32))


@dataclass
class Workload:
    """One synthetic build + query problem."""
    name: str
    kind: int                # POINTS or BOXES
    prims: np.ndarray        # [n,3] or [n,6] float32
    code_bits: int           # 30 or 63
    qkind: int               # SPHERES or QBOXES
    queries: np.ndarray      # [m,4] or [m,6] float32
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.prims.shape[0])

    @property
    def m(self) -> int:
        return int(self.queries.shape[0])


# Full sizes of the five workloads.
FULL = {
    "small_points": dict(n=16384, m=1024),
    "large_points": dict(n=1 << 23, m=1 << 20),
    "clustered_boxes": dict(n=1 << 24, m=1 << 20),
    "batched_scenes": dict(S=4096, m_per=64),
    "serving_stream": dict(rate=2000.0, seconds=30.0, m=10000),
}

CFG_ID = {"small_points": 1, "large_points": 2, "clustered_boxes": 3,
          "batched_scenes": 4, "serving_stream": 5}


def small_points(n: int = 16384, m: int = 1024) -> Workload:
    """16384 uniform points, 30-bit codes, 1024 spheres of radius 0.02."""
    p = uniform_points(n, _rng(1, 0))
    q = spheres(uniform_points(m, _rng(1, 1)), np.float32(0.02))
    return Workload("small_points", POINTS, p, 30, SPHERES, q)


def large_points(n: int = 1 << 23, m: int = 1 << 20) -> Workload:
    """2^23 uniform points, 63-bit codes, 2^20 spheres with about 16
    expected neighbours (radius computed for this n)."""
    p = uniform_points(n, _rng(2, 0))
    r = neighbour_radius(n, 16.0)
    q = spheres(uniform_points(m, _rng(2, 1)), np.float32(r))
    return Workload("large_points", POINTS, p, 63, SPHERES, q, {"radius": r})


def clustered(n: int = 1 << 24, m: int = 1 << 20) -> Workload:
    """2^24 boxes from a 64-component Gaussian mixture (sigma 0.005),
    lognormal sides (mu -7, s 0.5), 30-bit codes (heavy duplicate codes);
    2^20 query boxes of side 0.01 with uniform centres."""
    b = clustered_boxes(n, _rng(3, 0))
    q = query_boxes(m, 0.01, _rng(3, 1))
    return Workload("clustered_boxes", BOXES, b, 30, QBOXES, q)


def clustered_rays(n: int = 1 << 24, m: int = 1 << 20, segments: bool = False,
                   length: float = 0.002) -> Workload:
    """Rays and segments on the clustered boxes (the same 2^24 boxes as
    ``clustered``).  Rays (first hit): from origins uniform in [0,1)^3
    through a random point of a random box, [0, +inf).  Segments (all
    hits): from a random point of a random box, ``length`` long, uniform
    direction.  Both aim at the boxes, so most of them meet some."""
    b = clustered_boxes(n, _rng(3, 0))
    q = clustered_ray_queries(b, m, segments, length)
    name = "clustered_segments" if segments else "clustered_rays"
    return Workload(name, BOXES, b, 30, RAYS, q, {"length": length} if segments else {})


def clustered_ray_queries(boxes: np.ndarray, m: int, segments: bool,
                          length: float = 0.002) -> np.ndarray:
    """The queries of ``clustered_rays`` for the given boxes."""
    rng = _rng(3, 3 if segments else 4)
    p = points_in_boxes(boxes, m, rng)
    return segments_from(p, length, rng) if segments else rays_toward(p, rng)


def batched_scene_sizes(S: int = 4096, lo: int = 32, hi: int = 65536,
                        rng: np.random.Generator | None = None) -> np.ndarray:
    """Scene sizes floor(exp(U(ln lo, ln hi)))."""
    rng = rng if rng is not None else _rng(4, 2)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=S))
                    ).astype(np.int64)


def batched(S: int = 4096, m_per: int = 64, lo: int = 32, hi: int = 65536):
    """Many independent uniform point sets (each in its own [0,1)^3), 63-bit
    codes, m_per spheres of radius 0.05 per set.  Returns
    (points_concat, seg_offsets[S+1], spheres_concat, qseg_offsets[S+1])."""
    sizes = batched_scene_sizes(S, lo, hi)
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    pts = uniform_points(int(off[-1]), _rng(4, 0))
    q = spheres(uniform_points(S * m_per, _rng(4, 1)), np.float32(0.05))
    qoff = np.arange(S + 1, dtype=np.int64) * m_per
    return pts, off, q, qoff


def serving_trace(rate: float = 2000.0, seconds: float = 30.0,
                  lo: float = 1e3, hi: float = 4e6, seed_stream: int = 2):
    """Poisson arrival times and request sizes for the serving stream."""
    rng = _rng(5, seed_stream)
    t, times = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        times.append(t)
    times = np.asarray(times)
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi),
                                        size=times.size))).astype(np.int64)
    return times, sizes


def serving_request(k: int, n: int, m: int = 10000) -> Workload:
    """Request k of the serving stream: n uniform points (63-bit codes) and
    m spheres with about 8 expected neighbours."""
    rng = np.random.default_rng([5, 10, k])
    p = uniform_points(n, rng)
    r = neighbour_radius(n, 8.0)
    q = spheres(uniform_points(m, rng), np.float32(r))
    return Workload(f"serving_{k}", POINTS, p, 63, SPHERES, q, {"radius": r})


def by_name(name: str, scale: float = 1.0) -> Workload:
    """Single-scene workloads by name; ``scale`` shrinks n and m (same
    distribution, same seeds) for tests that need the oracle to be quick."""
    if name == "small_points":
        return small_points(max(1, int(16384 * scale)), max(1, int(1024 * scale)))
    if name == "large_points":
        return large_points(max(1, int((1 << 23) * scale)),
                            max(1, int((1 << 20) * scale)))
    if name == "clustered_boxes":
        return clustered(max(1, int((1 << 24) * scale)),
                         max(1, int((1 << 20) * scale)))
    if name in ("clustered_rays", "clustered_segments"):
        return clustered_rays(max(1, int((1 << 24) * scale)), max(1, int((1 << 20) * scale)),
                              segments=name == "clustered_segments")
    raise KeyError(name)


SERVING_POOL_POINTS = 1 << 24      # rows of the serving point pool (>= the largest request)
SERVING_POOL_CENTRES = 1 << 20


def serving_pools(points: int = SERVING_POOL_POINTS, centres: int = SERVING_POOL_CENTRES):
    """Payload pools of the serving stream: float32 [points,3] and
    [centres,3], uniform in [0,1)^3.  A request's points are a row range of
    the first, its sphere centres a row range of the second."""
    rng = _rng(5, 20)
    return (rng.random((points, 3), dtype=np.float32),
            rng.random((centres, 3), dtype=np.float32))


def serving_plan(rate: float = 2000.0, seconds: float = 30.0, m: int = 10000,
                 lo: float = 1e3, hi: float = 4e6, neighbours: float = 8.0,
                 pool_points: int = SERVING_POOL_POINTS,
                 pool_centres: int = SERVING_POOL_CENTRES, seed_stream: int = 2) -> dict:
    """The serving stream as arrays: Poisson arrival times (s), sizes n
    (log-uniform in [lo, hi]), query counts m, payload row offsets into the
    pools (point offsets a multiple of 4 rows, so every request's points
    start 16-byte aligned) and the sphere radius for about ``neighbours``
    expected neighbours."""
    times, sizes = serving_trace(rate, seconds, lo, hi, seed_stream)
    sizes = np.minimum(sizes, pool_points)
    rng = _rng(5, 30 + seed_stream)
    p_off = rng.integers(0, (pool_points - sizes) // 4 + 1) * 4
    q_off = rng.integers(0, pool_centres - m + 1, size=sizes.size)
    radius = np.array([neighbour_radius(int(n), neighbours) if n > 0 else 0.0 for n in sizes],
                      np.float32)
    return {"arrival": times, "n": sizes.astype(np.int64), "m": np.full(sizes.size, m, np.int64),
            "p_off": p_off.astype(np.int64), "q_off": q_off.astype(np.int64), "radius": radius}
