"""Pins of the oracle's ray / segment queries (Sec. 1 names "all primitives a
ray meets" as a range search; Alg. 1 answers it with the slab predicate).

The predicate is pinned to exact rational arithmetic on dyadic inputs (where
every binary32 operation of the slab test is exact, so the float result must
equal the mathematical one), to hand-worked cases, and to its monotonicity
under box inclusion (what makes Alg. 1 exact for it).  The queries are
pinned to brute force: all hits in leaf order, and the first hit as the
smallest entry parameter with ties to the smallest leaf position."""

from fractions import Fraction

import numpy as np
import pytest

import oracle

INF = float("inf")


def ray(o, d, tmin=0.0, tmax=INF):
    return np.array([o[0], o[1], o[2], tmin, d[0], d[1], d[2], tmax], np.float32)


def exact_slab(box, q):
    """{t in [tmin, tmax] : lo <= o + t*d <= hi} in exact rationals:
    (hit, smallest such t)."""
    lo_t = None if q[3] == -INF else Fraction(float(q[3]))
    hi_t = None if q[7] == INF else Fraction(float(q[7]))
    for a in range(3):
        o, d = Fraction(float(q[a])), Fraction(float(q[4 + a]))
        lo, hi = Fraction(float(box[a])), Fraction(float(box[3 + a]))
        if d == 0:
            if not (lo <= o <= hi):
                return False, None
            continue
        t1, t2 = (lo - o) / d, (hi - o) / d
        a_lo, a_hi = min(t1, t2), max(t1, t2)
        lo_t = a_lo if lo_t is None else max(lo_t, a_lo)
        hi_t = a_hi if hi_t is None else min(hi_t, a_hi)
    if lo_t is not None and hi_t is not None and lo_t > hi_t:
        return False, None
    return True, (-INF if lo_t is None else lo_t)


def test_predicate_equals_exact_arithmetic_on_dyadic_inputs():
    """Coordinates on a 1/8 grid in [-4, 4] and direction components that are
    0 or powers of two: 1/d, the differences and the products are exact in
    binary32, so hit and entry parameter must equal the rational ones."""
    rng = np.random.default_rng([31, 0])
    dirs = np.array([0.0, 0.5, 1.0, 2.0, 4.0, -0.5, -1.0, -2.0, -4.0])
    hits = 0
    for _ in range(4000):
        lo = rng.integers(-32, 32, 3) / 8.0
        hi = lo + rng.integers(0, 16, 3) / 8.0
        box = np.concatenate([lo, hi]).astype(np.float32)
        if rng.random() < 0.5:   # anywhere, any direction
            o = rng.integers(-40, 40, 3) / 8.0
            d = rng.choice(dirs, 3)
        else:                    # through a grid point of the box (or near it) at t = k
            p = lo + np.floor(rng.random(3) * ((hi - lo) * 8 + 1)) / 8.0 + rng.integers(-1, 2, 3) / 8.0
            d = rng.choice(dirs, 3)
            o = p - rng.choice([0.25, 0.5, 1.0, 2.0]) * d
        tmin = rng.choice([-INF, 0.0, 0.25, 1.0])
        tmax = rng.choice([INF, 1.0, 1.5, 0.125, tmin if np.isfinite(tmin) else 0.0])
        q = ray(o, d, tmin, tmax)
        got, e = oracle.pred_ray(box, q)
        want, we = exact_slab(box, q)
        assert got == want, (box, q)
        if want:
            hits += 1
            assert Fraction(e) == we if we != -INF else e == -INF, (box, q, e, we)
    assert 400 < hits < 3600   # both outcomes well represented


def test_hand_worked_cases():
    box = np.array([0, 0, 0, 1, 1, 1], np.float32)
    # along +x through the middle: enters at t = 1 (x = 0), leaves at t = 2
    assert oracle.pred_ray(box, ray((-1, 0.5, 0.5), (1, 0, 0))) == (True, 1.0)
    # the same line backwards from x = 3: enters at x = 1, t = 2
    assert oracle.pred_ray(box, ray((3, 0.5, 0.5), (-1, 0, 0))) == (True, 2.0)
    # grazing the face y = 1 (closed box): hit; just above it: miss
    assert oracle.pred_ray(box, ray((-1, 1, 0.5), (1, 0, 0)))[0]
    assert not oracle.pred_ray(box, ray((-1, np.nextafter(np.float32(1), np.float32(2)), 0.5),
                                        (1, 0, 0)))[0]
    # a segment that ends exactly on the face x = 0 touches it; one that ends
    # just before does not
    assert oracle.pred_ray(box, ray((-1, 0.5, 0.5), (1, 0, 0), 0.0, 1.0)) == (True, 1.0)
    assert not oracle.pred_ray(box, ray((-1, 0.5, 0.5), (1, 0, 0), 0.0,
                                        np.nextafter(np.float32(1), np.float32(0))))[0]
    # starting inside: the entry parameter is tmin
    assert oracle.pred_ray(box, ray((0.5, 0.5, 0.5), (1, 2, 3), 0.125, INF)) == (True, 0.125)
    # pointing away, and an empty parameter range
    assert not oracle.pred_ray(box, ray((2, 0.5, 0.5), (1, 0, 0)))[0]
    assert not oracle.pred_ray(box, ray((0.5, 0.5, 0.5), (1, 0, 0), 1.0, 0.5))[0]
    # diagonal through a corner: (-1,-1,-1) + t(1,1,1) meets the box on t in [1, 2]
    assert oracle.pred_ray(box, ray((-1, -1, -1), (1, 1, 1))) == (True, 1.0)
    # a direction component whose reciprocal overflows counts as parallel
    tiny = np.float32(1e-40)
    assert oracle.pred_ray(box, ray((0.5, -1, 0.5), (tiny, 1, 0)))[0]
    assert not oracle.pred_ray(box, ray((2.0, -1, 0.5), (tiny, 1, 0)))[0]
    # a point (degenerate box) is met only by rays through it
    pt = np.array([0.5, 0.5, 0.5, 0.5, 0.5, 0.5], np.float32)
    assert oracle.pred_ray(pt, ray((0, 0.5, 0.5), (1, 0, 0))) == (True, 0.5)
    assert not oracle.pred_ray(pt, ray((0, 0.5, 0.25), (1, 0, 0)))[0]


def test_predicate_is_monotone_under_box_inclusion():
    """For B inside B': a ray that meets B meets B', and enters B' no later:
    what lets Alg. 1 prune a subtree by its box, exactly, in binary32."""
    rng = np.random.default_rng([31, 1])
    checked = 0
    for _ in range(20000):
        c = rng.random(3).astype(np.float32)
        s = (rng.random(3) * 0.2).astype(np.float32)
        inner = np.concatenate([c - s, c + s]).astype(np.float32)
        grow = (rng.random(6) * rng.choice([0.0, 1e-7, 1e-3, 0.1], 6)).astype(np.float32)
        outer = np.concatenate([inner[:3] - grow[:3], inner[3:] + grow[3:]]).astype(np.float32)
        assert np.all(outer[:3] <= inner[:3]) and np.all(outer[3:] >= inner[3:])
        o = (rng.random(3) * 3 - 1).astype(np.float32)
        # aimed at a point near the inner box, some components tiny or zero
        aim = c + (rng.random(3) * 2 - 1) * s * 1.2 - o
        d = (aim * rng.choice([1.0, 1.0, 1e-6, 0.0], 3)).astype(np.float32)
        q = ray(o, d, rng.choice([0.0, -INF]), rng.choice([INF, 1.0, 0.3]))
        hi_, ei = oracle.pred_ray(inner, q)
        ho, eo = oracle.pred_ray(outer, q)
        if hi_:
            checked += 1
            assert ho and eo <= ei, (inner, outer, q, ei, eo)
    assert checked > 1500


def boxes_on_a_line():
    """Ten boxes [k, k+0.5] x [0, 0.5]^2, k = 0..9."""
    b = np.zeros((10, 6), np.float32)
    for k in range(10):
        b[k] = [k, 0, 0, k + 0.5, 0.5, 0.5]
    return b


def test_worked_queries_on_boxes_along_a_line():
    prims = boxes_on_a_line()
    t = oracle.build(oracle.BOXES, prims, 30)
    rays = np.stack([ray((-1, 0.25, 0.25), (1, 0, 0)),          # first hit box 0 at t = 1
                     ray((20, 0.25, 0.25), (-1, 0, 0)),         # first hit box 9 at t = 10.5
                     ray((-1, 0.25, 0.25), (5.75, 0, 0), 0.0, 1.0),   # segment to x = 4.75
                     ray((0, 1, 0.25), (1, 0, 0)),              # above every box: no hit
                     ray((4.75, 0.25, 0.25), (0, 0, 1))])       # in the gap between 4 and 5
    hit, tt, _ = oracle.ray_first_traverse(rays, t)
    assert hit.tolist() == [0, 9, 0, -1, -1]
    assert tt[0] == 1.0 and tt[1] == 10.5 and tt[2] == np.float32(1 / 5.75)
    off, idx, _ = oracle.query_traverse(oracle.RAYS, rays, t)
    assert np.diff(off).tolist() == [10, 10, 5, 0, 0]
    # the x-extent orders the Morton codes here, so leaf order is box order
    assert idx[off[2]:off[3]].tolist() == [0, 1, 2, 3, 4]
    assert sorted(idx[off[0]:off[1]].tolist()) == list(range(10))


def test_first_hit_ties_go_to_the_first_leaf():
    """Two copies of a box (same code, so leaf order = input order): the ray
    enters both at the same t and the first leaf wins."""
    prims = np.array([[5, 5, 5, 6, 6, 6], [0, 0, 0, 1, 1, 1], [0, 0, 0, 1, 1, 1],
                      [2, 2, 2, 3, 3, 3]], np.float32)
    t = oracle.build(oracle.BOXES, prims, 30)
    pos = {int(p): k for k, p in enumerate(t.perm)}
    assert pos[1] < pos[2]
    rays = np.stack([ray((-1, 0.5, 0.5), (1, 0, 0))])
    hit, tt, _ = oracle.ray_first_traverse(rays, t)
    assert hit.tolist() == [1] and tt[0] == 1.0
    assert oracle.ray_first_brute(rays, 0, oracle.BOXES, prims, t.perm) == (1, 1.0)


def random_rays(m, rng, segment):
    o = rng.random((m, 3)).astype(np.float32)
    d = rng.standard_normal((m, 3)).astype(np.float32)
    if segment:
        d *= np.float32(0.05)
        return np.concatenate([o, np.zeros((m, 1), np.float32), d, np.ones((m, 1), np.float32)], 1)
    return np.concatenate([o, np.zeros((m, 1), np.float32), d, np.full((m, 1), np.inf, np.float32)], 1)


@pytest.mark.parametrize("kind", [oracle.BOXES, oracle.POINTS])
def test_alg1_equals_brute_force_for_segments_and_rays(kind):
    import workloads
    rng = np.random.default_rng([31, 2 + kind])
    n = 3000
    if kind == oracle.BOXES:   # boxes of side 0.005 .. 0.06: a few per ray
        c = rng.random((n, 3))
        h = rng.uniform(0.0025, 0.03, (n, 3))
        prims = np.concatenate([c - h, c + h], 1).astype(np.float32)
    else:
        prims = workloads.uniform_points(n, rng)
    t = oracle.build(kind, prims, 30)
    for segment in (True, False):
        rays = random_rays(200, rng, segment)
        if kind == oracle.POINTS:
            # rays aimed exactly at a primitive (from an origin on an axis
            # line through it) so that points are met
            k = rng.integers(0, n, 200)
            rays[:, 0] = prims[k, 0] - 1.0
            rays[:, 1:3] = prims[k, 1:3]
            rays[:, 4:7] = [1.0, 0.0, 0.0]
            rays[:, 7] = np.inf if not segment else 2.0
        off, idx, vis = oracle.query_traverse(oracle.RAYS, rays, t)
        total = 0
        for j in range(rays.shape[0]):
            want = oracle.query_brute(oracle.RAYS, rays, j, kind, prims, t.perm)
            assert np.array_equal(idx[off[j]:off[j + 1]], want), j
            total += want.size
        assert total > 0
        fh, ft, fvis = oracle.ray_first_traverse(rays, t)
        for j in range(rays.shape[0]):
            h, e = oracle.ray_first_brute(rays, j, kind, prims, t.perm)
            assert fh[j] == h and (ft[j] == e or (h < 0 and np.isinf(ft[j]))), j
            if h >= 0:   # the first hit is one of the hits, with the least entry
                row = idx[off[j]:off[j + 1]]
                assert h in row
        assert fvis <= vis   # pruning only removes visits


def test_first_hit_against_float64_geometry():
    """Away from ties, the first hit is the primitive whose box the ray
    enters first, computed in float64 from the same binary32 inputs."""
    rng = np.random.default_rng([31, 9])
    c = rng.random((2000, 3))
    h = rng.uniform(0.0025, 0.03, (2000, 3))
    prims = np.concatenate([c - h, c + h], 1).astype(np.float32)
    t = oracle.build(oracle.BOXES, prims, 30)
    rays = random_rays(300, rng, segment=False)
    fh, ft, _ = oracle.ray_first_traverse(rays, t)
    P = prims.astype(np.float64)
    agree = 0
    for j in range(rays.shape[0]):
        q = rays[j].astype(np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (P[:, :3] - q[:3]) / q[4:7]
            t2 = (P[:, 3:] - q[:3]) / q[4:7]
        tn = np.maximum(np.minimum(t1, t2).max(1), q[3])
        tf = np.minimum(np.maximum(t1, t2).min(1), q[7])
        ok = tn <= tf
        if not ok.any():
            assert fh[j] == -1
            continue
        order = np.argsort(np.where(ok, tn, np.inf), kind="stable")
        best, second = tn[order[0]], tn[order[1]] if ok.sum() > 1 else np.inf
        if second - best > 1e-5 * max(1.0, abs(best)):   # no near tie: unambiguous
            assert fh[j] == order[0], j
            assert abs(ft[j] - best) <= 1e-6 * max(1.0, abs(best))
            agree += 1
    assert agree > 50
