/*
 * Plain CPU oracle for the rope-LBVH of Prokopenko & Lebrun-Grandie,
 * "Revising Apetrei's bounding volume hierarchy construction algorithm to
 * allow stackless traversal" (arXiv 2402.00665).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may include, link
 * or call this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark use it.  It shares no code with the HIP kernels.
 *
 * The oracle computes each result from its plain definition, with algorithms
 * that differ from the paper's bottom-up pass on purpose:
 *   - scene box by a linear min/max scan;
 *   - Morton codes by bit-by-bit interleaving (Sec. 3.1, step 1);
 *   - sort by the C library's qsort on (code, index) pairs (Sec. 3.1, step 2);
 *   - the binary radix tree top-down from the split definition (Sec. 3.1:
 *     a node over [i,j] splits where adjacent keys differ in the highest bit,
 *     children take indices gamma and gamma+1);
 *   - skip-connections (ropes) by an explicit depth-first walk, the extra
 *     pass the paper's method removes (Sec. 2: a rope points to the right
 *     child of the last ancestor whose left subtree holds the node; the
 *     right-most path points to the sentinel);
 *   - each internal box as the min/max over all leaf boxes of its range;
 *   - range queries by brute force over all primitives and, separately, by
 *     the stackless walk of Alg. 1 on the oracle's own tree.
 *
 * Floating point: IEEE binary32, round to nearest even, no contraction
 * (compile with -ffp-contract=off), no flush of denormals.
 *
 * Threads: the loops whose iterations are independent (scene box, Morton
 * codes, delta*, boxes, one Alg. 1 walk per query) carry OpenMP pragmas so
 * that the benchmark can also time the oracle on several host cores
 * (orc_threads).  Each iteration computes exactly what it computes alone,
 * and min/max are exact, so every result is bit-identical for any thread
 * count; the sort, the top-down split recursion and the rope walk stay
 * sequential.
 *
 * Conventions where the paper is silent or garbled (each is a reading):
 *   - delta* is a dissimilarity: the rank of the highest differing bit of the
 *     two adjacent augmented keys (code, sorted position), with
 *     delta*(-1) = delta*(n-1) = +inf (stored as 255).  Codes that differ
 *     rank as 64 + bit, equal codes rank by the bit of i xor (i+1).
 *   - Node ids are unified: internal k -> k, leaf k -> n-1+k, sentinel -1.
 *     Node 0 is the root; for n = 1 it is leaf 0.
 *   - Morton: scene box = union of primitive boxes; centroid of a box is
 *     (lo+hi)*0.5f; b bits per axis (b = 10 for 30-bit codes, b = 21 for
 *     63-bit); scale = 2^b / extent (correctly rounded), 0 for a flat axis;
 *     t = (c - lo) * scale; q = 0 if !(t > 0), 2^b-1 if t >= 2^b-1, else
 *     floor(t); x takes the most significant bit of each 3-bit group.
 *   - Sphere predicate: per axis d = max(max(lo - c, c - hi), 0);
 *     hit iff (dx*dx + dy*dy) + dz*dz <= r*r.  Box predicate: closed-interval
 *     overlap on every axis.
 *   - Ray / segment predicate (Sec. 1 names the primitives a ray meets as a
 *     range search): a query is o.xyz, tmin, d.xyz, tmax, the points
 *     o + t*d with tmin <= t <= tmax (a segment from a to b is o = a,
 *     d = b - a, [0, 1]; a ray has tmax = +inf).  Closed slab test in
 *     binary32: per axis, inv = 1/d (correctly rounded); if d = 0 or inv
 *     overflows, the axis passes iff lo <= o <= hi; else t1 = (lo - o)*inv,
 *     t2 = (hi - o)*inv.  enter = max(tmin, min(t1,t2) of each axis),
 *     exit = min(tmax, max(t1,t2) of each axis), hit iff enter <= exit.
 *     First hit of a ray: among the primitives it meets, the smallest
 *     enter, ties to the smallest leaf position (Morton order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_POINTS 0
#define ORC_BOXES 1
#define ORC_SPHERES 0
#define ORC_QBOXES 1
#define ORC_RAYS 2

/* ---------------------------------------------------------------- boxes */

static void prim_box(int kind, const float *prims, int64_t i, float box[6])
{
    if (kind == ORC_POINTS) {
        const float *p = prims + 3 * i;
        box[0] = p[0]; box[1] = p[1]; box[2] = p[2];
        box[3] = p[0]; box[4] = p[1]; box[5] = p[2];
    } else {
        const float *b = prims + 6 * i;
        for (int a = 0; a < 6; ++a) box[a] = b[a];
    }
}

static float fmin_(float a, float b) { return b < a ? b : a; }
static float fmax_(float a, float b) { return b > a ? b : a; }

/* Number of host threads the parallel loops use (1 = plain sequential). */
void orc_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}

/* Scene box: componentwise min of lo and max of hi over all primitives
 * (each thread folds its share, then the shares are folded together: for
 * finite coordinates min and max are exact, so the order does not matter). */
int orc_scene_box(int kind, const float *prims, int64_t n, float out[6])
{
    if (n <= 0) return -1;
    prim_box(kind, prims, 0, out);
#pragma omp parallel
    {
        float part[6], box[6];
        memcpy(part, out, sizeof(part));
#pragma omp for schedule(static)
        for (int64_t i = 1; i < n; ++i) {
            prim_box(kind, prims, i, box);
            for (int a = 0; a < 3; ++a) {
                part[a] = fmin_(part[a], box[a]);
                part[3 + a] = fmax_(part[3 + a], box[3 + a]);
            }
        }
#pragma omp critical
        for (int a = 0; a < 3; ++a) {
            out[a] = fmin_(out[a], part[a]);
            out[3 + a] = fmax_(out[3 + a], part[3 + a]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------- Morton */

static uint32_t quantize(float t, float maxq)
{
    if (!(t > 0.0f)) return 0u;
    if (t >= maxq) return (uint32_t)maxq;
    return (uint32_t)t; /* truncation == floor for t > 0 */
}

/* Bit-by-bit interleave: bit k of x goes to 3k+2, of y to 3k+1, of z to 3k. */
static uint64_t interleave(uint32_t qx, uint32_t qy, uint32_t qz, int b)
{
    uint64_t code = 0;
    for (int k = 0; k < b; ++k) {
        code |= (uint64_t)((qx >> k) & 1u) << (3 * k + 2);
        code |= (uint64_t)((qy >> k) & 1u) << (3 * k + 1);
        code |= (uint64_t)((qz >> k) & 1u) << (3 * k);
    }
    return code;
}

/* Per-axis quantisation scale, 2^b / extent in binary32 (0 for a flat axis). */
void orc_scales(const float scene[6], int bits, float scale[3])
{
    int b = bits / 3;
    float two_b = (float)(1u << b);
    for (int a = 0; a < 3; ++a) {
        float ext = scene[3 + a] - scene[a];
        scale[a] = ext > 0.0f ? two_b / ext : 0.0f;
    }
}

/* Morton code of every primitive's centroid, in input order. */
int orc_morton(int kind, const float *prims, int64_t n, int bits,
               const float scene[6], uint64_t *codes)
{
    if (bits != 30 && bits != 63) return -1;
    int b = bits / 3;
    float maxq = (float)((1u << b) - 1u);
    float scale[3];
    orc_scales(scene, bits, scale);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float box[6];
        prim_box(kind, prims, i, box);
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            float c = kind == ORC_POINTS ? box[a] : (box[a] + box[3 + a]) * 0.5f;
            float t = (c - scene[a]) * scale[a];
            q[a] = quantize(t, maxq);
        }
        codes[i] = interleave(q[0], q[1], q[2], b);
    }
    return 0;
}

/* --------------------------------------------------------------- sort */

typedef struct { uint64_t code; int64_t idx; } pair_t;

static int cmp_pair(const void *x, const void *y)
{
    const pair_t *a = (const pair_t *)x, *b = (const pair_t *)y;
    if (a->code != b->code) return a->code < b->code ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Stable ascending sort of codes: sorting the distinct (code, index) pairs
 * lexicographically keeps equal codes in input order. */
int orc_sort(const uint64_t *codes, int64_t n, uint64_t *sorted, int32_t *perm)
{
    pair_t *pr = (pair_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(pair_t));
    if (!pr) return -2;
    for (int64_t i = 0; i < n; ++i) { pr[i].code = codes[i]; pr[i].idx = i; }
    qsort(pr, (size_t)n, sizeof(pair_t), cmp_pair);
    for (int64_t i = 0; i < n; ++i) { sorted[i] = pr[i].code; perm[i] = (int32_t)pr[i].idx; }
    free(pr);
    return 0;
}

/* ------------------------------------------------------------- delta* */

static int highest_bit(uint64_t x)
{
    int b = -1;
    while (x) { x >>= 1; ++b; }
    return b;
}

/* delta*(i) for 0 <= i < n-1 (Sec. 3.1 and Sec. 3.2: XOR dissimilarity,
 * keys augmented with their index when codes are equal). */
int orc_delta(const uint64_t *sorted, int64_t n, uint8_t *delta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n - 1; ++i) {
        uint64_t x = sorted[i] ^ sorted[i + 1];
        if (x) delta[i] = (uint8_t)(64 + highest_bit(x));
        else delta[i] = (uint8_t)highest_bit((uint64_t)i ^ (uint64_t)(i + 1));
    }
    return 0;
}

/* ------------------------------------------------------ top-down tree */

/* Karras binary radix tree, top-down from the split definition.
 * left/right: [n-1] unified child ids; rlo/rhi: [n-1] leaf range of each
 * internal node.  Self-checks: returns -3 if an internal index would be
 * assigned twice and -4 if the highest-ranked boundary of a range is not
 * unique (neither can happen for distinct augmented keys). */
int orc_topdown(const uint8_t *delta, int64_t n, int32_t *left, int32_t *right,
                int32_t *rlo, int32_t *rhi)
{
    if (n < 2) return 0;
    int64_t ni = n - 1;
    for (int64_t k = 0; k < ni; ++k) { left[k] = right[k] = -2; rlo[k] = rhi[k] = -1; }
    int32_t *stack = (int32_t *)malloc((size_t)ni * sizeof(int32_t));
    if (!stack) return -2;
    int64_t sp = 0;
    rlo[0] = 0; rhi[0] = (int32_t)(n - 1);
    stack[sp++] = 0;
    while (sp > 0) {
        int32_t id = stack[--sp];
        int32_t i = rlo[id], j = rhi[id];
        int32_t g = i, ties = 0;
        for (int32_t k = i + 1; k < j; ++k) {
            if (delta[k] > delta[g]) { g = k; ties = 0; }
            else if (delta[k] == delta[g]) ++ties;
        }
        if (ties) { free(stack); return -4; } /* split must be unique */
        /* children [i, g] and [g+1, j] take indices g and g+1 */
        if (g == i) {
            left[id] = (int32_t)(ni + g);
        } else {
            if (rlo[g] != -1) { free(stack); return -3; }
            left[id] = g; rlo[g] = i; rhi[g] = g;
            stack[sp++] = g;
        }
        if (g + 1 == j) {
            right[id] = (int32_t)(ni + g + 1);
        } else {
            if (rlo[g + 1] != -1) { free(stack); return -3; }
            right[id] = g + 1; rlo[g + 1] = g + 1; rhi[g + 1] = j;
            stack[sp++] = g + 1;
        }
    }
    free(stack);
    return 0;
}

/* ---------------------------------------------------------------- ropes */

/* Explicit depth-first walk: rope(root) = sentinel; for an internal node N
 * with children A (left) and B (right): rope(A) = B, rope(B) = rope(N). */
int orc_ropes(const int32_t *left, const int32_t *right, int64_t n, int32_t *rope)
{
    if (n <= 0) return 0;
    int64_t total = 2 * n - 1, ni = n - 1;
    int32_t *st_node = (int32_t *)malloc((size_t)total * sizeof(int32_t));
    int32_t *st_rope = (int32_t *)malloc((size_t)total * sizeof(int32_t));
    if (!st_node || !st_rope) { free(st_node); free(st_rope); return -2; }
    int64_t sp = 0;
    st_node[sp] = 0; st_rope[sp] = -1; ++sp;
    while (sp > 0) {
        --sp;
        int32_t nd = st_node[sp], r = st_rope[sp];
        rope[nd] = r;
        if (nd < ni) {
            st_node[sp] = right[nd]; st_rope[sp] = r; ++sp;
            st_node[sp] = left[nd]; st_rope[sp] = right[nd]; ++sp;
        }
    }
    free(st_node); free(st_rope);
    return 0;
}

/* ---------------------------------------------------------------- boxes */

/* Leaf k holds the box of primitive perm[k]; an internal node holds the
 * componentwise min/max over the boxes of all leaves in its range. */
int orc_aabbs(int kind, const float *prims, const int32_t *perm,
              const int32_t *rlo, const int32_t *rhi, int64_t n, float *aabb)
{
    if (n <= 0) return 0;
    int64_t ni = n - 1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) prim_box(kind, prims, perm[k], aabb + 6 * (ni + k));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t id = 0; id < ni; ++id) {
        float *dst = aabb + 6 * id;
        const float *first = aabb + 6 * (ni + rlo[id]);
        for (int a = 0; a < 6; ++a) dst[a] = first[a];
        for (int32_t k = rlo[id] + 1; k <= rhi[id]; ++k) {
            const float *lb = aabb + 6 * (ni + k);
            for (int a = 0; a < 3; ++a) {
                dst[a] = fmin_(dst[a], lb[a]);
                dst[3 + a] = fmax_(dst[3 + a], lb[3 + a]);
            }
        }
    }
    return 0;
}

/* ----------------------------------------------------------- full build */

/* Everything the build produces.  Arrays are caller-allocated:
 * scene[6], codes[n] (input order), sorted[n], perm[n], delta[n-1],
 * left[n-1], right[n-1], rlo[n-1], rhi[n-1], rope[2n-1], aabb[(2n-1)*6]. */
int orc_build(int kind, const float *prims, int64_t n, int bits,
              float *scene, uint64_t *codes, uint64_t *sorted, int32_t *perm,
              uint8_t *delta, int32_t *left, int32_t *right, int32_t *rlo,
              int32_t *rhi, int32_t *rope, float *aabb)
{
    int rc;
    if (n <= 0) return 0;
    if ((rc = orc_scene_box(kind, prims, n, scene))) return rc;
    if ((rc = orc_morton(kind, prims, n, bits, scene, codes))) return rc;
    if ((rc = orc_sort(codes, n, sorted, perm))) return rc;
    if ((rc = orc_delta(sorted, n, delta))) return rc;
    if ((rc = orc_topdown(delta, n, left, right, rlo, rhi))) return rc;
    if ((rc = orc_ropes(left, right, n, rope))) return rc;
    return orc_aabbs(kind, prims, perm, rlo, rhi, n, aabb);
}

/* ------------------------------------------------------------- queries */

int orc_pred_sphere(const float box[6], const float q[4])
{
    float d[3];
    for (int a = 0; a < 3; ++a) {
        float below = box[a] - q[a];
        float above = q[a] - box[3 + a];
        float m = below > above ? below : above;
        d[a] = m > 0.0f ? m : 0.0f;
    }
    float d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 <= q[3] * q[3];
}

int orc_pred_box(const float box[6], const float q[6])
{
    for (int a = 0; a < 3; ++a)
        if (!(q[a] <= box[3 + a] && box[a] <= q[3 + a])) return 0;
    return 1;
}

/* Ray / segment q = (o.xyz, tmin, d.xyz, tmax) against a box: 1 if some
 * t in [tmin, tmax] has o + t*d in the closed box; then *enter (if
 * non-NULL) receives the entry parameter, the largest lower end of the
 * per-axis slab intervals and tmin. */
int orc_pred_ray(const float box[6], const float q[8], float *enter)
{
    float t_in = q[3], t_out = q[7];
    for (int a = 0; a < 3; ++a) {
        const float o = q[a], d = q[4 + a];
        const float inv = 1.0f / d;
        if (d == 0.0f || inv == INFINITY || inv == -INFINITY) {
            /* parallel to the slab: in it for every t, or never */
            if (!(box[a] <= o && o <= box[3 + a])) return 0;
            continue;
        }
        const float t1 = (box[a] - o) * inv;
        const float t2 = (box[3 + a] - o) * inv;
        const float near_ = t1 < t2 ? t1 : t2;
        const float far_ = t1 < t2 ? t2 : t1;
        if (near_ > t_in) t_in = near_;
        if (far_ < t_out) t_out = far_;
    }
    if (!(t_in <= t_out)) return 0;
    if (enter) *enter = t_in;
    return 1;
}

static int pred(int qkind, const float *box, const float *q)
{
    if (qkind == ORC_RAYS) return orc_pred_ray(box, q, NULL);
    return qkind == ORC_SPHERES ? orc_pred_sphere(box, q) : orc_pred_box(box, q);
}

static int query_width(int qkind) { return qkind == ORC_SPHERES ? 4 : (qkind == ORC_QBOXES ? 6 : 8); }

/* Brute force for query j: every primitive whose box satisfies the
 * predicate, listed in ascending leaf position (perm is the sorted order).
 * Writes at most cap ids to out; returns the number of hits. */
int64_t orc_query_brute(int qkind, const float *queries, int64_t j, int kind,
                        const float *prims, const int32_t *perm, int64_t n,
                        int32_t *out, int64_t cap)
{
    int qw = query_width(qkind);
    const float *q = queries + qw * j;
    float box[6];
    int64_t h = 0;
    for (int64_t k = 0; k < n; ++k) {
        prim_box(kind, prims, perm[k], box);
        if (pred(qkind, box, q)) {
            if (h < cap) out[h] = perm[k];
            ++h;
        }
    }
    return h;
}

/* Alg. 1 for one query from the root: a passing internal node sends the
 * walk to its left child, a passing leaf is reported and the walk follows
 * its rope, a failing node sends it along its rope, the sentinel ends it.
 * Writes the hits (primitive ids, in traversal order) to out if non-NULL;
 * returns the number of hits and adds the node visits to *visits. */
static int64_t walk_one(int qkind, const float *q, int64_t n, const int32_t *left,
                        const int32_t *rope, const float *aabb, const int32_t *perm,
                        int32_t *out, int64_t *visits)
{
    int64_t ni = n - 1, hits = 0, nvis = 0;
    if (n > 0) {
        int32_t node = 0; /* root */
        do {
            ++nvis;
            if (pred(qkind, aabb + 6 * (int64_t)node, q)) {
                if (node >= ni) {
                    if (out) out[hits] = perm[node - ni];
                    ++hits;
                    node = rope[node];
                } else {
                    node = left[node];
                }
            } else {
                node = rope[node];
            }
        } while (node != -1);
    }
    *visits += nvis;
    return hits;
}

/* Alg. 1 on the oracle tree for queries [0, m): offsets[m+1] receives the
 * CSR offsets (each query's hit count, then their running sum); visits, if
 * non-NULL, the total number of node visits.  Returns the total number of
 * hits.  The walks are independent (one per query). */
int64_t orc_query_traverse(int qkind, const float *queries, int64_t m, int64_t n,
                           const int32_t *left, const int32_t *rope,
                           const float *aabb, const int32_t *perm,
                           int64_t *offsets, int64_t *visits)
{
    int qw = query_width(qkind);
    int64_t nvis = 0;
    offsets[0] = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nvis)
    for (int64_t j = 0; j < m; ++j) {
        int64_t v = 0;
        offsets[j + 1] = walk_one(qkind, queries + qw * j, n, left, rope, aabb, perm, NULL, &v);
        nvis += v;
    }
    for (int64_t j = 0; j < m; ++j) offsets[j + 1] += offsets[j];
    if (visits) *visits = nvis;
    return offsets[m];
}

/* The hits of Alg. 1 for queries [0, m): query j's primitive ids, in
 * traversal order, into indices[offsets[j] .. offsets[j+1]) (offsets as
 * orc_query_traverse wrote them). */
int orc_query_fill(int qkind, const float *queries, int64_t m, int64_t n,
                   const int32_t *left, const int32_t *rope, const float *aabb,
                   const int32_t *perm, const int64_t *offsets, int32_t *indices)
{
    int qw = query_width(qkind);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < m; ++j) {
        int64_t v = 0;
        walk_one(qkind, queries + qw * j, n, left, rope, aabb, perm, indices + offsets[j], &v);
    }
    return 0;
}

/* ------------------------------------------------------ first hit (rays) */

/* First hit of ray j by brute force: every primitive in ascending leaf
 * position; keep the one with the smallest entry parameter (a later leaf
 * replaces it only if strictly smaller).  Returns the primitive id or -1;
 * *t receives its entry parameter (+inf if none). */
int32_t orc_ray_first_brute(const float *rays, int64_t j, int kind, const float *prims,
                            const int32_t *perm, int64_t n, float *t)
{
    const float *q = rays + 8 * j;
    float box[6], best = INFINITY, e;
    int32_t hit = -1;
    for (int64_t k = 0; k < n; ++k) {
        prim_box(kind, prims, perm[k], box);
        if (orc_pred_ray(box, q, &e) && (hit < 0 || e < best)) {
            hit = perm[k];
            best = e;
        }
    }
    *t = best;
    return hit;
}

/* First hit of one ray with Alg. 1 and pruning: a node is entered only if
 * the ray meets its box with an entry parameter below the best hit found
 * so far (any entry while none is found).  Boxes of a subtree contain the
 * boxes below them, so a pruned subtree holds no leaf that would win, and
 * Alg. 1 reaches leaves in ascending position, so on equal entries the
 * first leaf found stays. */
static int32_t first_walk(const float *q, int64_t n, const int32_t *left, const int32_t *rope,
                          const float *aabb, const int32_t *perm, float *t, int64_t *visits)
{
    int64_t ni = n - 1, nvis = 0;
    int32_t hit = -1;
    float best = INFINITY, e;
    if (n > 0) {
        int32_t node = 0;
        do {
            ++nvis;
            if (orc_pred_ray(aabb + 6 * (int64_t)node, q, &e) && (hit < 0 || e < best)) {
                if (node >= ni) {
                    hit = perm[node - ni];
                    best = e;
                    node = rope[node];
                } else {
                    node = left[node];
                }
            } else {
                node = rope[node];
            }
        } while (node != -1);
    }
    *t = best;
    *visits += nvis;
    return hit;
}

/* First hits of rays [0, m) on the oracle tree: hit[j] (primitive or -1),
 * t[j]; visits, if non-NULL, the total node visits.  One walk per ray. */
int orc_ray_first_traverse(const float *rays, int64_t m, int64_t n, const int32_t *left,
                           const int32_t *rope, const float *aabb, const int32_t *perm,
                           int32_t *hit, float *t, int64_t *visits)
{
    int64_t nvis = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nvis)
    for (int64_t j = 0; j < m; ++j) {
        int64_t v = 0;
        hit[j] = first_walk(rays + 8 * j, n, left, rope, aabb, perm, t + j, &v);
        nvis += v;
    }
    if (visits) *visits = nvis;
    return 0;
}
