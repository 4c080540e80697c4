// Query-side device code shared by the single-tree and batched query
// translation units: the two predicates (with their containment tests), the
// tree walker, the split and leaf-walk kernels and the CSR scan.
#pragma once
#pragma clang fp contract(off)

#include "lbvh_internal.hpp"

namespace lbvh {
namespace {

struct Sphere {
    static constexpr int kFloats = 4;   // x, y, z, r
    float cx, cy, cz, r, r2;
    __device__ void load(const float *q, int j)
    {
        const float4 v = reinterpret_cast<const float4 *>(q)[j];
        cx = v.x; cy = v.y; cz = v.z; r = v.w; r2 = v.w * v.w;
    }
    // a box around the query (only steers the schedule, never a result)
    __device__ void bounds(float lo[3], float hi[3]) const
    {
        lo[0] = cx - r; lo[1] = cy - r; lo[2] = cz - r;
        hi[0] = cx + r; hi[1] = cy + r; hi[2] = cz + r;
    }
    __device__ bool test(float4 lo, float4 hi) const
    {
        const float dx = fmaxf(fmaxf(lo.x - cx, cx - hi.x), 0.0f);
        const float dy = fmaxf(fmaxf(lo.y - cy, cy - hi.y), 0.0f);
        const float dz = fmaxf(fmaxf(lo.z - cz, cz - hi.z), 0.0f);
        return (dx * dx + dy * dy) + dz * dz <= r2;
    }
    // The box lies inside the ball: its farthest corner passes.  Every box
    // inside it then passes `test` too, also after rounding: each per-axis
    // term of `test` for an inner box is <= the corresponding far term here
    // (rounding is monotone), and squares and sums of non-negative terms
    // keep the order.
    __device__ bool contains(float4 lo, float4 hi) const
    {
        const float fx = fmaxf(cx - lo.x, hi.x - cx);
        const float fy = fmaxf(cy - lo.y, hi.y - cy);
        const float fz = fmaxf(cz - lo.z, hi.z - cz);
        return (fx * fx + fy * fy) + fz * fz <= r2;
    }
};

struct QBox {
    static constexpr int kFloats = 6;   // lo.xyz, hi.xyz
    float lx, ly, lz, hx, hy, hz;
    __device__ void load(const float *q, int j)
    {
        const float2 *p = reinterpret_cast<const float2 *>(q + 6 * (int64_t)j);
        const float2 a = p[0], b = p[1], c = p[2];
        lx = a.x; ly = a.y; lz = b.x; hx = b.y; hy = c.x; hz = c.y;
    }
    __device__ bool test(float4 lo, float4 hi) const
    {
        return lx <= hi.x && lo.x <= hx && ly <= hi.y && lo.y <= hy && lz <= hi.z && lo.z <= hz;
    }
    __device__ void bounds(float lo[3], float hi[3]) const
    {
        lo[0] = lx; lo[1] = ly; lo[2] = lz;
        hi[0] = hx; hi[1] = hy; hi[2] = hz;
    }
    // The box lies inside the query box, so every box inside it overlaps.
    __device__ bool contains(float4 lo, float4 hi) const
    {
        return lx <= lo.x && hi.x <= hx && ly <= lo.y && hi.y <= hy && lz <= lo.z && hi.z <= hz;
    }
};

// Ray or segment: the points o + t*d with tmin <= t <= tmax (a segment from
// a to b is o = a, d = b - a, [0, 1]; a ray has tmax = +inf).  Sec. 1 counts
// the primitives a ray meets among the range searches a BVH answers.  Closed
// slab test in binary32: per axis, inv = 1/d correctly rounded; an axis with
// d = 0, or whose reciprocal overflows, passes iff o lies in the slab
// [lo, hi]; otherwise its parameter interval has the ends (lo - o)*inv and
// (hi - o)*inv.  enter = the largest of tmin and the intervals' lower ends,
// exit = the smallest of tmax and their upper ends; hit iff enter <= exit.
// Each step is a monotone function of lo (non-increasing) and hi
// (non-decreasing), also after rounding, so a box inside a passing box can
// only fail or pass with an entry parameter at least as large: Alg. 1's
// pruning is exact, and so is the first-hit walk's pruning on the entry.
struct Ray {
    static constexpr int kFloats = 8;   // o.xyz, tmin, d.xyz, tmax
    float o[3], d[3], inv[3], tmin, tmax;
    bool par[3];
    __device__ void load(const float *q, int j)
    {
        const float4 *p = reinterpret_cast<const float4 *>(q) + 2 * (int64_t)j;
        const float4 a = p[0], b = p[1];
        o[0] = a.x; o[1] = a.y; o[2] = a.z; tmin = a.w;
        d[0] = b.x; d[1] = b.y; d[2] = b.z; tmax = b.w;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            inv[k] = __fdiv_rn(1.0f, d[k]);
            par[k] = d[k] == 0.0f || inv[k] == INFINITY || inv[k] == -INFINITY;
        }
    }
    // the entry parameter in *enter when the ray meets the box
    __device__ bool enter(float4 lo4, float4 hi4, float *enter) const
    {
        const float lo[3] = {lo4.x, lo4.y, lo4.z}, hi[3] = {hi4.x, hi4.y, hi4.z};
        float t_in = tmin, t_out = tmax;
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (par[k]) {
                ok = ok && lo[k] <= o[k] && o[k] <= hi[k];
            } else {
                const float t1 = (lo[k] - o[k]) * inv[k];
                const float t2 = (hi[k] - o[k]) * inv[k];
                const float nr = t1 < t2 ? t1 : t2;
                const float fr = t1 < t2 ? t2 : t1;
                t_in = nr > t_in ? nr : t_in;
                t_out = fr < t_out ? fr : t_out;
            }
        }
        *enter = t_in;
        return ok && t_in <= t_out;
    }
    __device__ bool test(float4 lo, float4 hi) const
    {
        float e;
        return enter(lo, hi, &e);
    }
    // A thin set contains no box of positive volume; claiming none only
    // forgoes a shortcut.
    __device__ bool contains(float4, float4) const { return false; }
    // the start point as a degenerate box: it keys the query order by where
    // the ray starts, and makes the mixed leaf schedule walk (not scan) a
    // ray's pieces
    __device__ void bounds(float lo[3], float hi[3]) const
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float t = (tmin == -INFINITY || d[k] == 0.0f) ? 0.0f : tmin;
            lo[k] = hi[k] = o[k] + t * d[k];
        }
    }
};

// Error word values of a query call (the count call's workspace).
constexpr uint32_t kQErrWalkBudget = 5;   // a walk ran out of its node-visit budget

struct Tree {
    const float4 *nodes;
    const int32_t *perm;   // leaf k -> primitive
    int n;
    uint32_t *err = nullptr;   // count calls: where a walk that ran out of budget is flagged
    int64_t budget = 0;        // node visits allowed per walk; 0: 2n (every node once)
    bool points = false;       // a tree of points: every leaf box has hi == lo
    __device__ int64_t walk_budget() const { return budget > 0 ? budget : 2 * (int64_t)n; }
    // a walk stopped with its budget spent: its count is short; report it
    __device__ void budget_spent() const
    {
        if (err) __hip_atomic_store(err, kQErrWalkBudget, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ int leaf0() const { return n - 1; }
    __device__ int index(int v) const { return v >= n - 1 ? v - (n - 1) : v; }
    __device__ void load(int v, float4 &a, float4 &b) const
    {
        const float4 *p = nodes + 2 * (int64_t)v;
        a = p[0];
        b = p[1];
    }
    // the box of leaf record v for a test: in a tree of points the upper
    // corner equals the lower one, so only the record's first half is read
    // (b.w, the rope, is then not loaded)
    __device__ void load_leaf_box(int v, float4 &a, float4 &b) const
    {
        const float4 *p = nodes + 2 * (int64_t)v;
        a = p[0];
        b = points ? make_float4(a.x, a.y, a.z, 0.0f) : p[1];
    }
    // right bound of node v whose record half `b` holds the rope
    __device__ int right_bound(float4 b) const
    {
        const int r = __float_as_int(b.w);
        return r == -1 ? n - 1 : index(r) - 1;
    }
    // largest node whose range starts at leaf r (r <= n-1)
    __device__ int first_at(int r) const
    {
        if (r <= n - 2) {
            const int l = __float_as_int(nodes[2 * (int64_t)r].w);
            if (index(l) >= r) return r;   // internal r is a right child
        }
        return n - 1 + r;
    }
};

// A piece: query, start node, left bound of the start node, end (exclusive)
// of the leaf range the walk covers.  Start node kAllHits marks a range
// whose leaves all pass (it lies under a node the query contains).
constexpr int kAllHits = -2;
__device__ __forceinline__ int4 piece(int q, int v, int i, int hi) { return make_int4(q, v, i, hi); }

constexpr int kWavesPerBlock = kBlock / 64;

// all lanes of the wave have issued their LDS accesses before any lane's
// later ones (LDS executes a wave's accesses in order; this keeps the
// compiler from moving them across)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// set lanes of mask below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// One split level's count pass: Alg. 1 from each item (a query, or a piece
// of the level above), cut at aligned blocks of 2^shift leaves.  Every
// piece it finds is appended to a list together with its item and its rank
// among that item's pieces.  After the scan of the counts, k_split_scatter
// puts each piece at its item's offset plus its rank: the order a second
// walk would emit them in, so no item is walked twice.  Past `cap` pieces
// the list stops growing; an item one of whose pieces did not fit is
// marked (kDropBit in its count) and passes through the level unsplit, as
// one piece, while every other item is split as usual.  The counts are
// accumulated atomically (the mark can come from another lane's flush at
// any time), so each level's count array starts at zero.
//
// Appends go to the wave's LDS stage.  After each append step the wave's
// active lanes check the stage and, once it holds kAppendStage - 64 or more
// entries (one step adds at most 64), move it to the list with one atomic;
// the wave flushes the rest when its items are done.  The lanes of a wave
// execute together, so the active ones can do this from inside their
// diverged walks.
constexpr int kAppendStage = 256;
constexpr int32_t kDropBit = 1 << 30;   // an item of a split level left unsplit

struct AppendLds {
    int4 piece[kWavesPerBlock][kAppendStage];
    int64_t item[kWavesPerBlock][kAppendStage];
    int32_t rank[kWavesPerBlock][kAppendStage];
    uint32_t n[kWavesPerBlock];
};

struct WaveAppend {
    int4 *piece;
    int64_t *item;
    int32_t *rank;
    uint32_t *n;
    unsigned long long *count;
    int64_t cap;
    int4 *g_piece;
    int64_t *g_item;
    int32_t *g_rank;
    int32_t *counts;   // per-item piece counts of the level (kDropBit: left unsplit)

    __device__ void to_list(unsigned long long slot, int4 pc, int64_t t, int32_t r) const
    {
        if (slot < (unsigned long long)cap) {
            g_piece[slot] = pc;
            g_item[slot] = t;
            g_rank[slot] = r;
        } else {
            atomicOr(&counts[t], kDropBit);
        }
    }
    // by the wave's active lanes, all with the same view of the stage
    __device__ void flush() const
    {
        wave_sync();
        const uint32_t total = *n;
        const uint32_t staged = total < (uint32_t)kAppendStage ? total : (uint32_t)kAppendStage;
        const uint64_t act = __ballot(1);
        const int r = (int)lanes_below(act), na = __popcll(act), first = __ffsll((unsigned long long)act) - 1;
        unsigned long long base = 0;
        if (r == 0 && staged > 0u) base = atomicAdd(count, (unsigned long long)staged);
        base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(base >> 32), first) << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, first);
        for (uint32_t k = r; k < staged; k += na) to_list(base + k, piece[k], item[k], rank[k]);
        wave_sync();
        if (r == 0) *n = 0u;
        wave_sync();
    }
    // The stage holds fewer than kAppendStage - 64 entries before a step
    // (it is flushed after any step that reaches that), and a step adds at
    // most 64, so k < kAppendStage.
    __device__ void put(int4 pc, int64_t t, int32_t r) const
    {
        // one LDS atomic for the step's active lanes, entries in lane order
        const uint64_t act = __ballot(1);
        const uint32_t below = lanes_below(act), cnt = (uint32_t)__popcll(act);
        const int first = __ffsll((unsigned long long)act) - 1;
        uint32_t base = 0u;
        if (below == 0u) base = atomicAdd(n, cnt);
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, first);
        const uint32_t k = base + below;
        piece[k] = pc;
        item[k] = t;
        rank[k] = r;
        if (base + cnt >= (uint32_t)(kAppendStage - 64)) flush();
    }
};

template <class Q, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_split(Tree tr, const float *__restrict__ queries, int m,
                                                  const int4 *__restrict__ in, const int64_t *in_count,
                                                  int shift, int32_t *__restrict__ counts,
                                                  unsigned long long *app_count, int64_t cap,
                                                  int4 *__restrict__ app_piece,
                                                  int64_t *__restrict__ app_item,
                                                  int32_t *__restrict__ app_rank)
{
    __shared__ AppendLds lds;
    const int wv = threadIdx.x >> 6;
    const WaveAppend ap{lds.piece[wv], lds.item[wv], lds.rank[wv], &lds.n[wv], app_count, cap,
                        app_piece, app_item, app_rank, counts};
    if ((threadIdx.x & 63) == 0) lds.n[wv] = 0u;
    wave_sync();
    const int64_t T = FIRST ? (int64_t)m : *in_count;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < T; t += (int64_t)gridDim.x * kBlock) {
        const int4 it = FIRST ? piece((int)t, 0, 0, tr.n) : in[t];
        int cnt = 0;
        auto emit = [&](int4 pc) {
            ap.put(pc, t, cnt);
            ++cnt;
        };
        // all-hit range [a, b): one all-hit piece per block it touches
        auto emit_range = [&](int a, int b) {
            while (a < b) {
                const int blk_end = ((a >> shift) + 1) << shift;
                const int e = blk_end < b ? blk_end : b;
                emit(piece(it.x, kAllHits, a, e));
                a = e;
            }
        };
        if (it.y == kAllHits) {
            emit_range(it.z, it.w);
        } else {
            Q q;
            q.load(queries, it.x);
            int v = it.y, i = it.z;
            const int hi = it.w;
            int64_t budget = tr.walk_budget();   // a walk visits each node at most once
            while (v != -1 && i < hi && --budget >= 0) {
                float4 a, b;
                tr.load(v, a, b);
                const int j = tr.right_bound(b);
                if (!q.test(a, b)) {
                    v = __float_as_int(b.w);
                    i = j + 1;
                    continue;
                }
                if ((i >> shift) == (j >> shift)) {
                    const int r = ((i >> shift) + 1) << shift;   // next block start
                    const int end = r < hi ? r : hi;
                    emit(piece(it.x, v, i, end));
                    if (r >= hi || r > tr.n - 1) break;
                    v = tr.first_at(r);
                    i = r;
                    continue;
                }
                if (q.contains(a, b)) {   // multi-block node with only hits below
                    emit_range(i, j + 1 < hi ? j + 1 : hi);
                    v = __float_as_int(b.w);
                    i = j + 1;
                    continue;
                }
                v = __float_as_int(a.w);   // multi-block node: descend
            }
            if (budget < 0) tr.budget_spent();
        }
        atomicAdd(&counts[t], cnt);   // the count array starts at zero
    }
    ap.flush();   // every lane of the wave
}

// A split level's output: each appended piece of an item that was split to
// slot out_off[item] + rank, and each item left unsplit (kDropBit) to its
// own slot out_off[item], unchanged.  Also clears the next level's counts
// (`next_counts`, next_n entries) before that level accumulates into them.
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_split_scatter(int n, int m, const int4 *__restrict__ in,
                                                          const int64_t *in_count,
                                                          const int64_t *__restrict__ out_off,
                                                          const int32_t *__restrict__ counts,
                                                          const unsigned long long *app_count,
                                                          int64_t cap,
                                                          const int4 *__restrict__ app_piece,
                                                          const int64_t *__restrict__ app_item,
                                                          const int32_t *__restrict__ app_rank,
                                                          int4 *__restrict__ out,
                                                          int32_t *__restrict__ next_counts,
                                                          int64_t next_n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t T = FIRST ? (int64_t)m : *in_count;
    for (int64_t t = t0; t < T; t += stride)
        if (counts[t] & kDropBit) out[out_off[t]] = FIRST ? piece((int)t, 0, 0, n) : in[t];
    const unsigned long long a = *app_count;
    const int64_t A = a < (unsigned long long)cap ? (int64_t)a : cap;   // pieces kept in the list
    for (int64_t k = t0; k < A; k += stride) {
        const int64_t t = app_item[k];
        if (!(counts[t] & kDropBit)) out[out_off[t] + app_rank[k]] = app_piece[k];
    }
    for (int64_t j = t0; j < next_n; j += stride) next_counts[j] = 0;
}

// The leaf level.  A level-2 piece covers the leaves [i, hi) of one aligned
// block of at most 2^split2 leaves, and Alg. 1 restricted to [i, hi)
// reports exactly the leaves of that range whose boxes pass, in index
// order: the tests are monotone under box inclusion, so every ancestor of a
// passing leaf passes too.  A piece can therefore be
//   * scanned by one wave, 64 consecutive leaf records per step with
//     coalesced loads, each step's ballot counting the hits and kept as a
//     word of the piece's hit mask (best for dense pieces: most leaves hit,
//     and a walk would be a long chain of dependent loads), or
//   * walked with Alg. 1 by one lane (best for sparse pieces: the walk
//     prunes).
// Two schedules (knob query_leaf_mode): 0 scans every piece; 1 walks the
// pieces whose start-node box lies mostly outside the query's bounding box
// and scans the rest.  Both give the same hits.  All-hit pieces are copied
// from leaf_perm, and a piece wider than kLeafScanMax leaves (left unsplit
// after a capacity overflow) is always walked.

constexpr int kLeafScanMax = 1024;

// Leaf-hit masks.  The count pass gives every level-2 piece at most
// kMaskLeaves (256) wide one bit per leaf of its range [i, hi) (bit k of word w:
// leaf i + 64 w + k), set for each hit.  The fill pass writes leaf_perm of
// the set bits in ascending leaf order, which is the order Alg. 1 reports
// them in, without loading or testing a box again.  Wider pieces (a split
// of more than 8 levels, or a level left unsplit after a capacity overflow)
// are tested again by the fill.
struct LeafMask {
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    // bits [a, e) of the mask, 0 <= a <= e <= kMaskLeaves
    __device__ void set(int a, int e)
    {
        auto part = [&](int w) -> uint64_t {
            const int lo = a > 64 * w ? a - 64 * w : 0;
            const int hi = e < 64 * w + 64 ? e - 64 * w : 64;
            if (lo >= hi) return 0;
            const uint64_t ones = hi - lo == 64 ? ~0ull : ((1ull << (hi - lo)) - 1ull);
            return ones << lo;
        };
        w0 |= part(0); w1 |= part(1); w2 |= part(2); w3 |= part(3);
    }
    __device__ void store(uint64_t *dst, int width) const
    {
        dst[0] = w0;
        if (width > 64) dst[1] = w1;
        if (width > 128) dst[2] = w2;
        if (width > 192) dst[3] = w3;
    }
};

// Alg. 1 restricted to the leaves [i, hi) from node v, by one lane: counts
// the hits, and writes them from slot pos of out (FILL; at most `limit`,
// the count the count call found for the piece, so a fill never writes
// past the piece's slots) or, with `keep`, sets them in `mask` (count
// pass, pieces at most kMaskLeaves wide).  The mask is a reference with a
// flag, not a pointer that may be null: that keeps it in registers.
template <class Q, bool FILL>
__device__ int64_t walk_piece(const Tree &tr, const Q &q, int v, int i, int hi, int32_t *out,
                              int64_t pos, LeafMask &mask, bool keep, int64_t limit = 0)
{
    const int leaf0 = tr.leaf0();
    const int i0 = i;
    int64_t cnt = 0;
    int64_t budget = tr.walk_budget();
    while (v != -1 && i < hi && --budget >= 0) {
        float4 a, b;
        tr.load(v, a, b);
        const int left = __float_as_int(a.w);
        const int j = tr.right_bound(b);
        if (q.test(a, b)) {
            if (v >= leaf0) {
                if (FILL) {
                    if (cnt < limit) out[pos + cnt] = left;
                } else if (keep) {
                    mask.set(i - i0, i - i0 + 1);
                }
                ++cnt;
            } else if (q.contains(a, b)) {
                const int e = j + 1 < hi ? j + 1 : hi;
                if (FILL)
                    for (int k = i; k < e && cnt + (k - i) < limit; ++k) out[pos + cnt + (k - i)] = tr.perm[k];
                else if (keep)
                    mask.set(i - i0, e - i0);
                cnt += e - i;
            } else {
                v = left;
                continue;
            }
        }
        v = __float_as_int(b.w);
        i = j + 1;
    }
    if (budget < 0) tr.budget_spent();
    return cnt;
}

// Is most of the node box inside the query's bounding box?  (Decides the
// schedule of a piece only: both schedules give the same hits.)  (Fraction of
// its volume, per-axis ratios; a flat axis counts as covered.)
template <class Q>
__device__ bool dense_piece(const Q &q, float4 a, float4 b)
{
    float ql[3], qh[3];
    q.bounds(ql, qh);
    const float lo[3] = {a.x, a.y, a.z}, hi[3] = {b.x, b.y, b.z};
    float f = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float e = hi[k] - lo[k];
        const float o = fminf(hi[k], qh[k]) - fmaxf(lo[k], ql[k]);
        f *= e > 0.0f ? fmaxf(o, 0.0f) / e : 1.0f;
    }
    return f >= 0.25f;
}

// One wave tests the leaves [lo, hi) of a piece, 64 consecutive leaf
// records per step (two steps in flight), and returns the hit count; with
// FILL it writes the hits from slot pos of out (at most `limit` of them),
// else, for a piece at most kMaskLeaves wide, it stores the ballots as the
// piece's mask.
template <class Q, bool FILL>
__device__ int64_t scan_piece(const Tree &tr, const Q &q, int lo, int hi, int32_t *out, int64_t pos,
                              uint64_t *mask, int64_t limit = 0)
{
    const int lane = threadIdx.x & 63;
    const bool keep = !FILL && hi - lo <= kMaskLeaves;
    int64_t c = 0;
    for (int k0 = lo; k0 < hi; k0 += 128) {
        const int k = k0 + lane, k2 = k + 64;
        float4 a, b, e, f;
        if (k < hi) tr.load_leaf_box(tr.leaf0() + k, a, b);
        if (k2 < hi) tr.load_leaf_box(tr.leaf0() + k2, e, f);
        const bool h = k < hi && q.test(a, b);
        const bool h2 = k2 < hi && q.test(e, f);
        const uint64_t m = __ballot(h), m2 = __ballot(h2);
        if (FILL) {
            const int64_t r1 = c + lanes_below(m), r2 = c + __popcll(m) + lanes_below(m2);
            if (h && r1 < limit) out[pos + r1] = __float_as_int(a.w);   // leaf: its primitive
            if (h2 && r2 < limit) out[pos + r2] = __float_as_int(e.w);
        } else if (keep && lane == 0) {
            const int w = (k0 - lo) >> 6;
            mask[w] = m;
            if (k0 + 64 < hi) mask[w + 1] = m2;
        }
        c += __popcll(m) + __popcll(m2);
    }
    return c;
}

// Plain schedule (query_leaf_mode 0): one wave per piece.
template <class Q>
__global__ __launch_bounds__(kBlock) void k_leaf_scan_count(Tree tr, const float *__restrict__ queries,
                                                       const int4 *__restrict__ in,
                                                       const int64_t *in_count,
                                                       int32_t *__restrict__ counts,
                                                       uint64_t *__restrict__ masks)
{
    const int64_t T = *in_count;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t t = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; t < T; t += nw) {
        const int4 it = in[t];
        int64_t cnt = it.w - it.z;
        if (it.y != kAllHits) {
            if (it.w - it.z > kLeafScanMax) continue;   // k_leaf_count_wide
            Q q;
            q.load(queries, it.x);
            cnt = scan_piece<Q, false>(tr, q, it.z, it.w, nullptr, 0, masks + t * kMaskWords);
        }
        if (lane == 0) counts[t] = (int32_t)cnt;
    }
}

// Count of the pieces wider than kLeafScanMax (left unsplit after a split
// level overflowed) for the plain schedule: Alg. 1 by one lane per piece,
// all lanes in parallel.
template <class Q>
__global__ __launch_bounds__(kBlock) void k_leaf_count_wide(Tree tr, const float *__restrict__ queries,
                                                       const int4 *__restrict__ in,
                                                       const int64_t *in_count,
                                                       int32_t *__restrict__ counts)
{
    const int64_t T = *in_count;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < T; t += (int64_t)gridDim.x * kBlock) {
        const int4 it = in[t];
        if (it.y == kAllHits || it.w - it.z <= kLeafScanMax) continue;
        Q q;
        q.load(queries, it.x);
        LeafMask none;
        counts[t] = (int32_t)walk_piece<Q, false>(tr, q, it.y, it.z, it.w, nullptr, 0, none, false);
    }
}

// Mixed schedule (query_leaf_mode 1): each wave takes 64 pieces; sparse ones
// are walked by their own lane, then the wave scans its dense pieces one at
// a time.  Better when most pieces are sparse (few hits per piece); the
// plain scan above is better when most are dense.  Both record the same
// masks.
template <class Q>
__global__ __launch_bounds__(kBlock) void k_leaf_mixed_count(Tree tr, const float *__restrict__ queries,
                                                             const int4 *__restrict__ in,
                                                             const int64_t *in_count,
                                                             int32_t *__restrict__ counts,
                                                             uint64_t *__restrict__ masks)
{
    const int64_t T = *in_count;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); t0 < T; t0 += stride) {
        const int64_t t = t0 + lane;
        int4 it = make_int4(0, -1, 0, 0);
        bool scan = false;
        int64_t cnt = 0;
        if (t < T) {
            it = in[t];
            if (it.y == kAllHits) {
                cnt = it.w - it.z;
            } else {
                Q q;
                q.load(queries, it.x);
                bool walk = true;
                if (it.w - it.z <= kLeafScanMax) {
                    float4 a, b;
                    tr.load(it.y, a, b);
                    walk = !dense_piece(q, a, b);
                }
                if (walk) {
                    const bool keep = it.w - it.z <= kMaskLeaves;
                    LeafMask mk;
                    cnt = walk_piece<Q, false>(tr, q, it.y, it.z, it.w, nullptr, 0, mk, keep);
                    if (keep) mk.store(masks + t * kMaskWords, it.w - it.z);
                } else {
                    scan = true;
                }
            }
        }
        uint64_t todo = __ballot(scan);
        while (todo) {
            const int L = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int qi = __builtin_amdgcn_readlane(it.x, L);
            const int lo = __builtin_amdgcn_readlane(it.z, L);
            const int hi = __builtin_amdgcn_readlane(it.w, L);
            Q q;
            q.load(queries, qi);
            const int64_t c = scan_piece<Q, false>(tr, q, lo, hi, nullptr, 0, masks + (t0 + L) * kMaskWords);
            if (lane == L) cnt = c;
        }
        if (t < T) counts[t] = (int32_t)cnt;
    }
}

// Fill for both schedules, 64 pieces per wave at a time, with the hits of
// all 64 spread evenly over the lanes:
//   1. lane l loads piece t0 + l: its descriptor, output slot and mask (an
//      all-hit piece at most kMaskLeaves wide counts as a full mask);
//   2. a wave scan of the masks' popcounts gives each piece's first hit
//      among the wave's H hits;
//   3. lane l takes hits l, l + 64, ...: it finds the piece (binary search
//      over the scan, read from other lanes with __shfl), the set bit of
//      that rank in the piece's mask, and writes leaf_perm of that leaf to
//      the piece's slot plus the rank.  kFillUnroll hits per lane are
//      loaded before any is stored, so a wave's pieces cost a round trip
//      for the descriptors and about one per 64 * kFillUnroll hits.
// When the wave's pieces average kDenseFill hits or more, it instead writes
// each piece's mask words with the whole wave (a lane per leaf, coalesced),
// four pieces per step.  Bits are ranked in ascending leaf order, Alg. 1's
// order.  All-hit pieces
// wider than kMaskLeaves are copied by the whole wave; other wider pieces
// are left to k_leaf_fill_wide.
constexpr int kFillUnroll = 4;
constexpr int kDenseFill = 16;   // hits per piece (wave average) from which whole-wave writes win

// position of the set bit of rank r (r < popcount(x)) in x
__device__ __forceinline__ int select_bit(uint64_t x, int r)
{
    int pos = 0;
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
        const uint64_t low = x & ((1ull << half) - 1ull);
        const int c = __popcll(low);
        if (r >= c) {
            r -= c;
            x >>= half;
            pos += half;
        } else {
            x = low;
        }
    }
    return pos;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// The count call can process the queries in another order than the
// caller's (the "query_order" knob).  Then the pieces name positions in a
// reordered copy of the queries, and the hits of a piece go to its offset
// in that order plus its query's shift (caller-order offset minus
// reordered offset).  `flag`, written by the count call, says which case
// holds, so the fill does not depend on the knob.
struct QueryMap {
    const int32_t *flag;     // nonzero: the queries were reordered
    const float *sorted;     // the reordered copy
    const int64_t *shift;    // per reordered position
};

template <class Q>
__global__ __launch_bounds__(kBlock) void k_leaf_fill(Tree tr, const int4 *__restrict__ in,
                                                 const int64_t *in_count,
                                                 const int64_t *__restrict__ hit_off,
                                                 const uint64_t *__restrict__ masks,
                                                 QueryMap qm, int32_t *__restrict__ out)
{
    const int64_t T = *in_count;
    const bool reordered = *qm.flag != 0;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); t0 < T; t0 += stride) {
        const int64_t t = t0 + lane;
        int4 it = make_int4(0, kAllHits, 0, 0);   // past the end: empty
        int64_t pos = 0;
        uint64_t w[kMaskWords] = {0ull, 0ull, 0ull, 0ull};
        if (t < T) {
            it = in[t];
            pos = hit_off[t] + (reordered ? qm.shift[it.x] : 0);
            const int width = it.w - it.z;
            if (width <= kMaskLeaves) {
                if (it.y == kAllHits) {
                    LeafMask full;
                    full.set(0, width);
                    w[0] = full.w0; w[1] = full.w1; w[2] = full.w2; w[3] = full.w3;
                } else {
#pragma unroll
                    for (int k = 0; k < kMaskWords; ++k)
                        if (64 * k < width) w[k] = masks[t * kMaskWords + k];
                }
            }
        }
        const int c = __popcll(w[0]) + __popcll(w[1]) + __popcll(w[2]) + __popcll(w[3]);
        // wave scan: first hit of each piece among the wave's hits
        int incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        const int base = incl - c;
        const int H = __shfl(incl, 63);
        if (H >= 64 * kDenseFill) {
            // dense pieces: the whole wave writes one mask word of one piece
            // per step (coalesced), four pieces' loads in flight
            for (int g0 = 0; g0 < 64; g0 += 4) {
                int32_t v[4][kMaskWords];
                int64_t d[4][kMaskWords];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int L = g0 + g;
                    const int z = __builtin_amdgcn_readlane(it.z, L);
                    const int64_t p = ((int64_t)__builtin_amdgcn_readlane((int)(pos >> 32), L) << 32) |
                                      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pos, L);
                    int prefix = 0;
#pragma unroll
                    for (int k = 0; k < kMaskWords; ++k) {
                        const uint64_t wk =
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(w[k] >> 32), L) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)w[k], L);
                        d[g][k] = -1;
                        if ((wk >> lane) & 1ull) {
                            v[g][k] = tr.perm[z + 64 * k + lane];
                            d[g][k] = p + prefix + lanes_below(wk);
                        }
                        prefix += __popcll(wk);
                    }
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int k = 0; k < kMaskWords; ++k)
                        if (d[g][k] >= 0) out[d[g][k]] = v[g][k];
            }
        } else
        for (int h0 = 0; h0 < H; h0 += 64 * kFillUnroll) {
            int32_t v[kFillUnroll];
            int64_t dst[kFillUnroll];
#pragma unroll
            for (int u = 0; u < kFillUnroll; ++u) {
                const int h = h0 + u * 64 + lane;
                dst[u] = -1;
                // every lane takes part in the shuffles; only h < H is used
                int lo = 0, hi = 63;   // the last piece whose first hit is <= h
#pragma unroll
                for (int step = 0; step < 6; ++step) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (__shfl(base, mid) <= h) lo = mid;
                    else hi = mid - 1;
                }
                const int r0 = h - __shfl(base, lo);   // rank of hit h in its piece
                int r = r0;
                const int z = __shfl(it.z, lo);
                const int64_t p = (int64_t)shfl64((uint64_t)pos, lo);
                uint64_t x = 0ull;
                int word = 0;
#pragma unroll
                for (int k = 0; k < kMaskWords; ++k) {
                    const uint64_t wk = shfl64(w[k], lo);
                    const int ck = __popcll(wk);
                    if (x == 0ull) {
                        if (r < ck) { x = wk; word = k; }
                        else r -= ck;
                    }
                }
                if (h < H && x != 0ull) {   // no lane-crossing reads in here
                    const int leaf = z + 64 * word + select_bit(x, r);
                    v[u] = tr.perm[leaf];
                    dst[u] = p + r0;
                }
            }
#pragma unroll
            for (int u = 0; u < kFillUnroll; ++u)
                if (dst[u] >= 0) out[dst[u]] = v[u];
        }
        // all-hit pieces wider than a mask: the whole wave copies each
        uint64_t wide = __ballot(t < T && it.y == kAllHits && it.w - it.z > kMaskLeaves);
        while (wide) {
            const int L = __ffsll((unsigned long long)wide) - 1;
            wide &= wide - 1;
            const int z = __builtin_amdgcn_readlane(it.z, L);
            const int e = __builtin_amdgcn_readlane(it.w, L);
            const int64_t p = (int64_t)shfl64((uint64_t)pos, L);
            for (int k = lane; k < e - z; k += 64) out[p + k] = tr.perm[z + k];
        }
    }
}

// Fill of the pieces wider than kMaskLeaves (only after a split level
// overflowed, or with split2 above 8), 64 pieces per wave at a time: a
// sparse piece, or one wider than kLeafScanMax, is walked with Alg. 1 by its
// own lane; the wave then scans its dense ones one after another.
template <class Q>
__global__ __launch_bounds__(kBlock) void k_leaf_fill_wide(Tree tr, const float *__restrict__ queries_in,
                                                      const int4 *__restrict__ in,
                                                      const int64_t *in_count,
                                                      const int64_t *__restrict__ hit_off,
                                                      QueryMap qm, int32_t *__restrict__ out)
{
    const int64_t T = *in_count;
    const bool reordered = *qm.flag != 0;
    const float *queries = reordered ? qm.sorted : queries_in;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); t0 < T; t0 += stride) {
        const int64_t t = t0 + lane;
        int4 it = make_int4(0, kAllHits, 0, 0);
        int64_t pos = 0, limit = 0;
        bool scan = false;
        if (t < T) {
            it = in[t];
            const int64_t h0 = hit_off[t];
            pos = h0 + (reordered ? qm.shift[it.x] : 0);
            limit = hit_off[t + 1] - h0;
            if (it.y != kAllHits && it.w - it.z > kMaskLeaves && limit > 0) {
                Q q;
                q.load(queries, it.x);
                bool walk = true;
                if (it.w - it.z <= kLeafScanMax) {
                    float4 a, b;
                    tr.load(it.y, a, b);
                    walk = !dense_piece(q, a, b);
                }
                LeafMask none;
                if (walk) walk_piece<Q, true>(tr, q, it.y, it.z, it.w, out, pos, none, false, limit);
                else scan = true;
            }
        }
        uint64_t todo = __ballot(scan);
        while (todo) {
            const int L = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int qi = __builtin_amdgcn_readlane(it.x, L);
            const int lo = __builtin_amdgcn_readlane(it.z, L);
            const int hi = __builtin_amdgcn_readlane(it.w, L);
            const int plo = __builtin_amdgcn_readlane((int)(pos & 0xffffffff), L);
            const int phi = __builtin_amdgcn_readlane((int)(pos >> 32), L);
            const int64_t lim = (int64_t)shfl64((uint64_t)limit, L);
            Q q;
            q.load(queries, qi);
            scan_piece<Q, true>(tr, q, lo, hi, out, ((int64_t)phi << 32) | (uint32_t)plo, nullptr, lim);
        }
    }
}

// Staged output of a fill pass, per wave.  The 64 items (pieces or
// queries) a wave takes at a time have consecutive output ranges (item
// order is output order), so the wave gathers their hits in its own LDS
// region and writes them out in one coalesced run:
//   1. each lane walks its item; a leaf hit goes to the stage at its offset
//      from the wave's first output slot (put), an all-hit leaf range
//      becomes a job: output slot, first leaf_perm entry, length;
//   2. the wave copies the jobs from leaf_perm, 64 entries per lane step,
//      with up to kCopyDepth independent loads per lane in flight (a dense
//      query's pieces are mostly such ranges: copying them one dependent
//      load at a time is what made filling slower than counting);
//   3. the wave writes the stage to the output.
// Hits past the stage capacity, and jobs past the job list, are written
// straight to the output: every hit lands in the same slot either way.
// Only the wave synchronises with itself, so a long walk holds up its own
// wave and no other.
constexpr int kWaveHits = 1024;
constexpr int kWaveJobs = 128;
constexpr int kCopyDepth = 8;

struct HitJob {
    int32_t rel;              // output slot - the wave's first slot
    int32_t a, len;
};

struct WaveStageLds {
    int32_t hits[kWavesPerBlock][kWaveHits];
    HitJob jobs[kWavesPerBlock][kWaveJobs];
    int njobs[kWavesPerBlock];
};

struct HitStage {
    int32_t *hits;            // the wave's LDS [kWaveHits]
    HitJob *jobs;             // the wave's LDS [kWaveJobs]
    int *njobs;               // the wave's LDS counter
    int32_t *out;
    const int32_t *perm;      // leaf_perm that job ranges index
    int64_t base;             // output slot of the wave's first item

    __device__ void put(int64_t pos, int32_t v) const
    {
        const int64_t r = pos - base;
        if (r < kWaveHits) hits[r] = v;
        else out[pos] = v;
    }
    // perm[a .. a+len) go to output slots pos .. pos+len
    __device__ void range(int64_t pos, int32_t a, int32_t len) const
    {
        if (len <= 0) return;
        const int64_t rel = pos - base;
        const int j = rel <= INT32_MAX ? atomicAdd(njobs, 1) : kWaveJobs;
        if (j < kWaveJobs) {
            jobs[j] = HitJob{(int32_t)rel, a, len};
            return;
        }
        // no room: this lane copies the range, kCopyDepth loads at a time
        for (int k0 = 0; k0 < len; k0 += kCopyDepth) {
            int32_t v[kCopyDepth];
#pragma unroll
            for (int u = 0; u < kCopyDepth; ++u)
                if (k0 + u < len) v[u] = perm[a + k0 + u];
#pragma unroll
            for (int u = 0; u < kCopyDepth; ++u)
                if (k0 + u < len) put(pos + k0 + u, v[u]);
        }
    }
    // steps 2 and 3; every lane of the wave calls it
    __device__ void flush(int64_t total) const
    {
        const int lane = threadIdx.x & 63;
        wave_sync();
        const int nj = *njobs < kWaveJobs ? *njobs : kWaveJobs;
        // walk the jobs in 64-entry slices; each round loads up to
        // kCopyDepth slices (of one or more jobs) before storing any
        int j = 0, off = 0;   // next slice: job j from entry off (uniform)
        while (j < nj) {
            int32_t v[kCopyDepth];
            int64_t dst[kCopyDepth];
#pragma unroll
            for (int u = 0; u < kCopyDepth; ++u) {
                dst[u] = -1;
                if (j < nj) {
                    const HitJob jb = jobs[j];
                    const int k = off + lane;
                    if (k < jb.len) {
                        v[u] = perm[jb.a + k];
                        dst[u] = base + jb.rel + k;
                    }
                    off += 64;
                    if (off >= jb.len) { ++j; off = 0; }
                }
            }
#pragma unroll
            for (int u = 0; u < kCopyDepth; ++u)
                if (dst[u] >= 0) put(dst[u], v[u]);
        }
        wave_sync();
        const int staged = total < kWaveHits ? (int)total : kWaveHits;
        for (int k = lane; k < staged; k += 64) out[base + k] = hits[k];
        if (lane == 0) *njobs = 0;
        wave_sync();   // the stage is reused by the wave's next items
    }
};

__device__ __forceinline__ HitStage wave_stage(WaveStageLds &lds, int32_t *out, const int32_t *perm,
                                               int64_t base)
{
    const int w = threadIdx.x >> 6;
    return HitStage{lds.hits[w], lds.jobs[w], &lds.njobs[w], out, perm, base};
}

// Offsets of a count call with nothing to walk: all zero; and the call's
// error word cleared.
__global__ void k_zero_i64(int64_t *p, int64_t count, uint32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = 0;
    if (i == 0) *err = 0u;
}

// -------------------------------------------------------------- scan
//
// Exclusive scan of `m` int32 counts into int64 offsets[0..m] (offsets[m] =
// total).  The count is either a host value (m_dev == nullptr) or read on
// the device; grids are sized for `cap`, the largest count possible.

template <typename T>
__device__ __forceinline__ T block_excl_scan_total(T v, T *sh /* [kBlock/64] */, T *block_total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    T before = 0, all = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) before += sh[w];
        all += sh[w];
    }
    *block_total = all;
    return before + x - v;
}

__device__ __forceinline__ int64_t count_of(int64_t cap, const int64_t *m_dev)
{
    return m_dev ? *m_dev : cap;
}

// a split level's count of an item: its pieces, or 1 if it is left unsplit.
// The scans also run over hit counts, which stay below kDropBit: a piece
// covers at most LBVH_MAX_PRIMS < 2^30 leaves.
__device__ __forceinline__ int32_t piece_count(int32_t c) { return (c & kDropBit) ? 1 : c; }

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ counts, int64_t cap,
                                                        const int64_t *m_dev, int64_t *__restrict__ partials)
{
    __shared__ int64_t sh[kBlock / 64];
    const int64_t m = count_of(cap, m_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    if ((int64_t)blockIdx.x * kScanTile >= m) return;   // whole block past the end
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += piece_count(counts[base + k]);
    int64_t total;
    block_excl_scan_total<int64_t>(s, sh, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(int64_t *partials, int64_t cap,
                                                          const int64_t *m_dev)
{
    __shared__ int64_t sh[kBlock / 64];
    const int64_t m = count_of(cap, m_dev);
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? partials[b] : 0;
        int64_t total;
        const int64_t e = block_excl_scan_total<int64_t>(v, sh, &total);
        if (b < nb) partials[b] = carry + e;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_final(const int32_t *__restrict__ counts, int64_t cap,
                                                       const int64_t *m_dev,
                                                       const int64_t *__restrict__ partials,
                                                       int64_t *__restrict__ offsets)
{
    __shared__ int64_t sh[kBlock / 64];
    const int64_t m = count_of(cap, m_dev);
    if (m == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
        return;
    }
    if ((int64_t)blockIdx.x * kScanTile >= m) return;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        c[k] = base + k < m ? piece_count(counts[base + k]) : 0;
        s += c[k];
    }
    int64_t total;
    int64_t run = partials[blockIdx.x] + block_excl_scan_total<int64_t>(s, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) offsets[base + k] = run;
        run += c[k];
        if (base + k == m - 1) offsets[m] = run;
    }
}

// The number of pieces a split level emits (its output always holds them:
// split items' pieces are at most the list capacity, and each unsplit item
// adds one).  The overflow word stays 0 (every level's offsets are valid).
__global__ void k_level_check(const int64_t *__restrict__ off, const int64_t *parent_dev,
                              int64_t parent_host, int32_t *__restrict__ overflow,
                              int64_t *__restrict__ count)
{
    const int64_t parents = parent_dev ? *parent_dev : parent_host;
    *overflow = 0;
    *count = off[parents];
}

// offsets[q] = hit offset of query q's first leaf-walk piece.  With `perm`
// (queries processed in another order: position q holds caller query
// perm[q]) it also writes query q's hit count to counts[perm[q]].
__global__ __launch_bounds__(kBlock) void k_compose(const int64_t *__restrict__ off1,
                                                    const int32_t *__restrict__ ovf1,
                                                    const int64_t *__restrict__ off2,
                                                    const int32_t *__restrict__ ovf2,
                                                    const int64_t *__restrict__ hit_off, int m,
                                                    int64_t *__restrict__ offsets,
                                                    const int32_t *__restrict__ perm,
                                                    int32_t *__restrict__ counts)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q > m) return;
    auto first_hit = [&](int64_t x) {
        const int64_t p1 = *ovf1 ? x : off1[x];
        const int64_t p2 = *ovf2 ? p1 : off2[p1];
        return hit_off[p2];
    };
    const int64_t h = first_hit(q);
    offsets[q] = h;
    if (perm && q < m) {
        const uint32_t j = (uint32_t)perm[q];
        if (j < (uint32_t)m) counts[j] = (int32_t)(first_hit(q + 1) - h);
    }
}

// Exclusive scan of int32 counts into int64 offsets (three launches).
void scan(const int32_t *counts, int64_t cap, const int64_t *m_dev, int64_t *partials,
          int64_t *offsets, hipStream_t s)
{
    const unsigned nb = (unsigned)((cap + kScanTile - 1) / kScanTile);
    const unsigned g = nb > 0 ? nb : 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(g), dim3(kBlock), 0, s, counts, cap, m_dev, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, partials, cap, m_dev);
    hipLaunchKernelGGL(k_scan_final, dim3(g), dim3(kBlock), 0, s, counts, cap, m_dev, partials,
                       offsets);
}

}  // namespace
}  // namespace lbvh
