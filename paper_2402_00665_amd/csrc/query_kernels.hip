// Stackless range queries on gfx950 (Alg. 1) and their CSR output.
//
// Alg. 1 walks the tree in preorder from the root: a node whose box passes
// the test sends the walk to its left child (internal node) or reports the
// primitive (leaf) and follows the rope; a node that fails sends it along
// the rope; the sentinel -1 ends it.  One thread per query makes the
// heaviest query the critical path (a query can hit 10^5 primitives, each a
// dependent node load), so each query's walk is cut into independent pieces
// by aligned blocks of leaves, without changing what is visited in order:
//
// * During a walk the current node's leaf range [i, j] is known for free:
//   i stays when descending left, and a rope leads to a node whose Karras
//   index is its left bound, so i = index(rope target); j = index(rope) - 1
//   (n - 1 at the sentinel).
// * A split walk covers the leaf range [i, hi) of its piece; at the first
//   passing node inside an aligned block of 2^S leaves it emits a piece
//   (node, i, block end) and jumps to the largest node starting at the next
//   block: internal node r if it is a right child (its split >= r), else
//   leaf r.  Everything it skips lies inside the emitted block.
// * Level 1 splits each query's whole walk by 2^split1 leaves, level 2
//   splits each level-1 piece by 2^split2 leaves (tuning knobs).
// * The leaf level tests a level-2 piece [i, hi) leaf by leaf, one wave per
//   piece, 64 leaves at a time (or, in the mixed schedule, walks sparse
//   pieces with Alg. 1, one lane each): both tests are monotone under box
//   inclusion (every ancestor of a passing leaf passes), so Alg. 1
//   restricted to [i, hi) reports exactly the passing leaves of [i, hi), in
//   index order.  A piece wider than kLeafScanMax leaves (left unsplit after
//   a capacity overflow) is walked with plain Alg. 1 by one lane.
// * A passing node whose box the query contains has only hits below it: its
//   leaf range [i, j] is reported from leaf_perm without visiting it (as
//   all-hit pieces in the split levels).  Alg. 1 would visit the same
//   leaves in the same order and report the same primitives.
// Pieces are emitted in walk order, so concatenating their hits gives the
// plain walk's hits in the plain walk's order.  A split level is one walk
// per item that appends each piece with its rank among the item's pieces,
// a scan of the per-item counts and a scatter of the pieces to offset +
// rank; a level whose pieces would exceed the workspace capacity passes its
// items through unsplit (same results, less parallel).  The leaf level's
// count records a hit mask per piece, and the fill call writes leaf_perm of
// the set bits.
// No contraction: the sphere test is evaluated exactly as written.
#pragma clang fp contract(off)

#include "query_common.hpp"
#include "radix_sort.hpp"

namespace lbvh {
namespace {

// ------------------------------------------------------------ query order
//
// With the "query_order" knob set, the count call first sorts the queries
// by a 16-bit Morton key of their centres (quantised in the root's box,
// clamped to it) and runs every split and leaf level on the sorted copy,
// so that neighbouring lanes and waves walk neighbouring parts of the tree
// and share its records in the caches.  Only the schedule changes: each
// query's pieces, hits and hit order are what they are in the caller's
// order.  At the end, the per-query counts go back to the caller's order,
// their scan gives the caller's offsets, and each sorted position gets the
// shift that moves its hits to its caller-order slot (applied by the fill).

// keys of the queries, their digit histograms (LDS, then one global add
// per digit and block), and the first sort pass's cleared look-back status
template <class Q>
__global__ __launch_bounds__(kBlock) void k_qorder_keys(Tree tr, const float *__restrict__ queries,
                                                   int m, uint32_t *__restrict__ keys,
                                                   uint32_t *hist, uint32_t *__restrict__ status0,
                                                   int64_t status_words)
{
    __shared__ uint32_t lh[kQOrderPasses * kRadix];
    for (int j = threadIdx.x; j < kQOrderPasses * kRadix; j += kBlock) lh[j] = 0u;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = gid; j < status_words; j += stride) status0[j] = 0u;
    __syncthreads();
    float4 a, b;
    tr.load(0, a, b);   // the root's box (leaf 0's when n = 1)
    const float rlo[3] = {a.x, a.y, a.z}, rhi[3] = {b.x, b.y, b.z};
    float scale[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float ext = rhi[k] - rlo[k];
        scale[k] = ext > 0.0f ? 1024.0f / ext : 0.0f;
    }
    for (int64_t i = gid; i < m; i += stride) {
        Q q;
        q.load(queries, (int)i);
        float lo[3], hi[3];
        q.bounds(lo, hi);
        uint32_t c[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float t = ((lo[k] + hi[k]) * 0.5f - rlo[k]) * scale[k];
            c[k] = (uint32_t)fminf(fmaxf(t, 0.0f), 1023.0f);   // NaN -> 0
        }
        const uint32_t key = Code<uint32_t>::make(c[0], c[1], c[2]) >> 14;
        keys[i] = key;
        atomicAdd(&lh[key & (kRadix - 1)], 1u);
        atomicAdd(&lh[kRadix + (key >> kRadixBits)], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kQOrderPasses * kRadix; j += kBlock)
        if (lh[j]) atomicAdd(&hist[j], lh[j]);
}

// the sorted copy of the queries
template <class Q>
__global__ __launch_bounds__(kBlock) void k_qorder_gather(const float *__restrict__ queries,
                                                     const int32_t *__restrict__ perm, int m,
                                                     float *__restrict__ sorted)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const uint32_t j = (uint32_t)perm[i];
        if (j >= (uint32_t)m) continue;   // never for a sort that completed; no stray reads otherwise
#pragma unroll
        for (int k = 0; k < Q::kFloats; ++k)
            sorted[Q::kFloats * i + k] = queries[Q::kFloats * (int64_t)j + k];
    }
}

// shift of each sorted position: caller-order offset - sorted-order offset
__global__ __launch_bounds__(kBlock) void k_qorder_shift(const int64_t *__restrict__ off_sorted,
                                                    const int32_t *__restrict__ perm,
                                                    const int64_t *__restrict__ offsets, int m,
                                                    int64_t *__restrict__ shift)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride)
        shift[i] = (uint32_t)perm[i] < (uint32_t)m ? offsets[perm[i]] - off_sorted[i] : 0;
}

// start of a count call: the split levels' append counters, the order
// flag the fill reads, the call's error word, (when reordering) the sort's
// tile counters and histograms, and the first split level's per-query
// counts (cnt1, m entries), which that level accumulates into
__global__ void k_query_reset(unsigned long long *app_count, int32_t *order_flag, int order,
                              uint32_t *tile_counters, uint32_t *hist, uint32_t *err,
                              int32_t *cnt1, int64_t m)
{
    if (blockIdx.x == 0) {
        if (threadIdx.x < 2) app_count[threadIdx.x] = 0ull;
        if (threadIdx.x == 0) {
            *order_flag = order;
            *err = 0u;
        }
        if (order) {
            if (threadIdx.x < kQOrderPasses) tile_counters[threadIdx.x] = 0u;
            for (int j = threadIdx.x; j < kQOrderPasses * kRadix; j += blockDim.x) hist[j] = 0u;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) cnt1[j] = 0;
}

// ---------------------------------------------------------- first hit
//
// First hit of each ray: among the primitives it meets, the one with the
// smallest entry parameter, ties to the smallest leaf position (Morton
// order).  One lane walks Alg. 1 from the root and enters a node only if the
// ray meets its box with an entry parameter below the best hit so far (any
// entry while there is none).  A box inside a node's box never has a smaller
// entry parameter (the slab test is monotone under box inclusion), so a
// pruned subtree holds no better hit; Alg. 1 reaches leaves in ascending
// position, so on equal entries the first leaf found stays.  An n = 0 tree
// gives every ray hit -1 and t = +inf (n = 0 never reaches here: the caller
// fills those).
__global__ __launch_bounds__(kBlock) void k_ray_first(Tree tr, const float *__restrict__ rays, int m,
                                                      int32_t *__restrict__ hit, float *__restrict__ t)
{
    const int leaf0 = tr.leaf0();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m; j += stride) {
        Ray q;
        q.load(rays, (int)j);
        int best_hit = -1, v = 0;
        float best = INFINITY;
        int64_t budget = tr.walk_budget();
        while (v != -1 && --budget >= 0) {
            float4 a, b;
            tr.load(v, a, b);
            float e;
            if (q.enter(a, b, &e) && (best_hit < 0 || e < best)) {
                if (v >= leaf0) {
                    best_hit = __float_as_int(a.w);
                    best = e;
                    v = __float_as_int(b.w);
                } else {
                    v = __float_as_int(a.w);
                }
            } else {
                v = __float_as_int(b.w);
            }
        }
        if (budget < 0) tr.budget_spent();
        hit[j] = best_hit;
        t[j] = best;
    }
}

__global__ __launch_bounds__(kBlock) void k_ray_none(int64_t m, int32_t *__restrict__ hit,
                                                     float *__restrict__ t, uint32_t *err)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t j0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j0 == 0) *err = 0u;
    for (int64_t j = j0; j < m; j += stride) {
        hit[j] = -1;
        t[j] = INFINITY;
    }
}

struct Scratch {
    int32_t *cnt1, *cnt2, *hcnt, *ovf;
    int64_t *off1, *off2, *hoff, *partials, *count;
    int4 *items1, *items2, *app_piece;
    int64_t *app_item;
    int32_t *app_rank;
    unsigned long long *app_count;
    uint64_t *hmask;
    int32_t *order_flag;     // nonzero: this count call reordered the queries
    uint32_t *sort_ctr;      // the order sort's tile counters [0], [1]
    uint32_t *err;           // the count call's error word (order sort, walk budgets)
    float *qsorted;
    int32_t *qperm;
    int64_t *qoff;
    uint32_t *qkeys[2], *qstatus[2], *qhist;
    int32_t *qvals;
};

Scratch carve(char *ws, const QueryLayout &L)
{
    Scratch S;
    S.cnt1 = reinterpret_cast<int32_t *>(ws + L.cnt1);
    S.off1 = reinterpret_cast<int64_t *>(ws + L.off1);
    S.items1 = reinterpret_cast<int4 *>(ws + L.items1);
    S.cnt2 = reinterpret_cast<int32_t *>(ws + L.cnt2);
    S.off2 = reinterpret_cast<int64_t *>(ws + L.off2);
    S.items2 = reinterpret_cast<int4 *>(ws + L.items2);
    S.app_piece = reinterpret_cast<int4 *>(ws + L.app_piece);
    S.app_item = reinterpret_cast<int64_t *>(ws + L.app_item);
    S.app_rank = reinterpret_cast<int32_t *>(ws + L.app_rank);
    S.hmask = reinterpret_cast<uint64_t *>(ws + L.hmask);
    S.hcnt = reinterpret_cast<int32_t *>(ws + L.hcnt);
    S.hoff = reinterpret_cast<int64_t *>(ws + L.hoff);
    S.partials = reinterpret_cast<int64_t *>(ws + L.partials);
    S.ovf = reinterpret_cast<int32_t *>(ws + L.ctrl);              // [0] level 1, [1] level 2
    S.count = reinterpret_cast<int64_t *>(ws + L.ctrl + 64);       // [0] pieces 1, [1] pieces 2
    S.app_count = reinterpret_cast<unsigned long long *>(ws + L.ctrl + 96);   // [0] level 1, [1] level 2
    S.order_flag = reinterpret_cast<int32_t *>(ws + L.ctrl + 8);
    S.sort_ctr = reinterpret_cast<uint32_t *>(ws + L.ctrl + 16);   // [0], [1] tiles
    S.err = reinterpret_cast<uint32_t *>(ws + L.ctrl + kQueryErrorByte);
    S.qsorted = reinterpret_cast<float *>(ws + L.qsorted);
    S.qperm = reinterpret_cast<int32_t *>(ws + L.qperm);
    S.qoff = reinterpret_cast<int64_t *>(ws + L.qoff);
    for (int k = 0; k < 2; ++k) {
        S.qkeys[k] = reinterpret_cast<uint32_t *>(ws + L.qkeys[k]);
        S.qstatus[k] = reinterpret_cast<uint32_t *>(ws + L.qstatus[k]);
    }
    S.qvals = reinterpret_cast<int32_t *>(ws + L.qvals);
    S.qhist = reinterpret_cast<uint32_t *>(ws + L.qhist);
    return S;
}

unsigned grid_for(int64_t items)
{
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g > kQueryGridMax) g = kQueryGridMax;
    return (unsigned)(g > 0 ? g : 1);
}

template <class Q>
hipError_t run_count(Tree tr, const float *q, int m, int64_t *offsets, char *ws,
                     const QueryLayout &L, hipStream_t s)
{
    Scratch S = carve(ws, L);
    tr.err = S.err;
    tr.budget = tune_get(TUNE_QBUDGET);
    const unsigned gm = grid_for(m);
    const int split1 = (int)tune_get(TUNE_QSPLIT1), split2 = (int)tune_get(TUNE_QSPLIT2);
    const bool order = tune_get(TUNE_QORDER) != 0 && m > 1;
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL(k_query_reset, dim3(gm), dim3(kBlock), 0, s, S.app_count, S.order_flag,
                       order ? 1 : 0, S.sort_ctr, S.qhist, S.err, S.cnt1, (int64_t)m);
    prof_end(K_QSPLIT, s);
    int64_t *const caller_offsets = offsets;
    if (order) {
        // sort the queries by key (two stable 8-bit passes), then copy them
        prof_begin(K_QORDER, s);
        const int64_t qtiles = ((int64_t)m + kQOrderTile - 1) / kQOrderTile;
        // few blocks, so that few global histogram adds meet on each word
        const unsigned gk = (unsigned)std::min<int64_t>(kQOrderKeyBlocks, (m + 16 * kBlock - 1) / (16 * kBlock));
        hipLaunchKernelGGL((k_qorder_keys<Q>), dim3(gk), dim3(kBlock), 0, s, tr, q, m, S.qkeys[0],
                           S.qhist, S.qstatus[0], qtiles * kRadix);
        const SortSegs one{nullptr, nullptr, 1, 0};
        hipLaunchKernelGGL((k_onesweep<uint32_t, 512, 4, kRadixBits>), dim3((unsigned)qtiles), dim3(512), 0, s,
                           S.qkeys[0], S.qkeys[1], nullptr, S.qvals, (int64_t)m, one, 0, kRadixBits, S.qhist,
                           S.qstatus[0], S.qstatus[1], (uint32_t)qtiles, S.sort_ctr + 0, S.err,
                           (const uint32_t *)nullptr);
        hipLaunchKernelGGL((k_onesweep<uint32_t, 512, 4, kRadixBits>), dim3((unsigned)qtiles), dim3(512), 0, s,
                           S.qkeys[1], S.qkeys[0], S.qvals, S.qperm, (int64_t)m, one, kRadixBits, kRadixBits,
                           S.qhist + kRadix, S.qstatus[1], nullptr, 0u, S.sort_ctr + 1, S.err,
                           (const uint32_t *)nullptr);
        hipLaunchKernelGGL((k_qorder_gather<Q>), dim3(gm), dim3(kBlock), 0, s, q, S.qperm, m,
                           S.qsorted);
        prof_end(K_QORDER, s);
        q = S.qsorted;
        offsets = S.qoff;
    }
    // level 1: queries -> pieces of 2^split1 leaves
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL((k_split<Q, true>), dim3(gm), dim3(kBlock), 0, s, tr, q, m, nullptr, nullptr,
                       split1, S.cnt1, S.app_count + 0, L.cap1, S.app_piece, S.app_item, S.app_rank);
    prof_end(K_QSPLIT, s);
    prof_begin(K_SCAN, s);
    scan(S.cnt1, m, nullptr, S.partials, S.off1, s);
    hipLaunchKernelGGL(k_level_check, dim3(1), dim3(1), 0, s, S.off1, nullptr, (int64_t)m,
                       S.ovf + 0, S.count + 0);
    prof_end(K_SCAN, s);
    prof_begin(K_QSPLIT, s);
    // (also clears the level-2 counts)
    hipLaunchKernelGGL(k_split_scatter<true>, dim3(grid_for(L.out1)), dim3(kBlock), 0, s, tr.n, m,
                       nullptr, nullptr, S.off1, S.cnt1, S.app_count + 0, L.cap1, S.app_piece,
                       S.app_item, S.app_rank, S.items1, S.cnt2, L.out1);
    prof_end(K_QSPLIT, s);
    // level 2: pieces -> pieces of 2^split2 leaves
    const unsigned g1 = grid_for(L.out1);
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL((k_split<Q, false>), dim3(g1), dim3(kBlock), 0, s, tr, q, m, S.items1,
                       S.count + 0, split2, S.cnt2, S.app_count + 1, L.cap2, S.app_piece, S.app_item,
                       S.app_rank);
    prof_end(K_QSPLIT, s);
    prof_begin(K_SCAN, s);
    scan(S.cnt2, L.out1, S.count + 0, S.partials, S.off2, s);
    hipLaunchKernelGGL(k_level_check, dim3(1), dim3(1), 0, s, S.off2, S.count + 0, (int64_t)0,
                       S.ovf + 1, S.count + 1);
    prof_end(K_SCAN, s);
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL(k_split_scatter<false>, dim3(grid_for(L.out2)), dim3(kBlock), 0, s, tr.n, m,
                       S.items1, S.count + 0, S.off2, S.cnt2, S.app_count + 1, L.cap2, S.app_piece,
                       S.app_item, S.app_rank, S.items2, nullptr, (int64_t)0);
    prof_end(K_QSPLIT, s);
    // leaf level: count hits per piece, scan, per-query offsets
    const unsigned g2 = grid_for(L.out2);
    prof_begin(K_QCOUNT, s);
    if (tune_get(TUNE_QLEAF) == 1)
        hipLaunchKernelGGL((k_leaf_mixed_count<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2,
                           S.count + 1, S.hcnt, S.hmask);
    else {
        hipLaunchKernelGGL((k_leaf_scan_count<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2,
                           S.count + 1, S.hcnt, S.hmask);
        hipLaunchKernelGGL((k_leaf_count_wide<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2,
                           S.count + 1, S.hcnt);
    }
    prof_end(K_QCOUNT, s);
    prof_begin(K_SCAN, s);
    scan(S.hcnt, L.out2, S.count + 1, S.partials, S.hoff, s);
    // with the order: also the per-query counts in the caller's order (in
    // cnt1, free since level 1)
    hipLaunchKernelGGL(k_compose, dim3((unsigned)((m + kBlock) / kBlock)), dim3(kBlock), 0, s, S.off1,
                       S.ovf + 0, S.off2, S.ovf + 1, S.hoff, m, offsets,
                       order ? S.qperm : nullptr, S.cnt1);
    prof_end(K_SCAN, s);
    if (order) {
        // back to the caller's order: the counts' scan, and each sorted
        // position's shift (in off1, free since the compose)
        prof_begin(K_QORDER, s);
        scan(S.cnt1, m, nullptr, S.partials, caller_offsets, s);
        hipLaunchKernelGGL(k_qorder_shift, dim3(gm), dim3(kBlock), 0, s, S.qoff, S.qperm,
                           caller_offsets, m, S.off1);
        prof_end(K_QORDER, s);
    }
    return hipGetLastError();
}

template <class Q>
hipError_t run_fill(const Tree &tr, const float *q, int32_t *indices, char *ws, const QueryLayout &L,
                    hipStream_t s)
{
    Scratch S = carve(ws, L);
    prof_begin(K_QFILL, s);
    const unsigned g2 = grid_for(L.out2);
    const QueryMap qm{S.order_flag, S.qsorted, S.off1};
    hipLaunchKernelGGL((k_leaf_fill<Q>), dim3(g2), dim3(kBlock), 0, s, tr, S.items2, S.count + 1,
                       S.hoff, S.hmask, qm, indices);
    hipLaunchKernelGGL((k_leaf_fill_wide<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2,
                       S.count + 1, S.hoff, qm, indices);
    prof_end(K_QFILL, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_query(int qkind, int kind, const lbvh_node *nodes, const int32_t *leaf_perm, int n,
                        const float *q, int m, int64_t *offsets, int32_t *indices, bool fill,
                        char *ws, const QueryLayout &L, hipStream_t s)
{
    if (n == 0 || m == 0) {
        if (fill) return hipSuccess;
        const int64_t cnt = (int64_t)m + 1;
        hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, offsets, cnt, reinterpret_cast<uint32_t *>(ws + L.ctrl + kQueryErrorByte));
        return hipGetLastError();
    }
    Tree tr{reinterpret_cast<const float4 *>(nodes), leaf_perm, n};
    tr.points = kind == LBVH_POINTS;
    if (fill) {
        if (qkind == 2) return run_fill<Ray>(tr, q, indices, ws, L, s);
        return qkind == 0 ? run_fill<Sphere>(tr, q, indices, ws, L, s)
                          : run_fill<QBox>(tr, q, indices, ws, L, s);
    }
    if (qkind == 2) return run_count<Ray>(tr, q, m, offsets, ws, L, s);
    return qkind == 0 ? run_count<Sphere>(tr, q, m, offsets, ws, L, s)
                      : run_count<QBox>(tr, q, m, offsets, ws, L, s);
}

hipError_t launch_ray_none(int64_t m, int32_t *hit, float *t, char *ws, const QueryLayout &L,
                           hipStream_t s)
{
    Scratch S = carve(ws, L);
    hipLaunchKernelGGL(k_ray_none, dim3(grid_for(m)), dim3(kBlock), 0, s, m, hit, t, S.err);
    return hipGetLastError();
}

hipError_t launch_ray_first(const lbvh_node *nodes, int n, const float *rays, int m, int32_t *hit,
                            float *t, char *ws, const QueryLayout &L, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    Scratch S = carve(ws, L);
    Tree tr{reinterpret_cast<const float4 *>(nodes), nullptr, n, S.err, tune_get(TUNE_QBUDGET)};
    prof_begin(K_QCOUNT, s);
    hipLaunchKernelGGL(k_query_reset, dim3(1), dim3(kBlock), 0, s, S.app_count, S.order_flag, 0,
                       S.sort_ctr, S.qhist, S.err, nullptr, (int64_t)0);
    hipLaunchKernelGGL(k_ray_first, dim3(grid_for(m)), dim3(kBlock), 0, s, tr, rays, m, hit, t);
    prof_end(K_QCOUNT, s);
    return hipGetLastError();
}

}  // namespace lbvh
