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

namespace lbvh {
namespace {

struct Scratch {
    int32_t *cnt1, *cnt2, *hcnt, *ovf;
    int64_t *off1, *off2, *hoff, *partials, *count;
    int4 *items1, *items2, *app_piece;
    int64_t *app_item;
    int32_t *app_rank;
    unsigned long long *app_count;
    uint64_t *hmask;
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
    return S;
}

unsigned grid_for(int64_t items)
{
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g > kQueryGridMax) g = kQueryGridMax;
    return (unsigned)(g > 0 ? g : 1);
}

template <class Q>
hipError_t run_count(const Tree &tr, const float *q, int m, int64_t *offsets, char *ws,
                     const QueryLayout &L, hipStream_t s)
{
    Scratch S = carve(ws, L);
    const unsigned gm = grid_for(m);
    const int split1 = (int)tune_get(TUNE_QSPLIT1), split2 = (int)tune_get(TUNE_QSPLIT2);
    // level 1: queries -> pieces of 2^split1 leaves
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL(k_split_reset, dim3(1), dim3(64), 0, s, S.app_count);
    hipLaunchKernelGGL((k_split<Q, true>), dim3(gm), dim3(kBlock), 0, s, tr, q, m, nullptr, nullptr,
                       split1, S.cnt1, S.app_count + 0, L.cap1, S.app_piece, S.app_item, S.app_rank);
    prof_end(K_QSPLIT, s);
    prof_begin(K_SCAN, s);
    scan(S.cnt1, m, nullptr, S.partials, S.off1, s);
    hipLaunchKernelGGL(k_level_check, dim3(1), dim3(1), 0, s, S.off1, nullptr, (int64_t)m, L.cap1,
                       S.ovf + 0, S.count + 0);
    prof_end(K_SCAN, s);
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL(k_split_scatter<true>, dim3(grid_for(L.cap1)), dim3(kBlock), 0, s, tr.n, m,
                       nullptr, nullptr, S.off1, S.ovf + 0, S.app_count + 0, S.app_piece, S.app_item,
                       S.app_rank, S.items1);
    prof_end(K_QSPLIT, s);
    // level 2: pieces -> pieces of 2^split2 leaves
    const unsigned g1 = grid_for(L.cap1);
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL((k_split<Q, false>), dim3(g1), dim3(kBlock), 0, s, tr, q, m, S.items1,
                       S.count + 0, split2, S.cnt2, S.app_count + 1, L.cap2, S.app_piece, S.app_item,
                       S.app_rank);
    prof_end(K_QSPLIT, s);
    prof_begin(K_SCAN, s);
    scan(S.cnt2, L.cap1, S.count + 0, S.partials, S.off2, s);
    hipLaunchKernelGGL(k_level_check, dim3(1), dim3(1), 0, s, S.off2, S.count + 0, (int64_t)0, L.cap2,
                       S.ovf + 1, S.count + 1);
    prof_end(K_SCAN, s);
    prof_begin(K_QSPLIT, s);
    hipLaunchKernelGGL(k_split_scatter<false>, dim3(grid_for(L.cap2)), dim3(kBlock), 0, s, tr.n, m,
                       S.items1, S.count + 0, S.off2, S.ovf + 1, S.app_count + 1, S.app_piece,
                       S.app_item, S.app_rank, S.items2);
    prof_end(K_QSPLIT, s);
    // leaf level: count hits per piece, scan, per-query offsets
    const unsigned g2 = grid_for(L.cap2);
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
    scan(S.hcnt, L.cap2, S.count + 1, S.partials, S.hoff, s);
    hipLaunchKernelGGL(k_compose, dim3((unsigned)((m + kBlock) / kBlock)), dim3(kBlock), 0, s, S.off1,
                       S.ovf + 0, S.off2, S.ovf + 1, S.hoff, m, offsets);
    prof_end(K_SCAN, s);
    return hipGetLastError();
}

template <class Q>
hipError_t run_fill(const Tree &tr, const float *q, int32_t *indices, char *ws, const QueryLayout &L,
                    hipStream_t s)
{
    Scratch S = carve(ws, L);
    prof_begin(K_QFILL, s);
    const unsigned g2 = grid_for(L.cap2);
    hipLaunchKernelGGL((k_leaf_fill<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2, S.count + 1,
                       S.hoff, S.hmask, indices);
    hipLaunchKernelGGL((k_leaf_fill_wide<Q>), dim3(g2), dim3(kBlock), 0, s, tr, q, S.items2,
                       S.count + 1, S.hoff, indices);
    prof_end(K_QFILL, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_query(int qkind, const lbvh_node *nodes, const int32_t *leaf_perm, int n,
                        const float *q, int m, int64_t *offsets, int32_t *indices, bool fill,
                        char *ws, const QueryLayout &L, hipStream_t s)
{
    if (n == 0 || m == 0) {
        if (fill) return hipSuccess;
        const int64_t cnt = (int64_t)m + 1;
        hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, offsets, cnt);
        return hipGetLastError();
    }
    Tree tr{reinterpret_cast<const float4 *>(nodes), leaf_perm, n};
    if (fill)
        return qkind == 0 ? run_fill<Sphere>(tr, q, indices, ws, L, s)
                          : run_fill<QBox>(tr, q, indices, ws, L, s);
    return qkind == 0 ? run_count<Sphere>(tr, q, m, offsets, ws, L, s)
                      : run_count<QBox>(tr, q, m, offsets, ws, L, s);
}

}  // namespace lbvh
