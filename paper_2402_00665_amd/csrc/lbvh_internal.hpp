// Internal declarations shared by the library's HIP translation units:
// workspace layout, tuning constants, launcher prototypes and the
// per-kernel timing hooks.  Not part of the public C ABI (include/lbvh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

#include "lbvh.h"

namespace lbvh {

// ------------------------------------------------------------ constants

constexpr int kBlock = 256;           // threads per block of the simple kernels
constexpr int kRadixBits = 8;         // digit width of the query-order sort (16-bit keys)
constexpr int kRadix = 1 << kRadixBits;
constexpr int kBoundsBlocksMax = 1024;
constexpr int kMortonBlocksMax = 2048;
constexpr int kChunk = 1024;          // leaves per level-0 block of the bottom-up pass
constexpr int kBU0Threads = kChunk;     // one leaf per thread
constexpr int kFanout = 256;          // level-(L-1) blocks per level-L block
constexpr int kBUThreads = 2 * kFanout;  // one thread per handed-over climb
constexpr int kClimbBytes = 48;       // a climb handed between bottom-up levels
constexpr int kMaxBatchLevels = 3;    // kChunk * kFanout^3 >= LBVH_MAX_PRIMS
constexpr int kScanItems = 8;         // values per thread in the query scan
constexpr int kSplit1 = 12;           // default: query walks cut by aligned blocks of 2^12 leaves
constexpr int kSplit2 = 7;            // default: ... then by blocks of 2^7 leaves
constexpr int kQueryGridMax = 8192;   // blocks of the grid-stride query kernels
constexpr int kQOrderTile = 2048;     // keys per tile of the query-order sort (512 x 4)
constexpr int kQOrderPasses = 2;      // 16-bit query-order keys: two 8-bit digits
constexpr int kQOrderKeyBlocks = 256;  // blocks of the query-order key kernel
constexpr int kMaskLeaves = 256;     // widest level-2 piece that gets a leaf-hit mask
constexpr int kMaskWords = kMaskLeaves / 64;
constexpr int kScanTile = kBlock * kScanItems;

// the error word of a query call: byte offset in the query workspace's ctrl
// area (single tree and batched); nonzero after a count call means its
// results are not to be trusted (lbvh_query_check)
constexpr int kQueryErrorByte = 24;

// ctrl words at the start of the build workspace
constexpr int kCtrlTileCounter = 0;   // [0, 8): one per sort pass
constexpr int kCtrlError = 8;         // non-zero: a kernel flagged an error
constexpr int kCtrlWords = 64;

// look-back status word: 2 flag bits over a 30-bit count
constexpr uint32_t kFlagAggregate = 1u << 30;
constexpr uint32_t kFlagInclusive = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1u;

// Digit widths of the build's LSD radix sort (knobs radix_bits32 and
// radix_bits64): 8 or 10 bits for 30-bit codes, 8, 9 or 11 for 63-bit.
// Wider digits mean fewer passes over the keys, larger per-tile digit
// tables.  A pass's tile holds at least radix_min_tile(bits) keys, which
// bounds the look-back tables at half a status word per key.
inline bool radix_bits_ok(int code_bits, int bits)
{
    return code_bits <= 32 ? (bits == 8 || bits == 10) : (bits == 8 || bits == 9 || bits == 11);
}
inline int radix_passes(int code_bits, int bits) { return (code_bits + bits - 1) / bits; }
inline int radix_min_tile(int bits) { return bits >= 11 ? 4096 : 2048; }
// words of the digit histograms of all passes, the largest over the widths
// a code width allows (so a workspace fits every width)
inline int64_t radix_hist_words(int code_bits)
{
    int64_t w = 0;
    for (int b = 8; b <= 11; ++b)
        if (radix_bits_ok(code_bits, b)) w = std::max<int64_t>(w, (int64_t)radix_passes(code_bits, b) << b);
    return w;
}
// words of one look-back table for `tiles(min_tile)` tiles, the largest
// over the allowed widths; `extra_tiles` partial tiles (one per scene of a
// batch) on top
inline int64_t radix_status_words(int64_t n, int code_bits, int64_t extra_tiles)
{
    int64_t w = 0;
    for (int b = 8; b <= 11; ++b)
        if (radix_bits_ok(code_bits, b)) {
            const int64_t t = (n + radix_min_tile(b) - 1) / radix_min_tile(b) + extra_tiles;
            w = std::max<int64_t>(w, t << b);
        }
    return w;
}
int radix_bits(int code_bits);   // the knob's current width for this code width
inline int key_bytes(int code_bits) { return code_bits <= 32 ? 4 : 8; }

// --------------------------------------------------- workspace layout

struct BuildLayout {
    size_t scene;      // float4 lo, hi, scale (48 B)
    size_t partials;   // kBoundsBlocksMax x 8 floats
    size_t ctrl;       // kCtrlWords uint32
    size_t hist;       // radix_hist_words uint32 (global digit counts of every pass)
    size_t status[2];  // radix_status_words uint32 each (ping-pong look-back)
    size_t keys_alt;   // n keys (sort ping-pong partner of tree->codes)
    size_t vals[2];    // n int32 each (sort values: input indices)
    size_t store;      // n int32 (Alg. 4 arrival flags / parked range ends)
    size_t pend[2];    // handed-over climbs between bottom-up levels (kClimbBytes each)
    size_t total;
};

BuildLayout build_layout(int64_t n, int code_bits);

struct QueryLayout {
    int64_t cap1, cap2;  // capacities of the level-1 and level-2 append lists
    int64_t out1, out2;  // pieces each level can emit: its list plus one per unsplit item
    size_t cnt1;       // m int32: level-1 pieces per query
    size_t off1;       // m+1 int64
    size_t items1;     // out1 int4 (query, node, left bound, range end)
    size_t cnt2;       // out1 int32: level-2 pieces per level-1 piece
    size_t off2;       // out1+1 int64
    size_t items2;     // out2 int4
    size_t app_piece;  // cap2 int4: pieces appended by a split level's count pass
    size_t app_item;   // cap2 int64: ... the item each came from
    size_t app_rank;   // cap2 int32: ... and its rank among that item's pieces
    size_t hcnt;       // out2 int32: hits per level-2 piece
    size_t hmask;      // out2 x kMaskWords uint64: leaf-hit mask of each level-2 piece
    size_t hcache;     // batched: m x 64 int32, each query's first hits
    size_t hoff;       // out2+1 int64
    size_t partials;   // scan tile sums
    size_t ctrl;       // overflow flags, piece counts, query-order flag, sort counters, error word
    // query order (single tree): the reordered copy of the queries, each
    // reordered position's caller index, and the offsets in reordered order
    size_t qsorted;    // m x 8 float (the widest query, a ray)
    size_t qperm;      // m int32
    size_t qoff;       // m+1 int64
    // the order's radix sort, inside `hmask` (unused until the leaf level)
    size_t qkeys[2];   // m uint32 each
    size_t qvals;      // m int32 (first pass's values)
    size_t qstatus[2]; // qtiles x kRadix uint32 each
    size_t qhist;      // 2 x kRadix uint32
    size_t total;
};

QueryLayout query_layout(int64_t m);
QueryLayout batch_query_layout(int64_t m);   // counts, first hits, scan sums

struct BatchLayout {
    size_t ctrl;       // kCtrlWords uint32
    size_t scene_box;  // S x 3 float4 (lo, hi, scale)
    size_t tile_off;   // S+1 int32
    size_t order;      // S int32: scenes in decreasing size class (one-block-per-scene sort)
    size_t blk_off;    // (levels+1) x (S+1) int32
    size_t hist;       // S x radix_hist_words uint32
    size_t status[2];  // radix_status_words(N, bits, S) uint32 each
    size_t keys_alt;   // N keys
    size_t vals[2];    // N int32
    size_t store;      // N int32
    size_t pend[2];    // 2 x blocks_max[0] handed-over climbs
    size_t total;
    int levels;
    int64_t blocks_max[kMaxBatchLevels + 1]; // upper bound of bottom-up blocks per level
};

BatchLayout batch_layout(int64_t total_n, int S, int64_t max_scene, int code_bits);
int batch_levels(int64_t max_scene);

// ------------------------------------------------------------ tuning
// Launch-shape knobs read by the launchers; set through lbvh_tune.

enum TuneKnob {
    TUNE_SORT_VARIANT32 = 0, TUNE_SORT_VARIANT64, TUNE_BATCH_SORT, TUNE_QSPLIT1, TUNE_QSPLIT2, TUNE_QLEAF, TUNE_QORDER,
    TUNE_RADIX_BITS32, TUNE_RADIX_BITS64, TUNE_QBUDGET, TUNE_MORTON_ORDER, TUNE_BATCH_SORT_MODE,
    TUNE_RADIX_MODE,
    TUNE_NUM
};
int64_t tune_get(int knob);

// ------------------------------------------------------------ timing

enum KernelId {
    K_BOUNDS = 0, K_BOUNDS_FINAL, K_MORTON, K_SORT, K_BOTTOMUP,
    K_QCOUNT, K_QFILL, K_SCAN, K_QSPLIT, K_BOTTOMUP_UP, K_BATCH_PREP, K_QORDER, K_NUM
};

void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);

// ---------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  Arguments are already
// validated by the C ABI layer.

hipError_t launch_build(int kind, const float *prims, int n, int code_bits,
                        lbvh_node *nodes, void *codes, int32_t *leaf_perm, char *ws,
                        const BuildLayout &L, hipStream_t s);

// kind: the tree's primitives (LBVH_POINTS lets the leaf scan read half of
// each leaf record)
hipError_t launch_query(int qkind, int kind, const lbvh_node *nodes, const int32_t *leaf_perm, int n,
                        const float *q, int m, int64_t *offsets,
                        int32_t *indices, bool fill, char *ws,
                        const QueryLayout &L, hipStream_t s);

hipError_t launch_build_batched(int kind, const float *prims, const lbvh_batch *b, int levels,
                                char *ws, const BatchLayout &L, hipStream_t s);

// first hit of each ray (Alg. 1 pruned on the entry parameter)
hipError_t launch_ray_first(const lbvh_node *nodes, int n, const float *rays, int m, int32_t *hit,
                            float *t, char *ws, const QueryLayout &L, hipStream_t s);
// ... on an empty tree: every ray misses
hipError_t launch_ray_none(int64_t m, int32_t *hit, float *t, char *ws, const QueryLayout &L,
                           hipStream_t s);

hipError_t launch_query_batched(int qkind, const lbvh_batch *b, const float *q,
                                const int64_t *qseg_off, int64_t m, int64_t *offsets,
                                int32_t *indices, bool fill, char *ws, const QueryLayout &L,
                                hipStream_t s);

}  // namespace lbvh
