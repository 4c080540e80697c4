// Alg. 4, the bottom-up pass, run in levels of blocks; for one tree or for
// many independent trees (batched scenes) at once.
#pragma once
#pragma clang fp contract(off)

#include "device_common.hpp"

namespace lbvh {
namespace {

// Alg. 4 runs in levels of blocks so that every compare-and-swap on `store`
// has all of its possible participants inside one workgroup and needs only
// workgroup-scope ordering (an agent-scope acquire-release CAS per tree
// level would write back and invalidate the XCD's L2 every time):
//   level 0   block b takes the kChunk leaves [A, B) = [b*kChunk, ...):
//             leaf records, then the climb with `store`, delta* and every
//             box of the chunk in LDS;
//   level L   block b takes the kFanout level-(L-1) blocks under its span
//             [A, B) and resumes their handed-over threads, with `store` and
//             the node records in global memory.
// A block owns the boundaries strictly inside [A, B).  A thread whose next
// parent is split at A-1 or B-1 stops and hands its state (node, range) to
// the level above; that parent's other child cannot be finished inside this
// block.  Parents split inside [A, B) meet their two children either inside
// the block or in a later launch, and launches on one stream see all writes
// of earlier ones.  The top level is one block owning [0, n), so the climb
// always reaches the root.  Every internal node is still written once, by
// the second thread to arrive, exactly as in Alg. 4.

//
// A climb handed to the level above carries its whole state (a Climb:
// node, leaf range, rope, delta* at the range's two outer boundaries, box),
// so the level above starts it without a load.  A climb that arrives first
// at a split p parks there: `store[p]` gets its far end and, for trees of
// at most 2^24 leaves (PACKED), delta* at its outer boundary on that side
// in the same word.  The second arriver then learns both from its
// compare-and-swap, and takes the parked sibling's box and rope from the
// sibling's record, which it loads together with the CAS: the sibling is
// node p+1 (or p) as a leaf or as an internal node, so both candidate
// records are loaded and the CAS result picks one.  One global round trip
// per climb step.  (A parent's rope is its right child's: Alg. 2 makes a
// node's rope depend only on the right end of its range.)  Climbs that
// meet within one upper-level launch exchange their state through LDS:
// the first marks `store[p]` with its thread and leaves its state in its
// LDS slot, and at the end of the launch every such mark becomes the
// parked word for the levels above.  Larger trees keep the far end alone
// in `store` and read delta* from one byte per boundary that level 0 writes
// (`dstar`, in a buffer the sort no longer needs).
//
// Batched trees: every scene is its own problem (local leaf and node ids);
// its leaves sit at seg_off[s] in the sorted arrays and its 2n_s-1 node
// records at record 2*seg_off[s].  Level-L blocks of all scenes share one
// launch; blk_off[s] is the first level-L block of scene s.

struct BatchLevel {
    const int64_t *seg_off;    // [S+1] scene starts (leaves); nullptr: one tree
    const int32_t *blk_off;    // [S+1] first block of each scene at this level
    const int32_t *child_off;  // [S+1] first block of each scene one level down
    int S;
    int last;                  // top level: no climb may stop at a boundary
    const int32_t *order;      // top level of a batch (at most one block per
                               // scene): block b takes scene order[b], the
                               // largest scenes first; nullptr: scene order
};

struct Climb {
    int4 id;     // node, rl, rr, rope (node -1: empty slot)
    float4 lo;   // lo.xyz; w: delta*(rl-1) | delta*(rr) << 8, as bits
    float4 hi;   // hi.xyz; w: 0
};

__device__ __forceinline__ Climb make_climb(int node, int rl, int rr, int rope, int dl, int dr,
                                            const float lo[3], const float hi[3])
{
    Climb c;
    c.id = make_int4(node, rl, rr, rope);
    c.lo = make_float4(lo[0], lo[1], lo[2], __int_as_float(dl | (dr << 8)));
    c.hi = make_float4(hi[0], hi[1], hi[2], 0.0f);
    return c;
}

__device__ __forceinline__ Climb empty_climb()
{
    Climb c;
    c.id = make_int4(-1, 0, 0, 0);
    c.lo = c.hi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return c;
}

// Packed `store` word: far end in bits 0..23, delta* in bits 24..30.  delta*
// ranks are at most 64 + 62 = 126 for codes and 29 for indices, so 127 can
// stand for +inf (255); bit 31 stays clear, so no packed word is the empty
// marker -1 or a same-launch mark (bit 31 set).
constexpr int kPackedMaxN = 1 << 24;
__device__ __forceinline__ int32_t pack_park(int far, int d) { return far | ((d > 127 ? 127 : d) << 24); }
__device__ __forceinline__ int park_far(int32_t v) { return v & 0xFFFFFF; }
__device__ __forceinline__ int park_delta(int32_t v)
{
    const int d = (v >> 24) & 127;
    return d == 127 ? 255 : d;
}

// min and max of two canonical floats (no signalling NaN): the hardware
// instruction alone.  fminf / fmaxf first quiet both operands (one more
// instruction each), which the merge loop below does not need: every box in
// its LDS copy is either a leaf box quieted once on load or a result of
// these operations.  Same results as fminf / fmaxf on such operands.
__device__ __forceinline__ float min_canon(float a, float b)
{
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float max_canon(float a, float b)
{
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int scene_of(const int32_t *off, int S, int b)
{
    int lo = 0, hi = S - 1;   // largest s with off[s] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int KIND, typename K, bool PACKED>
__global__ __launch_bounds__(kBU0Threads) void k_bottomup_l0(const K *__restrict__ codes_all,
                                                             const int32_t *__restrict__ perm_all,
                                                             const float *__restrict__ prims_all,
                                                             int n_all, int32_t *__restrict__ store_all,
                                                             float4 *__restrict__ nodes_all,
                                                             Climb *__restrict__ pend, BatchLevel bl,
                                                             uint8_t *__restrict__ dstar_all,
                                                             uint32_t *err)
{
    __shared__ K s_codes[kChunk + 3];        // codes[A-1 .. B+1]
    __shared__ uint8_t s_delta[kChunk + 2];  // delta*(g) for g in [A-1, B]
    __shared__ int32_t s_store[kChunk];      // store[A .. B-1]
    __shared__ float s_box[6][2 * kChunk];   // internal A.. then leaves A..
    __shared__ Climb s_pend[2];

    // this block's chunk: tree (codes, perm, ... of one scene), leaves [A, B)
    int64_t b0 = 0;
    int n = n_all, c = blockIdx.x;
    if (bl.seg_off) {
        if ((int)blockIdx.x >= bl.blk_off[bl.S]) return;   // grid is an upper bound
        const int s = scene_of(bl.blk_off, bl.S, blockIdx.x);
        b0 = bl.seg_off[s];
        n = (int)(bl.seg_off[s + 1] - b0);
        c = blockIdx.x - bl.blk_off[s];
    }
    const K *codes = codes_all + b0;
    const int32_t *perm = perm_all + b0;
    const float *prims = prims_all + b0 * (KIND == LBVH_POINTS ? 3 : 6);
    int32_t *store = store_all + b0;
    float4 *nodes = nodes_all + 4 * b0;   // record 2*b0, two float4 per record
    const int A = c * kChunk;
    const int B = min(A + kChunk, n);
    const int cn = B - A;
    const int leaf0 = n - 1;
    const int tid = threadIdx.x;

    for (int t = tid; t < cn + 3; t += kBU0Threads) {
        const int g = A - 1 + t;
        s_codes[t] = (g >= 0 && g < n) ? codes[g] : (K)0;
    }
    s_store[tid] = -1;
    if (tid < 2) s_pend[tid] = empty_climb();
    // this thread's leaf i: primitive id and box (a gather), loaded while
    // the codes arrive
    const int i = A + tid;
    int prim = 0;
    float lo[3], hi[3];
    if (i < B) {
        prim = perm[i];
        Prims<KIND>::one(prims, prim, lo, hi);
    }
    __syncthreads();

    // delta*(g) for g in [A-1, B], from the codes in LDS: the rank of the
    // highest differing bit of the augmented keys (code, sorted position) of
    // leaves g and g+1, codes ranking above any index bit; +inf (255) for
    // g = -1 and g = n-1
    auto delta_codes = [&](int g) -> int {
        if (g < 0 || g >= n - 1) return 255;
        const K x = s_codes[g - A + 1] ^ s_codes[g - A + 2];
        if (x) return 64 + highest_bit(x);
        return highest_bit((uint32_t)(g ^ (g + 1)));
    };
    for (int t = tid; t < cn + 2; t += kBU0Threads) s_delta[t] = (uint8_t)delta_codes(A - 1 + t);
    // the leaf's box as the merges below use it: quieted once
    float clo[3], chi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        clo[a] = __builtin_canonicalizef(lo[a]);
        chi[a] = __builtin_canonicalizef(hi[a]);
    }
    if (i < B) {
        const int sl = kChunk + tid;
#pragma unroll
        for (int a = 0; a < 3; ++a) { s_box[a][sl] = clo[a]; s_box[3 + a][sl] = chi[a]; }
    }
    __syncthreads();
    auto delta = [&](int g) -> int { return s_delta[g - A + 1]; };
    // leaf record: the box as given, primitive id, rope (Alg. 2 on the
    // range [i, i]; delta*(i + 1) is in the table, i + 1 <= B)
    int rope = -1;
    if (i < B) {
        rope = (i == n - 1) ? -1 : (delta(i) < delta(i + 1) ? leaf0 + i + 1 : i + 1);
        store_node(nodes, leaf0 + i, lo, prim, hi, rope);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) { lo[a] = clo[a]; hi[a] = chi[a]; }

    // Alg. 4's climb.  Both cases (the node is its parent's left or right
    // child) run the same instructions with selects, so a wave whose lanes
    // disagree does not run both.
    // this chunk's boundaries g in [A, B), g < n-1, for the upper levels of
    // a tree whose store words cannot carry delta*
    if (!PACKED && i < B && i < n - 1) dstar_all[b0 + i] = s_delta[tid + 1];
    if (n > 1 && i < B) {
        int rl = i, rr = i, cur = leaf0 + i;
        int dl = delta(i - 1), dr = delta(i);
        // one exit for the whole wave (a lane stops when it parks at a
        // chunk edge, is first at its parent, or reaches the root), so the
        // loop keeps no per-exit lane masks
        bool live = true, edge = false;
        int level = 0;
        do {
            if (live) {
                const bool is_left = dr < dl;              // left child of its parent
                const int p = is_left ? rr : rl - 1;       // the parent's split
                if (level == kMaxDepth) {
                    __hip_atomic_store(err, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    live = false;
                } else if (p == (is_left ? B - 1 : A - 1)) {   // the parent is split at a chunk edge
                    edge = true;
                    live = false;
                } else {
                    int other = -1;
                    const int far_mine = is_left ? rl : rr;   // this node's far end, seen from p
                    const int32_t park = PACKED ? pack_park(far_mine, is_left ? dl : dr) : far_mine;
                    if (__hip_atomic_compare_exchange_strong(&s_store[p - A], &other, park,
                                                             __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        live = false;                          // first to arrive
                    } else {
                        // second to arrive: `other` holds the sibling's far end
                        const int far = PACKED ? park_far(other) : other;
                        rr = is_left ? far : rr;
                        rl = is_left ? rl : far;
                        const int dn = delta(is_left ? rr : rl - 1);
                        dr = is_left ? dn : dr;
                        dl = is_left ? dl : dn;
                        // the sibling: leaf or internal node at split-side
                        // index sp (selects, not branches); its LDS slot
                        const int sp = is_left ? p + 1 : p;
                        const bool sleaf = is_left ? (sp == rr) : (sp == rl);
                        const int ss = sleaf ? kChunk + (sp - A) : sp - A;
                        // delta*(rr + 1): rr + 1 <= B, in the LDS table (255 at n - 1)
                        const int d_next = delta(rr + 1);
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            lo[a] = min_canon(lo[a], s_box[a][ss]);
                            hi[a] = max_canon(hi[a], s_box[3 + a][ss]);
                        }
                        const int q = dr < dl ? rr : rl;   // Karras index of the parent
                        const int left = (rl == p) ? leaf0 + p : p;
                        const int qrope = rr == n - 1 ? -1 : (dr < d_next ? leaf0 + rr + 1 : rr + 1);
                        store_node(nodes, q, lo, left, hi, qrope);
                        const int qs = q - A;
#pragma unroll
                        for (int a = 0; a < 3; ++a) { s_box[a][qs] = lo[a]; s_box[3 + a][qs] = hi[a]; }
                        cur = q;
                        rope = qrope;
                        live = q != 0;
                    }
                }
                ++level;
            }
        } while (__ballot(live) != 0);
        if (edge) s_pend[dr < dl ? 1 : 0] = make_climb(cur, rl, rr, rope, dl, dr, lo, hi);
    }
    __syncthreads();
    if (tid < cn) store[A + tid] = s_store[tid];
    if (tid < 2) {
        // field by field: a whole-struct copy around the atomic goes through
        // scratch memory, and scratch in any part of a kernel costs every wave
        const int4 id = s_pend[tid].id;
        const float4 slo = s_pend[tid].lo, shi = s_pend[tid].hi;
        if (bl.last && id.x >= 0)   // a climb stopped below the root of its tree
            __hip_atomic_store(err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Climb *o = pend + 2 * (int64_t)blockIdx.x + tid;
        o->id = id;
        o->lo = slo;
        o->hi = shi;
    }
}

template <bool PACKED>
__global__ __launch_bounds__(kBUThreads) void k_bottomup_up(const uint8_t *__restrict__ dstar_all,
                                                            int n_all, int64_t child_span, int64_t span,
                                                            int32_t *store_all, float4 *nodes_all,
                                                            const Climb *__restrict__ pend_in,
                                                            Climb *__restrict__ pend_out, BatchLevel bl,
                                                            uint32_t *err)
{
    // a climb parked in this launch: lo.xyz + far end (packed with delta*
    // if PACKED), hi.xyz + rope; delta* apart otherwise
    __shared__ float4 s_state[kBUThreads][2];
    __shared__ uint8_t s_dfar[PACKED ? 1 : kBUThreads];
    __shared__ Climb s_pend[2];
    // this block's span [A, B) of one tree and the handed-over slots of its
    // child blocks
    int64_t b0 = 0, slot_lo, slot_hi, A, B;
    int n = n_all;
    int lb = blockIdx.x;   // this block's number at its level (its hand-over slots)
    if (bl.seg_off) {
        int s;
        if (bl.order) {
            if ((int)blockIdx.x >= bl.S) return;
            s = bl.order[blockIdx.x];
            const int nb = bl.blk_off[s + 1] - bl.blk_off[s];
            if (nb == 0) return;   // the scene's tree is complete below this level
            if (nb > 1) {          // not expected: the top level has one block a scene
                if (threadIdx.x == 0) __hip_atomic_store(err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            lb = bl.blk_off[s];
        } else {
            if ((int)blockIdx.x >= bl.blk_off[bl.S]) return;
            s = scene_of(bl.blk_off, bl.S, blockIdx.x);
        }
        b0 = bl.seg_off[s];
        n = (int)(bl.seg_off[s + 1] - b0);
        const int g = lb - bl.blk_off[s];
        const int nchild = bl.child_off[s + 1] - bl.child_off[s];
        const int c0 = g * kFanout, c1 = min(c0 + kFanout, nchild);
        A = (int64_t)c0 * child_span;
        B = min(A + span, (int64_t)n);
        slot_lo = 2 * ((int64_t)bl.child_off[s] + c0);
        slot_hi = 2 * ((int64_t)bl.child_off[s] + c1);
    } else {
        A = (int64_t)blockIdx.x * span;
        B = A + span < n ? A + span : n;
        slot_lo = 2 * (A / child_span);
        slot_hi = 2 * ((B + child_span - 1) / child_span);
    }
    const uint8_t *dstar = dstar_all + b0;
    int32_t *store = store_all + b0;
    float4 *nodes = nodes_all + 4 * b0;
    const int leaf0 = n - 1;
    const int tid = threadIdx.x;
    // delta*(g), +inf (255) outside [0, n-2], as level 0 stored it
    auto delta = [&](int g) -> int { return (g < 0 || g >= n - 1) ? 255 : (int)dstar[g]; };
    if (tid < 2) s_pend[tid] = empty_climb();
    __syncthreads();

    int park_at = -1;      // the split this thread parked at in this launch
    int32_t park_word = 0; // ... and the store word the levels above read
    // at most kFanout child blocks, two slots each: one per thread
    const int64_t slot = slot_lo + tid;
    if (slot < slot_hi) {
        const Climb c = pend_in[slot];
        int cur = c.id.x, rl = c.id.y, rr = c.id.z, rope = c.id.w;
        const int dd = __float_as_int(c.lo.w);
        int dl = dd & 0xff, dr = (dd >> 8) & 0xff;
        float lo[3] = {c.lo.x, c.lo.y, c.lo.z}, hi[3] = {c.hi.x, c.hi.y, c.hi.z};
        for (int level = 0; cur >= 0; ++level) {
            if (level == kMaxDepth) {
                __hip_atomic_store(err, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            const bool is_left = dr < dl;              // left child of its parent
            const int p = is_left ? rr : rl - 1;       // the parent's split
            if (p == (is_left ? B - 1 : A - 1)) {      // split at this block's edge
                s_pend[is_left ? 1 : 0] = make_climb(cur, rl, rr, rope, dl, dr, lo, hi);
                break;
            }
            // a sibling parked by a lower level is node ci (internal) or
            // leaf ci: load both records while the CAS is in flight
            const int ci = is_left ? p + 1 : p;        // <= n-1: in bounds either way
            const float4 *ip = nodes + 2 * (int64_t)ci, *lp = nodes + 2 * (int64_t)(leaf0 + ci);
            const float4 i0 = ip[0], i1 = ip[1], l0 = lp[0], l1 = lp[1];
            // publish this climb's state for a sibling in this launch, then
            // claim p with this thread's mark
            const int far_mine = is_left ? rl : rr;
            const int d_mine = is_left ? dl : dr;
            const int32_t word = PACKED ? pack_park(far_mine, d_mine) : far_mine;
            s_state[tid][0] = make_float4(lo[0], lo[1], lo[2], __int_as_float(word));
            s_state[tid][1] = make_float4(hi[0], hi[1], hi[2], __int_as_float(rope));
            if (!PACKED) s_dfar[PACKED ? 0 : tid] = (uint8_t)d_mine;
            int other = -1;
            if (__hip_atomic_compare_exchange_strong(&store[p], &other, (int32_t)(0x80000000u | tid),
                                                     __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
                park_at = p;                           // first to arrive
                park_word = word;
                break;
            }
            int far, dfar;
            float4 s0, s1;
            if (other < 0) {                           // parked in this launch: LDS
                const int t = other & 0x7fffffff;
                s0 = s_state[t][0];
                s1 = s_state[t][1];
                const int w = __float_as_int(s0.w);
                far = PACKED ? park_far(w) : w;
                dfar = PACKED ? park_delta(w) : (int)s_dfar[PACKED ? 0 : t];
            } else {                                   // parked by a lower level
                far = PACKED ? park_far(other) : other;
                dfar = PACKED ? park_delta(other) : delta(is_left ? far : far - 1);
                const bool leaf_sib = is_left ? (far == p + 1) : (far == p);
                s0 = leaf_sib ? l0 : i0;
                s1 = leaf_sib ? l1 : i1;
            }
            rr = is_left ? far : rr;
            rl = is_left ? rl : far;
            dr = is_left ? dfar : dr;
            dl = is_left ? dl : dfar;
            rope = is_left ? __float_as_int(s1.w) : rope;   // the right child's
            lo[0] = fminf(lo[0], s0.x); lo[1] = fminf(lo[1], s0.y); lo[2] = fminf(lo[2], s0.z);
            hi[0] = fmaxf(hi[0], s1.x); hi[1] = fmaxf(hi[1], s1.y); hi[2] = fmaxf(hi[2], s1.z);
            const int q = dr < dl ? rr : rl;           // Karras index of the parent
            const int left = (rl == p) ? leaf0 + p : p;
            store_node(nodes, q, lo, left, hi, rope);
            cur = q;
            if (q == 0) break;
        }
    }
    __syncthreads();
    // every climb parked in this launch leaves its word for the levels
    // above (a consumed one is never read again)
    if (park_at >= 0) store[park_at] = park_word;
    if (tid < 2) {
        const int4 id = s_pend[tid].id;
        const float4 slo = s_pend[tid].lo, shi = s_pend[tid].hi;
        if (bl.last && id.x >= 0)
            __hip_atomic_store(err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Climb *o = pend_out + 2 * (int64_t)lb + tid;
        o->id = id;
        o->lo = slo;
        o->hi = shi;
    }
}

}  // namespace
}  // namespace lbvh
