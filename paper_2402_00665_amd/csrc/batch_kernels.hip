// Batched construction and queries: S independent scenes (each with its
// own scene box, Morton codes, sort and tree) built by one launch sequence
// that covers all of them, instead of one launch sequence per scene.
//
//   k_batch_plan     one block: per-scene radix tiles and bottom-up blocks
//                    per level (exclusive scans over the scenes), counters
//   k_batch_morton   one block per scene: scene box and scale, Morton codes,
//                    digit histograms of scenes that span several tiles
//   k_onesweep       segmented radix passes (tiles never cross scenes)
//   k_bottomup_*     Alg. 4 in levels of blocks, blocks never cross scenes
//   k_batch_count / k_batch_fill
//                    Alg. 1 per query on the tree of the query's scene
//
// Every scene's tree is exactly the tree a single build of that scene gives
// (local leaf, node and primitive ids), stored at record 2*seg_off[s].
#pragma clang fp contract(off)

#include "bottomup.hpp"
#include "device_common.hpp"
#include "query_common.hpp"
#include "radix_sort.hpp"

namespace lbvh {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int kSceneThreads = 512;

__device__ __forceinline__ int64_t scene_size(const int64_t *seg_off, int s)
{
    return seg_off[s + 1] - seg_off[s];
}

// Exclusive scans over scenes of: radix tiles per scene, and bottom-up
// blocks per scene at levels 0..levels (a scene needs a level-L block only
// while its level-(L-1) blocks are more than one).  Also clears the control
// words (tile counters, error flag).
__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(const int64_t *__restrict__ seg_off,
                                                             int S, int levels, int tile,
                                                             int32_t *__restrict__ tile_off,
                                                             int32_t *__restrict__ blk_off,
                                                             uint32_t *__restrict__ ctrl,
                                                             int32_t *__restrict__ order)
{
    __shared__ uint32_t sh[kPlanThreads / 64];
    __shared__ uint32_t s_total;
    __shared__ uint32_t s_len[32];   // scenes per bit length of their size, then cursors
    if (threadIdx.x < 32) s_len[threadIdx.x] = 0u;
    for (int w = threadIdx.x; w < kCtrlWords; w += kPlanThreads) ctrl[w] = 0u;
    uint32_t carry_t = 0;
    uint32_t carry_b[kMaxBatchLevels + 1] = {};
    for (int c = 0; c < S; c += kPlanThreads) {
        const int s = c + threadIdx.x;
        // exclusive scan of v over the scenes, continued across chunks
        auto scan_into = [&](uint32_t v, int32_t *dst, uint32_t &carry) {
            const uint32_t e = block_excl_scan<kPlanThreads>(v, sh);
            if (s < S) dst[s] = (int32_t)(carry + e);
            if (threadIdx.x == kPlanThreads - 1) s_total = e + v;
            __syncthreads();
            carry += s_total;
            __syncthreads();
        };
        const int64_t ns = s < S ? scene_size(seg_off, s) : 0;
        scan_into((uint32_t)((ns + tile - 1) / tile), tile_off, carry_t);
        uint32_t blk = (uint32_t)((ns + kChunk - 1) / kChunk);
        for (int L = 0; L <= levels; ++L) {
            if (L > 0) blk = blk > 1 ? (blk + kFanout - 1) / kFanout : 0u;
            scan_into(blk, blk_off + L * (S + 1), carry_b[L]);
        }
    }
    if (threadIdx.x == 0) {
        tile_off[S] = (int32_t)carry_t;
        for (int L = 0; L <= levels; ++L) blk_off[L * (S + 1) + S] = (int32_t)carry_b[L];
    }
    // the scenes in decreasing bit length of their size (for the one-block-
    // per-scene sort: the longest blocks start first); any order within a
    // length
    auto len_of = [&](int s) {
        const uint64_t n = (uint64_t)scene_size(seg_off, s);
        return n ? 64 - __clzll(n) : 0;   // 0 .. 31
    };
    for (int s = threadIdx.x; s < S; s += kPlanThreads) atomicAdd(&s_len[len_of(s)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t at = 0;
        for (int l = 31; l >= 0; --l) {
            const uint32_t c = s_len[l];
            s_len[l] = at;
            at += c;
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < S; s += kPlanThreads) order[atomicAdd(&s_len[len_of(s)], 1u)] = s;
}

// One block per scene: scene box (min/max), scale 2^b / extent, Morton codes
// (written in place of the scene's primitives' order), digit histograms
// (BITS-wide digits) of every radix pass for scenes spanning several tiles,
// and the first pass's look-back status of those tiles cleared.
template <int KIND, typename K, int BITS>
__global__ __launch_bounds__(kSceneThreads) void k_batch_morton(
    const float *__restrict__ prims, const int64_t *__restrict__ seg_off,
    const int32_t *__restrict__ tile_off, int bits_per_axis, float4 *__restrict__ scene_box,
    K *__restrict__ codes, uint32_t *__restrict__ hist, uint32_t *__restrict__ status0)
{
    constexpr int R = 1 << BITS;
    constexpr int PASSES = ((sizeof(K) == 4 ? 30 : 63) + BITS - 1) / BITS;
    __shared__ float sh[(kSceneThreads / 64) * 6];
    __shared__ float4 s_box[3];
    __shared__ uint32_t lh[PASSES * R];
    using P = Prims<KIND>;
    const int s = blockIdx.x;
    const int64_t b0 = seg_off[s];
    const int64_t ns = seg_off[s + 1] - b0;
    if (ns == 0) return;
    const bool multi = tile_off[s + 1] - tile_off[s] > 1;
    if (multi)
        for (int j = threadIdx.x; j < PASSES * R; j += kSceneThreads) lh[j] = 0u;

    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < ns; i += kSceneThreads) {
        float lo[3], hi[3];
        P::one(prims, b0 + i, lo, hi);
#pragma unroll
        for (int a = 0; a < 3; ++a) { v[a] = fminf(v[a], lo[a]); v[3 + a] = fmaxf(v[3 + a], hi[a]); }
    }
    block_minmax6<kSceneThreads>(v, sh);
    if (threadIdx.x == 0) {
        const float two_b = (float)(1u << bits_per_axis);
        float sc[3];
        for (int a = 0; a < 3; ++a) {
            const float ext = v[3 + a] - v[a];
            sc[a] = ext > 0.0f ? __fdiv_rn(two_b, ext) : 0.0f;
        }
        s_box[0] = make_float4(v[0], v[1], v[2], 0.0f);
        s_box[1] = make_float4(v[3], v[4], v[5], 0.0f);
        s_box[2] = make_float4(sc[0], sc[1], sc[2], 0.0f);
        scene_box[3 * s + 0] = s_box[0];
        scene_box[3 * s + 1] = s_box[1];
        scene_box[3 * s + 2] = s_box[2];
    }
    __syncthreads();
    const float4 slo = s_box[0], sc = s_box[2];
    for (int64_t i = threadIdx.x; i < ns; i += kSceneThreads) {
        float lo[3], hi[3];
        P::one(prims, b0 + i, lo, hi);
        const K c = code_of<KIND, K>(lo, hi, slo, sc);
        codes[b0 + i] = c;
        if (multi)
#pragma unroll
            for (int p = 0; p < PASSES; ++p)
                atomicAdd(&lh[p * R + (uint32_t)((c >> (p * BITS)) & (R - 1))], 1u);
    }
    if (!multi) return;
    __syncthreads();
    uint32_t *hs = hist + (int64_t)s * PASSES * R;
    for (int j = threadIdx.x; j < PASSES * R; j += kSceneThreads) hs[j] = lh[j];
    const int64_t w0 = (int64_t)tile_off[s] * R, w1 = (int64_t)tile_off[s + 1] * R;
    for (int64_t w = w0 + threadIdx.x; w < w1; w += kSceneThreads) status0[w] = 0u;
}

// ------------------------------------------------- one block per scene
//
// The other sort schedule of the batched build ("batch_sort_mode" 1): one
// block takes one whole scene (scenes in decreasing size, so the longest
// blocks start first) and runs every step up to the sorted codes itself:
// scene box and scale, the codes with every pass's digit histogram, then
// the sort.  A scene of one tile (T*I keys) is sorted on chip.  A larger
// scene is partitioned by its top digit in one pass over global memory and
// its runs of whole digit values, packed up to a tile, are sorted on chip;
// if one top-digit value holds more than a tile, each LSD pass runs over
// the scene in tiles instead.  A tile is ranked stably with wave64 ballots
// (as in the onesweep pass) and scattered through LDS so that global
// writes are runs of equal digits; the block's running start of each digit
// carries over from tile to tile, so no tile waits for another block (no
// look-back), and scenes need no tile plan.  Global writes of one pass are
// read by the next step of the same block after a workgroup barrier.
template <int KIND, typename K, int BITS, int T, int I>
__global__ __launch_bounds__(T) void k_scene_sort(
    const float *__restrict__ prims, const int64_t *__restrict__ seg_off,
    const int32_t *__restrict__ order, int code_bits, float4 *__restrict__ scene_box, K *key_a,
    K *key_b, int32_t *val_a, int32_t *val_b, int32_t *__restrict__ perm_out, uint32_t *err)
{
    constexpr int R = 1 << BITS;
    constexpr int W = T / 64;
    constexpr int TILE = T * I;
    constexpr int DPT = (R + T - 1) / T;
    constexpr int PASSES = ((sizeof(K) == 4 ? 30 : 63) + BITS - 1) / BITS;
    static_assert(TILE < 65536, "16-bit per-wave digit counters");
    using Cnt = typename std::conditional<(BITS <= 9), uint32_t, uint16_t>::type;
    using P = Prims<KIND>;
    __shared__ __align__(16) Cnt s_wcnt[W][R];
    __shared__ uint32_t s_start[R];   // tile-local start of each digit run
    __shared__ uint32_t s_run[2][R];  // scene-local start of the digit's next run
    __shared__ uint32_t s_hist[R];    // one digit's counts over the scene
    __shared__ uint32_t s_scan[2][W];
    __shared__ K s_buf[TILE];
    __shared__ int32_t s_val[TILE];
    __shared__ float sh[W * 6];
    __shared__ float4 s_box[3];
    __shared__ uint32_t s_flag;       // some top digit holds more than a tile
    __shared__ uint32_t s_last[2];    // last digit of the current run group

    const int s = order[blockIdx.x];
    const int64_t b0 = seg_off[s];
    const int64_t ns64 = seg_off[s + 1] - b0;
    if (ns64 == 0) return;
    const uint32_t ns = (uint32_t)ns64;   // a scene holds fewer than 2^30 primitives
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = tid; j < R; j += T) s_hist[j] = 0u;
    if (tid == 0) { s_flag = 0u; s_last[0] = 0u; }

    // scene box and scale (2^b / extent, correctly rounded; 0 when flat)
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = tid; i < ns; i += T) {
        float lo[3], hi[3];
        P::one(prims, b0 + i, lo, hi);
#pragma unroll
        for (int a = 0; a < 3; ++a) { v[a] = fminf(v[a], lo[a]); v[3 + a] = fmaxf(v[3 + a], hi[a]); }
    }
    block_minmax6<T>(v, sh);
    if (tid == 0) {
        const float two_b = (float)(1u << (code_bits / 3));
        float sc[3];
        for (int a = 0; a < 3; ++a) {
            const float ext = v[3 + a] - v[a];
            sc[a] = ext > 0.0f ? __fdiv_rn(two_b, ext) : 0.0f;
        }
        s_box[0] = make_float4(v[0], v[1], v[2], 0.0f);
        s_box[1] = make_float4(v[3], v[4], v[5], 0.0f);
        s_box[2] = make_float4(sc[0], sc[1], sc[2], 0.0f);
        scene_box[3 * s + 0] = s_box[0];
        scene_box[3 * s + 1] = s_box[1];
        scene_box[3 * s + 2] = s_box[2];
    }
    __syncthreads();
    // codes in input order, and (scenes of several tiles) the top digit's
    // counts; the other digits are counted only if the scene needs them
    const int top = PASSES - 1;
    const int top_shift = top * BITS;
    {
        const float4 slo = s_box[0], sc = s_box[2];
        const bool count = ns > (uint32_t)TILE;
        for (uint32_t i = tid; i < ns; i += T) {
            float lo[3], hi[3];
            P::one(prims, b0 + i, lo, hi);
            const K c = code_of<KIND, K>(lo, hi, slo, sc);
            key_a[b0 + i] = c;
            if (count) atomicAdd(&s_hist[(uint32_t)((c >> top_shift) & (R - 1))], 1u);
        }
    }
    __threadfence_block();
    __syncthreads();

    const int d0 = tid * DPT;
    auto owns = [&](int k) { return d0 + k < R; };
    constexpr int kZeroWords = W * R * (int)sizeof(Cnt) / 4;
    auto zero_counts = [&]() {
        for (int j = tid; j < kZeroWords; j += T) reinterpret_cast<uint32_t *>(&s_wcnt[0][0])[j] = 0u;
    };
    // The tile ranking shared by both paths below: key k of this thread is
    // the tile's key lofs + 64k (rem keys in the tile); returns each key's
    // position in the tile's stable order by this pass's digit.  The wave
    // counters must be zero on entry (each caller clears them, after its
    // last read of the previous ranking and before a barrier).
    auto rank_tile = [&](const K (&key)[I], uint32_t rem, uint32_t lofs, int shift,
                         uint32_t (&pos)[I], uint32_t (&total)[DPT], uint32_t (&start)[DPT]) {
        uint32_t rank[I];
        // the wave's first key (a scalar: rows with no key in the tile are
        // skipped by a branch of the whole wave)
        const uint32_t wbase = (uint32_t)__builtin_amdgcn_readfirstlane((int)(lofs - lane));
#pragma unroll
        for (int k = 0; k < I; ++k) {
            rank[k] = 0u;
            if (wbase + k * 64 >= rem) continue;
            const bool ok = lofs + k * 64 < rem;
            const uint32_t d = (uint32_t)(key[k] >> shift) & (R - 1);
            // bits of a narrower last digit are zero above it in every key
            const uint64_t peers = __ballot(ok) & ~digit_diff<BITS>(d);
            const uint32_t below = count_below(peers);
            const uint32_t cnt = s_wcnt[wave][d];
            rank[k] = cnt + below;
            if (ok && below == 0) s_wcnt[wave][d] = (Cnt)(cnt + (uint32_t)__popcll(peers));
        }
        __syncthreads();
        // per-wave exclusive offsets and the tile's digit totals
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            total[k] = 0;
            if (owns(k)) {
                const int d = d0 + k;
                uint32_t c[W];
#pragma unroll
                for (int w = 0; w < W; ++w) c[w] = s_wcnt[w][d];
#pragma unroll
                for (int w = 0; w < W; ++w) { s_wcnt[w][d] = (Cnt)total[k]; total[k] += c[w]; }
            }
        }
        digits_excl_scan<T, DPT>(total, start, s_scan[1]);
#pragma unroll
        for (int k = 0; k < DPT; ++k)
            if (owns(k)) s_start[d0 + k] = start[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < I; ++k) {
            pos[k] = 0u;
            if (wbase + k * 64 >= rem) continue;
            const uint32_t dk = (uint32_t)(key[k] >> shift) & (R - 1);
            pos[k] = s_start[dk] + s_wcnt[wave][dk] + rank[k];
        }
    };
    const uint32_t lofs = (uint32_t)(wave * 64 * I + lane);
    K *const kfinal = ((PASSES - 1) & 1) ? key_a : key_b;
    // Keys [off, off + cnt) of kin (cnt <= TILE) sorted on chip: each pass
    // reorders them through LDS and only the last pass writes, the sorted
    // codes to kfinal and the permutation to perm_out at the same places.
    // Values are vin's, or the scene-local index when vin is null.  kin may
    // be kfinal: every key is in registers before the first barrier.  The
    // caller's last barrier must follow its last read of the wave counters.
    auto sort_on_chip = [&](const K *kin, const int32_t *vin, uint32_t off, uint32_t cnt) {
        K key[I];
        int32_t val[I];
        zero_counts();
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const bool ok = lofs + k * 64 < cnt;
            const int64_t at = b0 + off + lofs + k * 64;
            key[k] = ok ? kin[at] : (K)0;
            val[k] = vin ? (ok ? vin[at] : 0) : (int32_t)(off + lofs + k * 64);
        }
        __syncthreads();
        for (int p = 0; p < PASSES; ++p) {
            const int shift = p * BITS;
            uint32_t pos[I], total[DPT], start[DPT];
            rank_tile(key, cnt, lofs, shift, pos, total, start);
            if (p + 1 == PASSES) {
#pragma unroll
                for (int k = 0; k < I; ++k)
                    if (lofs + k * 64 < cnt) {
                        kfinal[b0 + off + pos[k]] = key[k];
                        perm_out[b0 + off + pos[k]] = val[k];
                    }
                break;
            }
#pragma unroll
            for (int k = 0; k < I; ++k)
                if (lofs + k * 64 < cnt) {
                    s_buf[pos[k]] = key[k];
                    s_val[pos[k]] = val[k];
                }
            __syncthreads();
            zero_counts();   // every position is read
#pragma unroll
            for (int k = 0; k < I; ++k) {
                const bool ok = lofs + k * 64 < cnt;
                key[k] = ok ? s_buf[lofs + k * 64] : (K)0;
                val[k] = ok ? s_val[lofs + k * 64] : 0;
            }
            __syncthreads();
        }
    };
    // One stable pass over the whole scene by the digit at `shift` (its
    // counts in s_hist), tile after tile through global memory.  The
    // running start of each digit alternates between the two rows of s_run
    // (tile t reads row t & 1 and its owner writes the next row), so no
    // barrier guards it; returns the row that ends up holding the
    // scene-local end of each digit's run.
    auto global_pass = [&](const K *kin, K *kout, const int32_t *vin, int32_t *vout, int shift) -> int {
        zero_counts();
        {   // the scene-local start of each digit in this pass
            uint32_t h[DPT], st[DPT];
#pragma unroll
            for (int k = 0; k < DPT; ++k) h[k] = owns(k) ? s_hist[d0 + k] : 0u;
            digits_excl_scan<T, DPT>(h, st, s_scan[0]);
#pragma unroll
            for (int k = 0; k < DPT; ++k)
                if (owns(k)) s_run[0][d0 + k] = st[k];
        }
        int row = 0;
        for (uint32_t base = 0; base < ns; base += TILE, row ^= 1) {
            const uint32_t rem = ns - base < (uint32_t)TILE ? ns - base : (uint32_t)TILE;
            K key[I];
            int32_t val[I];
#pragma unroll
            for (int k = 0; k < I; ++k) {
                const bool ok = lofs + k * 64 < rem;
                const int64_t at = b0 + base + lofs + k * 64;
                key[k] = ok ? kin[at] : (K)0;
                val[k] = vin ? (ok ? vin[at] : 0) : (int32_t)(base + lofs + k * 64);
            }
            // stable rank within the wave, as in the onesweep pass
            uint32_t pos[I], total[DPT], start[DPT];
            rank_tile(key, rem, lofs, shift, pos, total, start);
            // the next tile's runs of each digit follow this tile's
#pragma unroll
            for (int k = 0; k < DPT; ++k)
                if (owns(k)) s_run[row ^ 1][d0 + k] = s_run[row][d0 + k] + total[k];
#pragma unroll
            for (int k = 0; k < I; ++k)
                if (lofs + k * 64 < rem) {
                    s_buf[pos[k]] = key[k];
                    s_val[pos[k]] = val[k];
                }
            __syncthreads();
            zero_counts();
#pragma unroll
            for (int k = 0; k < I; ++k) {
                const uint32_t q = (uint32_t)(k * T + tid);
                if (q < rem) {
                    const K kk = s_buf[q];
                    const uint32_t dk = (uint32_t)(kk >> shift) & (R - 1);
                    const uint32_t out = s_run[row][dk] + q - s_start[dk];   // < ns by construction
                    if (out < ns) {
                        kout[b0 + out] = kk;
                        vout[b0 + out] = s_val[q];
                    } else {   // inconsistent counts: flag it rather than write outside
                        __hip_atomic_store(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            __syncthreads();
        }
        // this pass's writes are the next reads (same block)
        __threadfence_block();
        __syncthreads();
        return row;
    };

    if (ns <= (uint32_t)TILE) {   // one tile: all passes on chip
        sort_on_chip(key_a, nullptr, 0u, ns);
        return;
    }
    // Several tiles.  When no value of the top digit holds more than a
    // tile's keys, one global pass partitions the scene by the top digit
    // (most significant first), and runs of whole digit values, packed up to
    // a tile, are then sorted on chip by the whole code: the final order of
    // each run's keys lies inside the run, and both steps are stable, so
    // equal codes keep their input order.  Two global passes instead of one
    // per digit.  Otherwise every pass runs over the scene (least
    // significant digit first).
    const int top_bits = BITS < code_bits - top_shift ? BITS : code_bits - top_shift;
#pragma unroll
    for (int k = 0; k < DPT; ++k)
        if (owns(k) && s_hist[d0 + k] > (uint32_t)TILE) s_flag = 1u;
    __syncthreads();
    if (s_flag == 0u && top_bits > 0) {
        const uint32_t *end = s_run[global_pass(key_a, key_b, nullptr, val_a, top_shift)];
        // digit d's keys now lie in [end[d-1], end[d]) of key_b / val_a;
        // group g takes digits gb..last, the most that fit a tile (slot
        // g & 1 of s_last holds gb before the max)
        uint32_t gb = 0;
        for (int g = 0;; ++g) {
            const uint32_t gstart = gb == 0 ? 0u : end[gb - 1];
            if (gb >= (uint32_t)R || gstart >= ns) break;
#pragma unroll
            for (int k = 0; k < DPT; ++k) {
                const uint32_t d = (uint32_t)(d0 + k);
                if (owns(k) && d >= gb && end[d] - gstart <= (uint32_t)TILE) atomicMax(&s_last[g & 1], d);
            }
            __syncthreads();
            const uint32_t last = s_last[g & 1];
            const uint32_t gend = end[last];
            if (tid == 0) s_last[(g + 1) & 1] = last + 1;
            if (gend <= gstart || gend > ns || gend - gstart > (uint32_t)TILE) {   // not expected
                if (tid == 0) __hip_atomic_store(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            sort_on_chip(key_b, val_a, gstart, gend - gstart);
            gb = last + 1;
        }
        return;
    }
    for (int p = 0; p < PASSES; ++p) {
        const K *kin = (p & 1) ? key_b : key_a;
        K *kout = (p & 1) ? key_a : key_b;
        const int32_t *vin = p == 0 ? nullptr : ((p & 1) ? val_a : val_b);
        int32_t *vout = p + 1 == PASSES ? perm_out : ((p & 1) ? val_b : val_a);
        const int shift = p * BITS;
        // this digit's counts (the previous pass read s_hist before its
        // last barrier)
        for (int j = tid; j < R; j += T) s_hist[j] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < ns; i += T)
            atomicAdd(&s_hist[(uint32_t)((kin[b0 + i] >> shift) & (R - 1))], 1u);
        __syncthreads();
        global_pass(kin, kout, vin, vout, shift);
    }
}

// Alg. 1 for query j on the tree of its scene (no splitting: batched
// workloads have many scenes and light queries).  Containment reports whole
// leaf ranges from leaf_perm, as in the single-tree leaf walk.
// Alg. 1 for query j on the tree of its scene (one thread per query); the
// fill pass writes through a HitStage (the block's queries have consecutive
// output ranges).
// The batched count keeps each query's first kBatchHitCache hits (scenes
// are small, so most queries have fewer); the fill copies them instead of
// walking again.
constexpr int kBatchHitCache = 64;

template <class Q>
__device__ __forceinline__ void batch_walk_one(const float4 *nodes_all, const int32_t *perm_all,
                                               const int64_t *seg_off, const int64_t *qseg_off, int S,
                                               const float *queries, int64_t j, int &cnt,
                                               const HitStage *st, int64_t pos,
                                               int32_t *kept = nullptr, uint32_t *err = nullptr,
                                               int64_t budget_cap = 0, int64_t end = 0)
{
    int lo = 0, hi = S - 1;   // scene of query j: largest s with qseg_off[s] <= j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (qseg_off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const int64_t b0 = seg_off[lo];
    const int n = (int)(seg_off[lo + 1] - b0);
    if (n <= 0) return;
    Tree tr{nodes_all + 4 * b0, perm_all + b0, n, err, budget_cap};
    Q q;
    q.load(queries, (int)j);
    const int leaf0 = n - 1;
    int v = 0, i = 0;
    int64_t budget = tr.walk_budget();
    while (v != -1 && --budget >= 0) {
        float4 a, b;
        tr.load(v, a, b);
        const int left = __float_as_int(a.w);
        const int rope = __float_as_int(b.w);
        const int jr = tr.right_bound(b);
        if (q.test(a, b)) {
            if (v >= leaf0) {
                if (st) {
                    if (pos < end) st->put(pos, left);   // never past the counted hits
                    ++pos;
                } else {
                    if (kept && cnt < kBatchHitCache) kept[cnt] = left;
                    ++cnt;
                }
            } else if (q.contains(a, b)) {
                if (st) {
                    const int64_t len = jr - i + 1 < end - pos ? jr - i + 1 : end - pos;
                    st->range(pos, (int32_t)b0 + i, (int32_t)len);   // perm_all index
                    pos += jr - i + 1;
                } else {
                    if (kept)
                        for (int k = i; k <= jr && cnt + (k - i) < kBatchHitCache; ++k)
                            kept[cnt + (k - i)] = tr.perm[k];
                    cnt += jr - i + 1;
                }
            } else {
                v = left;
                continue;
            }
        }
        v = rope;
        i = jr + 1;
    }
    if (budget < 0) tr.budget_spent();
}

template <class Q>
__global__ __launch_bounds__(kBlock) void k_batch_count(const float4 *__restrict__ nodes_all,
                                                        const int32_t *__restrict__ perm_all,
                                                        const int64_t *__restrict__ seg_off,
                                                        const int64_t *__restrict__ qseg_off, int S,
                                                        const float *__restrict__ queries, int64_t m,
                                                        int32_t *__restrict__ counts,
                                                        int32_t *__restrict__ cache, uint32_t *err,
                                                        int64_t budget_cap)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    int cnt = 0;
    batch_walk_one<Q>(nodes_all, perm_all, seg_off, qseg_off, S, queries, j, cnt, nullptr, 0,
                      cache + j * kBatchHitCache, err, budget_cap);
    counts[j] = cnt;
}

// Start of a batched count call: clear its error word.
__global__ void k_batch_query_reset(uint32_t *err)
{
    if (threadIdx.x == 0) *err = 0u;
}

template <class Q>
__global__ __launch_bounds__(kBlock) void k_batch_fill(const float4 *__restrict__ nodes_all,
                                                       const int32_t *__restrict__ perm_all,
                                                       const int64_t *__restrict__ seg_off,
                                                       const int64_t *__restrict__ qseg_off, int S,
                                                       const float *__restrict__ queries, int64_t m,
                                                       const int64_t *__restrict__ offsets,
                                                       const int32_t *__restrict__ cache,
                                                       int32_t *__restrict__ out)
{
    __shared__ WaveStageLds lds;
    const int64_t j0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63);   // the wave's first query
    if (j0 >= m) return;   // uniform over the wave
    const int lane = threadIdx.x & 63;
    const int64_t j = j0 + lane;
    const int64_t j_end = j0 + 64 < m ? j0 + 64 : m;
    if (lane == 0) lds.njobs[threadIdx.x >> 6] = 0;
    wave_sync();
    const HitStage st = wave_stage(lds, out, perm_all, offsets[j0]);
    int unused = 0;
    if (j < m) {
        const int64_t pos = offsets[j], have = offsets[j + 1] - pos;
        if (have <= kBatchHitCache)   // the count call kept them
            for (int k = 0; k < have; ++k) st.put(pos + k, cache[j * kBatchHitCache + k]);
        else
            batch_walk_one<Q>(nodes_all, perm_all, seg_off, qseg_off, S, queries, j, unused, &st, pos,
                              nullptr, nullptr, 0, pos + have);
    }
    st.flush(offsets[j_end] - st.base);
}

// Radix tile shapes of the batched build (threads x keys per thread); the
// knob "batch_sort_variant" picks one.  A shape below the digit width's
// minimum tile is replaced by 256 x 16.
struct BatchSortShape { int threads, items; };
constexpr BatchSortShape kBatchShapes[] = {{256, 16}, {256, 8}, {512, 8}, {512, 16}};

int batch_sort_variant(int bits)
{
    const int64_t v = tune_get(TUNE_BATCH_SORT);
    const int var = (v >= 0 && v < 4) ? (int)v : 0;
    return kBatchShapes[var].threads * kBatchShapes[var].items >= radix_min_tile(bits) ? var : 0;
}

template <typename K, int T, int I, int B>
void launch_seg(int64_t grid, const K *kin, K *kout, const int32_t *vin, int32_t *vout, int64_t N,
                const SortSegs &segs, int shift, int nbits, const uint32_t *hist, uint32_t *st,
                uint32_t *st_next, uint32_t *ctr, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL((k_onesweep<K, T, I, B>), dim3((unsigned)grid), dim3(T), 0, s, kin, kout, vin,
                       vout, N, segs, shift, nbits, hist, st, st_next, (uint32_t)grid, ctr, err,
                       (const uint32_t *)nullptr);
}

template <typename K, int B>
void launch_seg_variant(int v, int64_t grid, const K *kin, K *kout, const int32_t *vin, int32_t *vout,
                        int64_t N, const SortSegs &segs, int shift, int nbits, const uint32_t *hist,
                        uint32_t *st, uint32_t *st_next, uint32_t *ctr, uint32_t *err, hipStream_t s)
{
#define LBVH_SEG_ARGS grid, kin, kout, vin, vout, N, segs, shift, nbits, hist, st, st_next, ctr, err, s
    switch (v) {
    case 1: launch_seg<K, 256, 8, B>(LBVH_SEG_ARGS); break;
    case 2: launch_seg<K, 512, 8, B>(LBVH_SEG_ARGS); break;
    case 3: launch_seg<K, 512, 16, B>(LBVH_SEG_ARGS); break;
    default: launch_seg<K, 256, 16, B>(LBVH_SEG_ARGS); break;
    }
#undef LBVH_SEG_ARGS
}

// Per-scene codes and the segmented radix passes of one digit width.  The
// Morton kernel writes the codes to the buffer that makes the last pass end
// in the batch's codes array; the last pass writes leaf_perm.
template <int KIND, typename K, int B>
void run_batch_sort(const float *prims, const int64_t *seg_off, int S, int64_t N, int code_bits,
                    K *codes, int32_t *leaf_perm, int32_t *tile_off, float4 *scene_box, uint32_t *ctrl,
                    uint32_t *hist, uint32_t *status[2], K *keys_alt, int32_t *vals[2], int variant,
                    hipStream_t s)
{
    const int passes = radix_passes(code_bits, B);
    const int tile = kBatchShapes[variant].threads * kBatchShapes[variant].items;
    const int64_t tiles_grid = (N + tile - 1) / tile + S;   // within the look-back tables
    K *first = (passes & 1) ? keys_alt : codes;
    K *second = (passes & 1) ? codes : keys_alt;
    hipLaunchKernelGGL((k_batch_morton<KIND, K, B>), dim3(S), dim3(kSceneThreads), 0, s, prims,
                       seg_off, tile_off, code_bits / 3, scene_box, first, hist, status[0]);
    prof_end(K_BATCH_PREP, s);

    const SortSegs segs{seg_off, tile_off, S, (int64_t)passes << B};
    for (int p = 0; p < passes; ++p) {
        const K *kin = (p & 1) ? second : first;
        K *kout = (p & 1) ? first : second;
        const int32_t *vin = p == 0 ? nullptr : vals[(p - 1) & 1];
        int32_t *vout = p + 1 == passes ? leaf_perm : vals[p & 1];
        uint32_t *st_next = (p + 1 < passes) ? status[(p + 1) & 1] : nullptr;
        const int nbits = std::min(B, code_bits - p * B);
        prof_begin(K_SORT, s);
        launch_seg_variant<K, B>(variant, tiles_grid, kin, kout, vin, vout, N, segs, p * B, nbits,
                                 hist + ((int64_t)p << B), status[p & 1], st_next,
                                 ctrl + kCtrlTileCounter + p, ctrl + kCtrlError, s);
        prof_end(K_SORT, s);
    }
}

// The one-block-per-scene sort: codes go to the key buffer that makes the
// last pass end in the batch's codes array.  Block shapes (threads x keys
// per thread, the knob "batch_sort_variant" in this mode): wider blocks take
// a large scene in fewer tiles per pass; a shape whose tables and tile do
// not fit the LDS runs as 256 x 16.
constexpr size_t scene_sort_lds(int key_bytes, int threads, int items, int bits)
{
    // wave counters; digit counts, starts and two rows of runs; keys and values
    return (size_t)(threads / 64) * ((bits <= 9 ? 4u : 2u) << bits) + (16u << bits) +
           (size_t)threads * items * (key_bytes + 4);
}

template <int KIND, typename K, int B, int T, int I>
void launch_scene_sort(const float *prims, const int64_t *seg_off, const int32_t *order, int S,
                       int code_bits, K *ka, K *kb, int32_t *vals[2], int32_t *leaf_perm,
                       float4 *scene_box, uint32_t *err, hipStream_t s)
{
    if constexpr (scene_sort_lds(sizeof(K), T, I, B) > 150 * 1024) {
        launch_scene_sort<KIND, K, B, 256, 16>(prims, seg_off, order, S, code_bits, ka, kb, vals,
                                               leaf_perm, scene_box, err, s);
    } else {
        hipLaunchKernelGGL((k_scene_sort<KIND, K, B, T, I>), dim3(S), dim3(T), 0, s, prims, seg_off,
                           order, code_bits, scene_box, ka, kb, vals[0], vals[1], leaf_perm, err);
    }
}

template <int KIND, typename K, int B>
void run_scene_sort(const float *prims, const int64_t *seg_off, const int32_t *order, int S,
                    int code_bits, K *codes, int32_t *leaf_perm, float4 *scene_box, K *keys_alt,
                    int32_t *vals[2], uint32_t *err, hipStream_t s)
{
    const int passes = radix_passes(code_bits, B);
    K *ka = (passes & 1) ? keys_alt : codes;
    K *kb = (passes & 1) ? codes : keys_alt;
    prof_begin(K_SORT, s);
#define LBVH_SCENE_ARGS prims, seg_off, order, S, code_bits, ka, kb, vals, leaf_perm, scene_box, err, s
    switch (tune_get(TUNE_BATCH_SORT)) {
    case 1: launch_scene_sort<KIND, K, B, 512, 8>(LBVH_SCENE_ARGS); break;
    case 2: launch_scene_sort<KIND, K, B, 1024, 8>(LBVH_SCENE_ARGS); break;
    case 3: launch_scene_sort<KIND, K, B, 512, 16>(LBVH_SCENE_ARGS); break;
    default: launch_scene_sort<KIND, K, B, 256, 16>(LBVH_SCENE_ARGS); break;
    }
#undef LBVH_SCENE_ARGS
    prof_end(K_SORT, s);
}

template <int KIND, typename K>
hipError_t run_batch(const float *prims, const int64_t *seg_off, int S, int64_t N, int levels,
                     int code_bits, lbvh_node *nodes_, K *codes, int32_t *leaf_perm, char *ws,
                     const BatchLayout &L, hipStream_t s)
{
    uint32_t *ctrl = reinterpret_cast<uint32_t *>(ws + L.ctrl);
    float4 *scene_box = reinterpret_cast<float4 *>(ws + L.scene_box);
    int32_t *tile_off = reinterpret_cast<int32_t *>(ws + L.tile_off);
    int32_t *blk_off = reinterpret_cast<int32_t *>(ws + L.blk_off);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *status[2] = {reinterpret_cast<uint32_t *>(ws + L.status[0]),
                           reinterpret_cast<uint32_t *>(ws + L.status[1])};
    K *keys_alt = reinterpret_cast<K *>(ws + L.keys_alt);
    int32_t *vals[2] = {reinterpret_cast<int32_t *>(ws + L.vals[0]),
                        reinterpret_cast<int32_t *>(ws + L.vals[1])};
    int32_t *store = reinterpret_cast<int32_t *>(ws + L.store);
    Climb *pend[2] = {reinterpret_cast<Climb *>(ws + L.pend[0]), reinterpret_cast<Climb *>(ws + L.pend[1])};
    float4 *nodes = reinterpret_cast<float4 *>(nodes_);

    const int bits = radix_bits(code_bits);
    const int variant = batch_sort_variant(bits);
    const int tile = kBatchShapes[variant].threads * kBatchShapes[variant].items;
    int32_t *order = reinterpret_cast<int32_t *>(ws + L.order);
    prof_begin(K_BATCH_PREP, s);
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, s, seg_off, S, levels, tile,
                       tile_off, blk_off, ctrl, order);
    // one block per scene only while every scene is small (at most one
    // upper level: kChunk * kFanout primitives); a block alone on a scene of millions
    // would set the whole batch's time
    if (tune_get(TUNE_BATCH_SORT_MODE) == 1 && levels <= 1) {
        prof_end(K_BATCH_PREP, s);
#define LBVH_SSORT_ARGS prims, seg_off, order, S, code_bits, codes, leaf_perm, scene_box, keys_alt, \
                        vals, ctrl + kCtrlError, s
        if constexpr (sizeof(K) == 4) {
            if (bits == 10) run_scene_sort<KIND, K, 10>(LBVH_SSORT_ARGS);
            else run_scene_sort<KIND, K, 8>(LBVH_SSORT_ARGS);
        } else {
            if (bits == 11) run_scene_sort<KIND, K, 11>(LBVH_SSORT_ARGS);
            else if (bits == 9) run_scene_sort<KIND, K, 9>(LBVH_SSORT_ARGS);
            else run_scene_sort<KIND, K, 8>(LBVH_SSORT_ARGS);
        }
#undef LBVH_SSORT_ARGS
    } else {
#define LBVH_BSORT_ARGS prims, seg_off, S, N, code_bits, codes, leaf_perm, tile_off, scene_box, ctrl, \
                        hist, status, keys_alt, vals, variant, s
        if constexpr (sizeof(K) == 4) {
            if (bits == 10) run_batch_sort<KIND, K, 10>(LBVH_BSORT_ARGS);
            else run_batch_sort<KIND, K, 8>(LBVH_BSORT_ARGS);
        } else {
            if (bits == 11) run_batch_sort<KIND, K, 11>(LBVH_BSORT_ARGS);
            else if (bits == 9) run_batch_sort<KIND, K, 9>(LBVH_BSORT_ARGS);
            else run_batch_sort<KIND, K, 8>(LBVH_BSORT_ARGS);
        }
#undef LBVH_BSORT_ARGS
    }

    prof_begin(K_BOTTOMUP, s);
    BatchLevel bl{seg_off, blk_off, nullptr, S, levels == 0};
    // delta* bytes for the upper levels: in the sort's other key buffer, free now
    uint8_t *dstar = reinterpret_cast<uint8_t *>(keys_alt);
    // packed store words when the levels cover at most 2^24 leaves per
    // scene (a larger scene is flagged as beyond the cover, never built)
    int64_t cover = kChunk;
    for (int lv = 0; lv < levels; ++lv) cover *= kFanout;
    const bool packed = cover <= kPackedMaxN;
    if (packed)
        hipLaunchKernelGGL((k_bottomup_l0<KIND, K, true>), dim3((unsigned)L.blocks_max[0]),
                           dim3(kBU0Threads), 0, s, codes, leaf_perm, prims, (int)N, store, nodes,
                           pend[0], bl, dstar, ctrl + kCtrlError);
    else
        hipLaunchKernelGGL((k_bottomup_l0<KIND, K, false>), dim3((unsigned)L.blocks_max[0]),
                           dim3(kBU0Threads), 0, s, codes, leaf_perm, prims, (int)N, store, nodes,
                           pend[0], bl, dstar, ctrl + kCtrlError);
    prof_end(K_BOTTOMUP, s);
    int64_t span = kChunk;
    for (int lv = 1; lv <= levels; ++lv) {
        const int64_t next = span * kFanout;
        BatchLevel up{seg_off, blk_off + lv * (S + 1), blk_off + (lv - 1) * (S + 1), S, lv == levels,
                      lv == levels ? order : nullptr};
        prof_begin(K_BOTTOMUP_UP, s);
        if (packed)
            hipLaunchKernelGGL(k_bottomup_up<true>, dim3((unsigned)L.blocks_max[lv]), dim3(kBUThreads),
                               0, s, dstar, (int)N, span, next, store, nodes, pend[(lv - 1) & 1],
                               pend[lv & 1], up, ctrl + kCtrlError);
        else
            hipLaunchKernelGGL(k_bottomup_up<false>, dim3((unsigned)L.blocks_max[lv]), dim3(kBUThreads),
                               0, s, dstar, (int)N, span, next, store, nodes, pend[(lv - 1) & 1],
                               pend[lv & 1], up, ctrl + kCtrlError);
        prof_end(K_BOTTOMUP_UP, s);
        span = next;
    }
    return hipGetLastError();
}

template <class Q>
hipError_t run_batch_query(const lbvh_batch *b, const float *q, const int64_t *qseg_off, int64_t m,
                           int64_t *offsets, int32_t *indices, bool fill, char *ws,
                           const QueryLayout &L, hipStream_t s)
{
    const float4 *nodes = reinterpret_cast<const float4 *>(b->nodes);
    const unsigned g = (unsigned)((m + kBlock - 1) / kBlock);
    int32_t *cache = reinterpret_cast<int32_t *>(ws + L.hcache);
    if (fill) {
        prof_begin(K_QFILL, s);
        hipLaunchKernelGGL((k_batch_fill<Q>), dim3(g), dim3(kBlock), 0, s, nodes, b->leaf_perm,
                           b->seg_off, qseg_off, b->num_scenes, q, m, offsets, cache, indices);
        prof_end(K_QFILL, s);
        return hipGetLastError();
    }
    int32_t *counts = reinterpret_cast<int32_t *>(ws + L.cnt1);
    int64_t *partials = reinterpret_cast<int64_t *>(ws + L.partials);
    uint32_t *err = reinterpret_cast<uint32_t *>(ws + L.ctrl + kQueryErrorByte);
    prof_begin(K_QCOUNT, s);
    hipLaunchKernelGGL(k_batch_query_reset, dim3(1), dim3(64), 0, s, err);
    hipLaunchKernelGGL((k_batch_count<Q>), dim3(g), dim3(kBlock), 0, s, nodes, b->leaf_perm,
                       b->seg_off, qseg_off, b->num_scenes, q, m, counts, cache, err,
                       tune_get(TUNE_QBUDGET));
    prof_end(K_QCOUNT, s);
    prof_begin(K_SCAN, s);
    scan(counts, m, nullptr, partials, offsets, s);
    prof_end(K_SCAN, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_build_batched(int kind, const float *prims, const lbvh_batch *b, int levels,
                                char *ws, const BatchLayout &L, hipStream_t s)
{
    const int S = b->num_scenes;
    const int64_t N = b->total_n;
    if (b->code_bits == 30) {
        uint32_t *codes = static_cast<uint32_t *>(b->codes);
        if (kind == LBVH_POINTS)
            return run_batch<LBVH_POINTS, uint32_t>(prims, b->seg_off, S, N, levels, 30, b->nodes,
                                                    codes, b->leaf_perm, ws, L, s);
        return run_batch<LBVH_BOXES, uint32_t>(prims, b->seg_off, S, N, levels, 30, b->nodes, codes,
                                               b->leaf_perm, ws, L, s);
    }
    uint64_t *codes = static_cast<uint64_t *>(b->codes);
    if (kind == LBVH_POINTS)
        return run_batch<LBVH_POINTS, uint64_t>(prims, b->seg_off, S, N, levels, 63, b->nodes, codes,
                                                b->leaf_perm, ws, L, s);
    return run_batch<LBVH_BOXES, uint64_t>(prims, b->seg_off, S, N, levels, 63, b->nodes, codes,
                                           b->leaf_perm, ws, L, s);
}

hipError_t launch_query_batched(int qkind, const lbvh_batch *b, const float *q,
                                const int64_t *qseg_off, int64_t m, int64_t *offsets,
                                int32_t *indices, bool fill, char *ws, const QueryLayout &L,
                                hipStream_t s)
{
    if (m == 0) {
        if (fill) return hipSuccess;
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(kBlock), 0, s, offsets, (int64_t)1,
                           reinterpret_cast<uint32_t *>(ws + L.ctrl + kQueryErrorByte));
        return hipGetLastError();
    }
    return qkind == 0 ? run_batch_query<Sphere>(b, q, qseg_off, m, offsets, indices, fill, ws, L, s)
                      : run_batch_query<QBox>(b, q, qseg_off, m, offsets, indices, fill, ws, L, s);
}

}  // namespace lbvh
