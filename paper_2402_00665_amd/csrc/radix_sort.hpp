// LSD radix pass (onesweep) over one BITS-wide digit, for one key array or
// for many independent segments of it (batched scenes).
//
// A block takes the next tile id from a counter (so every tile it waits for
// is already running), ranks its THREADS*ITEMS keys stably with wave64
// ballots, publishes its per-digit counts, looks back over earlier tiles of
// its segment for their running totals, and scatters keys, then values,
// through one LDS buffer so that global writes are runs of equal digits.
// Tiles never straddle segments: tile_off[s] is the first tile of segment
// s, and the first tile of a segment starts its running totals at zero.  A
// segment that fits one tile needs no histogram; otherwise `hist` holds the
// segment's digit counts for this pass (written by the Morton kernel).
//
// Digit tables: with R = 2^BITS digits and THREADS threads, thread t owns
// the DPT = ceil(R/THREADS) consecutive digits from t*DPT that are below R.
// The per-wave digit counters are 32 bits wide up to 9-bit digits and 16
// bits wide above (a tile holds fewer than 2^16 keys), so an 11-bit digit
// costs 4 KiB of LDS per wave.
#pragma once
#pragma clang fp contract(off)

#include <type_traits>

#include "device_common.hpp"

namespace lbvh {
namespace {

struct SortSegs {
    const int64_t *seg_off;   // [S+1] segment starts; nullptr: one segment [0, n)
    const int32_t *tile_off;  // [S+1] first tile of each segment
    int S;
    int64_t hist_stride;      // words between consecutive segments' histograms
};

__device__ __forceinline__ int upper_segment(const int32_t *off, int S, uint32_t x)
{
    // largest s in [0, S) with off[s] <= x (off is non-decreasing, off[0] = 0)
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((uint32_t)off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Exclusive scan over the block of each thread's DPT values, in thread
// order then item order (the digits a thread owns are consecutive).
// The lanes of the wave whose BITS-bit digit differs from this lane's d in
// some bit: for each bit, the ballot of the lanes that have it, flipped
// where this lane has it (its bit sign-extended to a 32-bit mask), or-ed in
// with one three-input bit operation per half of the mask.  A bit that is
// zero in every lane's digit (above a narrower last digit) adds nothing,
// so no pass needs to skip it.
template <int BITS>
__device__ __forceinline__ uint64_t digit_diff(uint32_t d)
{
    uint32_t lo = 0u, hi = 0u;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t rep = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // 0 or ~0
        // the ballot of rep != 0 (33: not-equal), compared on rep itself
        // rather than re-derived from d by a shift
        const uint64_t m = __builtin_amdgcn_uicmp(rep, 0u, 33);
        // x | (y ^ z): the truth table is f(0xF0, 0xCC, 0xAA)
        lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m, rep, 0xF6);
        hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m >> 32), rep, 0xF6);
    }
    return ((uint64_t)hi << 32) | lo;
}

template <int THREADS, int DPT>
__device__ __forceinline__ void digits_excl_scan(const uint32_t (&v)[DPT], uint32_t (&out)[DPT],
                                                 uint32_t *sh /* [THREADS/64] */)
{
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) sum += v[k];
    uint32_t run = block_excl_scan<THREADS>(sum, sh);
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        out[k] = run;
        run += v[k];
    }
}

// Decoupled look-back for the DPT digits from d0 that this thread owns:
// sums the counts earlier tiles published (row j of `status`, R words a
// row) back from tile-1 until an inclusive prefix or the segment's first
// tile t0, then publishes this tile's inclusive prefix.  All of the
// thread's digits are in flight together.  A wait that never ends (not
// expected: every earlier tile is already running) is cut and flagged.
template <int DPT>
__device__ __forceinline__ void look_back(uint32_t *status, int R, uint32_t tile, uint32_t t0, int d0,
                                          const uint32_t (&total)[DPT], uint32_t (&excl)[DPT],
                                          uint32_t *err)
{
    auto owns = [&](int k) { return d0 + k < R; };
    int64_t j[DPT];
    bool done[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) { excl[k] = 0; j[k] = (int64_t)tile - 1; done[k] = !owns(k); }
    uint32_t spins = 0;
    while (true) {
        uint32_t sv[DPT];
#pragma unroll
        for (int k = 0; k < DPT; ++k)
            sv[k] = done[k] ? 0u
                            : __hip_atomic_load(status + j[k] * R + d0 + k, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        bool all = true, waiting = false;
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            if (done[k]) continue;
            const uint32_t flag = sv[k] & ~kValueMask;
            if (flag == 0u) { waiting = true; all = false; continue; }
            excl[k] += sv[k] & kValueMask;
            if (flag == kFlagInclusive || j[k] == (int64_t)t0) done[k] = true;
            else { --j[k]; all = false; }
        }
        if (all) break;
        if (waiting) {
            if (++spins > (1u << 24)) {   // never expected: bounded wait
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
#pragma unroll
    for (int k = 0; k < DPT; ++k)
        if (owns(k))
            __hip_atomic_store(status + (int64_t)tile * R + d0 + k, kFlagInclusive | (excl[k] + total[k]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce-then-scan form of a pass over one key array: the tiles' digit
// offsets are worked out before the scatter, so the scatter (k_onesweep
// with `toff`) waits for no other tile.  Measured on 2^24 keys, the
// look-back inside the scatter cost 30-110 us per pass (it touches R
// status words per tile); here it runs once per chunk of kCountChunk
// tiles, over the chunks' digit totals.
//
// One block per chunk (taken in order from a counter, so every chunk it
// waits for is already running): counts the digits of all the chunk's keys
// in one sweep, per tile, in LDS; turns them into running counts over the
// chunk's tiles; then the chunk's totals go through the look-back, and each
// tile's first output position per digit,
//   toff[t][d] = (keys of digits < d) + (digit d in earlier chunks)
//              + (digit d in earlier tiles of the chunk),
// is written for the scatter.
constexpr int kCountThreads = 1024;   // 16 waves: the digit matching is latency-bound
constexpr int kCountChunk = 8;       // tiles per chunk

template <typename K, int BITS, int TILE>
__global__ __launch_bounds__(kCountThreads) void k_radix_count(
    const K *__restrict__ keys, int64_t n, int shift, const uint32_t *__restrict__ hist,
    uint32_t *status, uint32_t *__restrict__ toff, uint32_t *chunk_counter, uint32_t *err)
{
    constexpr int R = 1 << BITS;
    constexpr int DPT = (R + kCountThreads - 1) / kCountThreads;   // digits per owning thread
    constexpr int kLoads = 4;                // 16-byte loads per thread in flight
    __shared__ uint32_t s_cnt[kCountChunk][R];   // per tile: digit counts, then the chunk's running counts
    __shared__ uint32_t s_scan[kCountThreads / 64];
    __shared__ uint32_t s_chunk;
    const int tid = threadIdx.x;
    if (tid == 0) s_chunk = atomicAdd(chunk_counter, 1u);
    for (int w = tid; w < kCountChunk * R; w += kCountThreads) (&s_cnt[0][0])[w] = 0u;
    __syncthreads();
    const uint32_t c = s_chunk;
    const int64_t tiles = (n + TILE - 1) / TILE;
    const int64_t tb = (int64_t)c * kCountChunk;
    const int nct = (int)(tiles - tb < kCountChunk ? tiles - tb : kCountChunk);   // >= 1: grid = chunks
    const int d0 = tid * DPT;
    auto owns = [&](int k) { return d0 + k < R; };
    // every key of the chunk's tiles in one sweep, counted under its tile
    const int64_t cb = tb * TILE;
    const int len = n - cb < (int64_t)nct * TILE ? (int)(n - cb) : nct * TILE;
    // 16-byte loads (the chunk starts 16-byte aligned: TILE is a multiple of
    // 256 keys), kLoads of them in flight per thread, then the ragged tail.
    // The lanes holding one digit find each other with one ballot per digit
    // bit and the lowest adds their number: one LDS atomic per distinct
    // digit of a wave's 64 keys, not one per key (equal codes, frequent in
    // clustered scenes, sit together after the first passes and would
    // serialize the atomics).  A wave's 64 keys (lanes in order) never
    // straddle a tile: the loads of a wave cover 64 * V consecutive keys
    // from a multiple of that.
    const K *kp = keys + cb;
    constexpr int V = 16 / (int)sizeof(K);   // keys per load
    const int nvec = len / V;
    const uint4 *vp = reinterpret_cast<const uint4 *>(kp);
    auto count = [&](bool ok, int i, K key) {   // all lanes together
        const uint32_t d = (uint32_t)(key >> shift) & (R - 1);
        uint64_t diff = 0;
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const uint32_t rep = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // 0 or ~0
            diff |= __ballot(rep != 0u) ^ (((uint64_t)rep << 32) | rep);
        }
        const uint64_t peers = __ballot(ok) & ~diff;
        if (ok && count_below(peers) == 0u) atomicAdd(&s_cnt[i / TILE][d], (uint32_t)__popcll(peers));
    };
    for (int i0 = 0; i0 < nvec; i0 += kLoads * kCountThreads) {
        uint4 vv[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int iv = i0 + u * kCountThreads + tid;
            vv[u] = iv < nvec ? vp[iv] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const int iv = i0 + u * kCountThreads + tid;
            const bool ok = iv < nvec;
            if constexpr (sizeof(K) == 4) {
                count(ok, iv * 4, (K)vv[u].x);
                count(ok, iv * 4 + 1, (K)vv[u].y);
                count(ok, iv * 4 + 2, (K)vv[u].z);
                count(ok, iv * 4 + 3, (K)vv[u].w);
            } else {
                count(ok, iv * 2, (K)(((uint64_t)vv[u].y << 32) | vv[u].x));
                count(ok, iv * 2 + 1, (K)(((uint64_t)vv[u].w << 32) | vv[u].z));
            }
        }
    }
    for (int i = nvec * V + tid; i < len; i += kCountThreads)   // fewer than V keys
        atomicAdd(&s_cnt[i / TILE][(uint32_t)(kp[i] >> shift) & (R - 1)], 1u);
    __syncthreads();
    // per digit: the running count over the chunk's tiles, and the total
    uint32_t run[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        run[k] = 0u;
        if (!owns(k)) continue;
        for (int j = 0; j < nct; ++j) {
            const uint32_t v = s_cnt[j][d0 + k];
            s_cnt[j][d0 + k] = run[k];
            run[k] += v;
        }
    }
    // the chunk's totals: published, then the earlier chunks' summed
    uint32_t excl[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
        excl[k] = 0u;
        if (owns(k))
            __hip_atomic_store(status + (int64_t)c * R + d0 + k,
                               (c == 0 ? kFlagInclusive : kFlagAggregate) | run[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (c > 0 && d0 < R) look_back<DPT>(status, R, c, 0u, d0, run, excl, err);
    uint32_t hv[DPT], hoff[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) hv[k] = owns(k) ? hist[d0 + k] : 0u;
    digits_excl_scan<kCountThreads, DPT>(hv, hoff, s_scan);
    for (int j = 0; j < nct; ++j)
#pragma unroll
        for (int k = 0; k < DPT; ++k)
            if (owns(k)) toff[(tb + j) * R + d0 + k] = hoff[k] + excl[k] + s_cnt[j][d0 + k];
}

// One pass over digit `shift .. shift+nbits` (nbits <= BITS: the last digit
// of a code can be narrower).  With `toff` (one key array, reduce-then-scan
// form): block b is tile b and takes its digits' output positions from
// toff[b] instead of the look-back; `next_rows` rows of `status_next` are
// cleared (by the tiles of those numbers) for the next pass either way.
template <typename K, int THREADS, int ITEMS, int BITS>
__global__ __launch_bounds__(THREADS) void k_onesweep(
    const K *__restrict__ keys_in, K *__restrict__ keys_out, const int32_t *__restrict__ vals_in,
    int32_t *__restrict__ vals_out, int64_t n, SortSegs seg, int shift, int nbits,
    const uint32_t *__restrict__ hist, uint32_t *status, uint32_t *__restrict__ status_next,
    uint32_t next_rows, uint32_t *tile_counter, uint32_t *err, const uint32_t *__restrict__ toff)
{
    constexpr int R = 1 << BITS;
    constexpr int W = THREADS / 64;
    constexpr int TILE = THREADS * ITEMS;
    constexpr int DPT = (R + THREADS - 1) / THREADS;   // digits per owning thread
    static_assert(THREADS % 64 == 0, "whole waves");
    static_assert(TILE < 65536, "16-bit per-wave digit counters");
    using Cnt = typename std::conditional<(BITS <= 9), uint32_t, uint16_t>::type;
    __shared__ uint32_t s_tile;
    __shared__ __align__(16) Cnt s_wcnt[W][R];   // per-wave digit counts, then exclusive offsets
    __shared__ uint32_t s_start[R];          // tile-local start of each digit run
    __shared__ uint32_t s_gbase[R];          // segment-local position of that run
    __shared__ uint32_t s_scan[2][W];
    __shared__ K s_buf[TILE];                // keys, then values

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_tile = toff ? blockIdx.x : atomicAdd(tile_counter, 1u);
    constexpr int kZeroWords = W * R * (int)sizeof(Cnt) / 4;
    for (int j = tid; j < kZeroWords; j += THREADS) reinterpret_cast<uint32_t *>(&s_wcnt[0][0])[j] = 0u;
    __syncthreads();
    const uint32_t tile = s_tile;

    // the tile's segment
    int64_t b0 = 0, ns = n;
    uint32_t t0 = 0, nt = (uint32_t)((n + TILE - 1) / TILE);
    int s = 0;
    if (seg.seg_off) {
        if (tile >= (uint32_t)seg.tile_off[seg.S]) return;   // grid is an upper bound
        s = upper_segment(seg.tile_off, seg.S, tile);
        b0 = seg.seg_off[s];
        ns = seg.seg_off[s + 1] - b0;
        t0 = (uint32_t)seg.tile_off[s];
        nt = (uint32_t)seg.tile_off[s + 1] - t0;
    }
    const uint32_t lt = tile - t0;           // tile index within the segment
    const int64_t base = (int64_t)lt * TILE; // segment-local
    if (status_next && tile < next_rows)
        for (int d = tid; d < R; d += THREADS) status_next[(int64_t)tile * R + d] = 0u;

    // wave w owns keys [base + w*64*ITEMS, ...); item k of lane l is key
    // base + w*64*ITEMS + k*64 + l, so (item, lane) order is input order
    // keys of this tile: rem = how many (at most TILE), tile-local offsets
    // from here on fit 32 bits
    const int64_t rem64 = ns - base;
    const int rem = rem64 < TILE ? (int)rem64 : TILE;
    const int lofs = wave * 64 * ITEMS + lane;   // tile-local offset of item 0
    const K *kp = keys_in + b0 + base + lofs;
    const int32_t *vp = vals_in ? vals_in + b0 + base + lofs : nullptr;
    K key[ITEMS];
    uint32_t dig[ITEMS];   // this pass's digit of each key
    const bool full = rem == TILE;   // every tile but a segment's last: no per-key test
    if (full) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) key[k] = kp[k * 64];
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) key[k] = lofs + k * 64 < rem ? kp[k * 64] : (K)0;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) dig[k] = (uint32_t)(key[k] >> shift) & (R - 1);
    // 64-bit keys wait in LDS (input order) while the tile is ranked: kept
    // in registers, the widest tiles spilled to scratch memory
    if constexpr (sizeof(K) == 8) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) s_buf[lofs + k * 64] = key[k];
    }

    // stable rank within the wave: lanes holding the same digit find each
    // other with one ballot per digit bit; the lowest of them advances the
    // wave's counter
    uint32_t rank[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const bool ok = lofs + k * 64 < rem;
        const uint32_t d = dig[k];
        // bits at or above nbits are zero in every key
        const uint64_t peers = __ballot(ok) & ~digit_diff<BITS>(d);
        const uint32_t below = count_below(peers);
        const uint32_t cnt = s_wcnt[wave][d];
        rank[k] = cnt + below;
        if (ok && below == 0) s_wcnt[wave][d] = (Cnt)(cnt + (uint32_t)__popcll(peers));
    }
    __syncthreads();

    // owning threads: per-wave exclusive offsets of their digits and the
    // tile's totals, published for later tiles
    const int d0 = tid * DPT;
    const bool owner = d0 < R;
    auto owns = [&](int k) { return d0 + k < R; };
    uint32_t total[DPT];
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
            if (nt > 1 && !toff)
                __hip_atomic_store(status + (int64_t)tile * R + d,
                                   (lt == 0 ? kFlagInclusive : kFlagAggregate) | total[k],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    uint32_t start[DPT], hoff[DPT], hv[DPT];
    digits_excl_scan<THREADS, DPT>(total, start, s_scan[0]);
    const uint32_t *hs = hist + (int64_t)s * seg.hist_stride;
#pragma unroll
    for (int k = 0; k < DPT; ++k) hv[k] = (owns(k) && nt > 1 && !toff) ? hs[d0 + k] : 0u;
    digits_excl_scan<THREADS, DPT>(hv, hoff, s_scan[1]);
    if (owner) {
        // decoupled look-back, all of this thread's digits in flight together
        uint32_t excl[DPT];
#pragma unroll
        for (int k = 0; k < DPT; ++k) excl[k] = 0;
        if (nt > 1 && lt > 0 && !toff) look_back<DPT>(status, R, tile, t0, d0, total, excl, err);
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
            if (!owns(k)) continue;
            s_start[d0 + k] = start[k];
            s_gbase[d0 + k] = toff ? toff[(int64_t)tile * R + d0 + k] : (nt > 1 ? hoff[k] + excl[k] : start[k]);
        }
    }
    __syncthreads();

    uint32_t pos[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t dk = dig[k];
        pos[k] = s_start[dk] + s_wcnt[wave][dk] + rank[k];
    }
    if constexpr (sizeof(K) == 8) {
        // the keys back from LDS before their slots are reused
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) key[k] = s_buf[lofs + k * 64];
        __syncthreads();
    }
    // the values, loaded only now (they are needed last; loading them with
    // the keys made the widest tiles spill registers to scratch memory)
    int32_t val[ITEMS];
    if (vp && full) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) val[k] = vp[k * 64];
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const bool ok = lofs + k * 64 < rem;
            val[k] = vp ? (ok ? vp[k * 64] : 0) : (int32_t)(base + lofs + k * 64);
        }
    }
    // keys: into LDS in tile-sorted order, then out in runs (segment-local
    // positions fit 32 bits: a segment holds at most 2^30 keys)
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (lofs + k * 64 < rem) s_buf[pos[k]] = key[k];
    __syncthreads();
    K *ko = keys_out + b0;
    int32_t *vo = vals_out + b0;
    const uint32_t nsu = (uint32_t)ns;
    uint32_t dst[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int p = k * THREADS + tid;
        dst[k] = ~0u;
        if (p < rem) {
            const K kk = s_buf[p];
            const uint32_t dk = (uint32_t)(kk >> shift) & (R - 1);
            const uint32_t out = s_gbase[dk] + (uint32_t)p - s_start[dk];
            if (out < nsu) {
                ko[out] = kk;
                dst[k] = out;
            } else {   // inconsistent histogram: flag it rather than write outside
                __hip_atomic_store(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
    // values: same slots, same destinations
    int32_t *s_vals = reinterpret_cast<int32_t *>(s_buf);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (lofs + k * 64 < rem) s_vals[pos[k]] = val[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (dst[k] != ~0u) vo[dst[k]] = s_vals[k * THREADS + tid];
}

}  // namespace
}  // namespace lbvh
