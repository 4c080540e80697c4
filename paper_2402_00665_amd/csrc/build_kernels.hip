// Rope-LBVH construction on gfx950 (CDNA4, wave64).
//
// Kernels, in launch order:
//   k_bounds / k_bounds_final  scene box: componentwise min/max of all
//                              primitive boxes, then the per-axis scale
//   k_morton                   Morton code per primitive + the digit
//                              histograms of every radix pass
//   k_onesweep (x passes)      LSD radix pass with decoupled look-back
//   k_bottomup_l0 / _up        Alg. 4 in levels of blocks: leaves up, one
//                              CAS per internal node, Karras-ordered parents
//                              with left child, rope and box written by the
//                              second thread to arrive
//
// Floating point follows binary32 with no contraction (the library is built
// with -ffp-contract=off and the pragma below repeats it), no fast-math and
// no denormal flushing, so the codes and boxes are bit-identical to a plain
// IEEE evaluation of the same expressions.
#pragma clang fp contract(off)

#include <math.h>

#include "lbvh_internal.hpp"

namespace lbvh {
namespace {

// ------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t count_below(uint64_t mask)
{
    // number of set bits of `mask` in lanes below this one
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int highest_bit(uint32_t x) { return 31 - __clz(x); }
__device__ __forceinline__ int highest_bit(uint64_t x) { return 63 - __clzll(x); }

// Primitives are read in groups of three float4 (48 bytes): four points or
// two boxes.  The input is 16-byte aligned (checked by the C ABI layer).
template <int KIND> struct Prims;

template <> struct Prims<LBVH_POINTS> {
    static constexpr int G = 4;      // primitives per 48-byte group
    __device__ static void group(const float *p, int64_t g, float lo[G][3], float hi[G][3])
    {
        const float4 *q = reinterpret_cast<const float4 *>(p) + 3 * g;
        float4 a = q[0], b = q[1], c = q[2];
        float v[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int x = 0; x < 3; ++x) lo[k][x] = hi[k][x] = v[3 * k + x];
    }
    __device__ static void one(const float *p, int64_t i, float lo[3], float hi[3])
    {
        const float *s = p + 3 * i;
        lo[0] = hi[0] = s[0]; lo[1] = hi[1] = s[1]; lo[2] = hi[2] = s[2];
    }
    __device__ static float centroid(float lo, float) { return lo; }
};

template <> struct Prims<LBVH_BOXES> {
    static constexpr int G = 2;
    __device__ static void group(const float *p, int64_t g, float lo[G][3], float hi[G][3])
    {
        const float4 *q = reinterpret_cast<const float4 *>(p) + 3 * g;
        float4 a = q[0], b = q[1], c = q[2];
        float v[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int x = 0; x < 3; ++x) { lo[k][x] = v[6 * k + x]; hi[k][x] = v[6 * k + 3 + x]; }
    }
    __device__ static void one(const float *p, int64_t i, float lo[3], float hi[3])
    {
        const float2 *s = reinterpret_cast<const float2 *>(p + 6 * i);
        float2 a = s[0], b = s[1], c = s[2];
        lo[0] = a.x; lo[1] = a.y; lo[2] = b.x; hi[0] = b.y; hi[1] = c.x; hi[2] = c.y;
    }
    __device__ static float centroid(float lo, float hi) { return (lo + hi) * 0.5f; }
};

// Wave64 butterfly min/max of six values, then across the block's waves.
__device__ __forceinline__ void block_minmax6(float v[6], float *sh /* [kBlock/64][6] */)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], __shfl_xor(v[a], off));
            v[3 + a] = fmaxf(v[3 + a], __shfl_xor(v[3 + a], off));
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int a = 0; a < 6; ++a) sh[wave * 6 + a] = v[a];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w)
            for (int a = 0; a < 3; ++a) {
                v[a] = fminf(v[a], sh[w * 6 + a]);
                v[3 + a] = fmaxf(v[3 + a], sh[w * 6 + 3 + a]);
            }
    }
}

// ----------------------------------------------------------- scene box

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_bounds(const float *__restrict__ prims, int n,
                                                   float *__restrict__ partials)
{
    using P = Prims<KIND>;
    __shared__ float sh[(kBlock / 64) * 6];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    const int64_t ng = n / P::G;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < ng; g += stride) {
        float lo[P::G][3], hi[P::G][3];
        P::group(prims, g, lo, hi);
#pragma unroll
        for (int k = 0; k < P::G; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) { v[a] = fminf(v[a], lo[k][a]); v[3 + a] = fmaxf(v[3 + a], hi[k][a]); }
    }
    if (blockIdx.x == 0) {
        for (int64_t i = ng * P::G + threadIdx.x; i < n; i += kBlock) {
            float lo[3], hi[3];
            P::one(prims, i, lo, hi);
            for (int a = 0; a < 3; ++a) { v[a] = fminf(v[a], lo[a]); v[3 + a] = fmaxf(v[3 + a], hi[a]); }
        }
    }
    block_minmax6(v, sh);
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) partials[blockIdx.x * 8 + a] = v[a];
}

// One block: reduce the partials, derive the per-axis quantisation scale
// 2^b / extent (correctly rounded, 0 for a flat axis) and reset the control
// words and digit histograms that the following kernels accumulate into.
__global__ __launch_bounds__(kBlock) void k_bounds_final(const float *__restrict__ partials, int nb,
                                                         int bits_per_axis, float4 *__restrict__ scene,
                                                         uint32_t *__restrict__ ctrl,
                                                         uint32_t *__restrict__ hist, int hist_words)
{
    __shared__ float sh[(kBlock / 64) * 6];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += kBlock)
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], partials[b * 8 + a]);
            v[3 + a] = fmaxf(v[3 + a], partials[b * 8 + 3 + a]);
        }
    block_minmax6(v, sh);
    if (threadIdx.x == 0) {
        const float two_b = (float)(1u << bits_per_axis);
        float s[3];
        for (int a = 0; a < 3; ++a) {
            float ext = v[3 + a] - v[a];
            s[a] = ext > 0.0f ? __fdiv_rn(two_b, ext) : 0.0f;
        }
        scene[0] = make_float4(v[0], v[1], v[2], 0.0f);
        scene[1] = make_float4(v[3], v[4], v[5], 0.0f);
        scene[2] = make_float4(s[0], s[1], s[2], 0.0f);
    }
    for (int w = threadIdx.x; w < kCtrlWords; w += kBlock) ctrl[w] = 0u;
    for (int w = threadIdx.x; w < hist_words; w += kBlock) hist[w] = 0u;
}

// -------------------------------------------------------------- Morton

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint64_t spread21(uint64_t x)
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

template <int B>
__device__ __forceinline__ uint32_t quantize(float c, float lo, float scale)
{
    const float t = (c - lo) * scale;
    constexpr uint32_t maxq = (1u << B) - 1u;
    if (!(t > 0.0f)) return 0u;
    if (t >= (float)maxq) return maxq;
    return (uint32_t)t;
}

template <typename K> struct Code;
template <> struct Code<uint32_t> {
    static constexpr int B = 10;
    __device__ static uint32_t make(uint32_t x, uint32_t y, uint32_t z)
    {
        return (spread10(x) << 2) | (spread10(y) << 1) | spread10(z);
    }
};
template <> struct Code<uint64_t> {
    static constexpr int B = 21;
    __device__ static uint64_t make(uint32_t x, uint32_t y, uint32_t z)
    {
        return (spread21(x) << 2) | (spread21(y) << 1) | spread21(z);
    }
};

template <int KIND, typename K>
__device__ __forceinline__ K code_of(const float lo[3], const float hi[3], float4 slo, float4 sc)
{
    using P = Prims<KIND>;
    constexpr int B = Code<K>::B;
    uint32_t qx = quantize<B>(P::centroid(lo[0], hi[0]), slo.x, sc.x);
    uint32_t qy = quantize<B>(P::centroid(lo[1], hi[1]), slo.y, sc.y);
    uint32_t qz = quantize<B>(P::centroid(lo[2], hi[2]), slo.z, sc.z);
    return Code<K>::make(qx, qy, qz);
}

// Codes in input order, LDS digit histograms of every radix pass folded
// into the global ones, and one side job that must precede the sort: clear
// the look-back status of the first sort pass.
template <int KIND, typename K>
__global__ __launch_bounds__(kBlock) void k_morton(const float *__restrict__ prims, int n,
                                                   const float4 *__restrict__ scene,
                                                   K *__restrict__ codes, uint32_t *__restrict__ hist,
                                                   int passes, uint32_t *__restrict__ status0,
                                                   int64_t status_words)
{
    using P = Prims<KIND>;
    __shared__ uint32_t lh[8 * kRadix];
    for (int j = threadIdx.x; j < passes * kRadix; j += kBlock) lh[j] = 0u;

    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t j = tid; j < status_words; j += stride) status0[j] = 0u;
    __syncthreads();

    const float4 slo = scene[0], sc = scene[2];
    const int64_t ng = n / P::G;
    for (int64_t g = tid; g < ng; g += stride) {
        float lo[P::G][3], hi[P::G][3];
        P::group(prims, g, lo, hi);
        K c[P::G];
#pragma unroll
        for (int k = 0; k < P::G; ++k) {
            c[k] = code_of<KIND, K>(lo[k], hi[k], slo, sc);
            for (int p = 0; p < passes; ++p)
                atomicAdd(&lh[p * kRadix + (uint32_t)((c[k] >> (p * kRadixBits)) & (kRadix - 1))], 1u);
        }
#pragma unroll
        for (int k = 0; k < P::G; ++k) codes[g * P::G + k] = c[k];
    }
    if (blockIdx.x == 0) {
        for (int64_t i = ng * P::G + threadIdx.x; i < n; i += kBlock) {
            float lo[3], hi[3];
            P::one(prims, i, lo, hi);
            K c = code_of<KIND, K>(lo, hi, slo, sc);
            for (int p = 0; p < passes; ++p)
                atomicAdd(&lh[p * kRadix + (uint32_t)((c >> (p * kRadixBits)) & (kRadix - 1))], 1u);
            codes[i] = c;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < passes * kRadix; j += kBlock)
        if (lh[j]) atomicAdd(&hist[j], lh[j]);
}

// ------------------------------------------------------ onesweep pass

// Exclusive scan across the block of one value per thread (THREADS values).
template <int THREADS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh /* [THREADS/64] */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += sh[w];
    return before + x - v;
}

// One LSD radix pass over the 8-bit digit at `shift`.  A block takes the
// next tile id from a counter (so every tile it waits for is already
// running), ranks its THREADS*ITEMS keys stably with wave64 ballots,
// publishes its per-digit counts, looks back over earlier tiles for their
// running totals, and scatters keys, then values, through one LDS buffer so
// that global writes are runs of equal digits.  vals_in == nullptr makes
// the values the input indices.  status_next, when set, is the next pass's
// look-back buffer, cleared here tile by tile.
template <typename K, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_onesweep(
    const K *__restrict__ keys_in, K *__restrict__ keys_out, const int32_t *__restrict__ vals_in,
    int32_t *__restrict__ vals_out, int n, int shift, const uint32_t *__restrict__ hist_pass,
    uint32_t *status, uint32_t *__restrict__ status_next, uint32_t *tile_counter, uint32_t *err)
{
    static_assert(THREADS >= kRadix && THREADS % 64 == 0, "one thread per digit");
    constexpr int W = THREADS / 64;
    constexpr int TILE = THREADS * ITEMS;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint32_t s_start[kRadix];     // tile-local start of each digit run
    __shared__ uint32_t s_gbase[kRadix];     // global position of that run
    __shared__ uint32_t s_scan[2][W];
    __shared__ K s_buf[TILE];                // keys, then values

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int j = tid; j < W * kRadix; j += THREADS) (&s_wcnt[0][0])[j] = 0u;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * TILE;
    if (status_next && tid < kRadix) status_next[(int64_t)tile * kRadix + tid] = 0u;

    // wave w owns keys [base + w*64*ITEMS, ...); item k of lane l is key
    // base + w*64*ITEMS + k*64 + l, so (item, lane) order is input order
    K key[ITEMS];
    int32_t val[ITEMS];
    const int64_t wbase = base + (int64_t)wave * 64 * ITEMS;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t idx = wbase + k * 64 + lane;
        const bool ok = idx < n;
        key[k] = ok ? keys_in[idx] : (K)0;
        val[k] = vals_in ? (ok ? vals_in[idx] : 0) : (int32_t)idx;
    }

    // stable rank within the wave: lanes holding the same digit find each
    // other with 8 ballots; the lowest of them advances the wave's counter
    uint32_t rank[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t idx = wbase + k * 64 + lane;
        const bool ok = idx < n;
        const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = count_below(peers);
        const uint32_t cnt = s_wcnt[wave][d];
        rank[k] = cnt + below;
        if (ok && below == 0) s_wcnt[wave][d] = cnt + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // threads d < 256: per-wave exclusive offsets of digit d and the total
    const uint32_t d = tid;
    uint32_t total = 0;
    if (tid < kRadix) {
        uint32_t c[W];
#pragma unroll
        for (int w = 0; w < W; ++w) c[w] = s_wcnt[w][d];
#pragma unroll
        for (int w = 0; w < W; ++w) { s_wcnt[w][d] = total; total += c[w]; }
        uint32_t *my = status + (int64_t)tile * kRadix + d;
        __hip_atomic_store(my, (tile == 0 ? kFlagInclusive : kFlagAggregate) | total,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t start = block_excl_scan<THREADS>(tid < kRadix ? total : 0u, s_scan[0]);
    const uint32_t hoff = block_excl_scan<THREADS>(tid < kRadix ? hist_pass[d] : 0u, s_scan[1]);
    if (tid < kRadix) {
        s_start[d] = start;
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t j = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (true) {
                const uint32_t sv = __hip_atomic_load(status + j * kRadix + d, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t flag = sv & ~kValueMask;
                if (flag == 0u) {
                    if (++spins > (1u << 24)) {   // never expected: bounded wait
                        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += sv & kValueMask;
                if (flag == kFlagInclusive || j == 0) break;
                --j;
            }
            __hip_atomic_store(status + (int64_t)tile * kRadix + d, kFlagInclusive | (excl + total),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_gbase[d] = hoff + excl;
    }
    __syncthreads();

    uint32_t pos[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t dk = (uint32_t)(key[k] >> shift) & (kRadix - 1);
        pos[k] = s_start[dk] + s_wcnt[wave][dk] + rank[k];
    }
    const int64_t rem = (int64_t)n - base;
    const int valid = rem < TILE ? (int)rem : TILE;

    // keys: into LDS in tile-sorted order, then out in runs
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (wbase + k * 64 + lane < n) s_buf[pos[k]] = key[k];
    __syncthreads();
    int64_t dst[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int p = k * THREADS + tid;
        dst[k] = -1;
        if (p < valid) {
            const K kk = s_buf[p];
            const uint32_t dk = (uint32_t)(kk >> shift) & (kRadix - 1);
            const int64_t out = (int64_t)s_gbase[dk] + (p - (int)s_start[dk]);
            if (out >= 0 && out < n) {
                keys_out[out] = kk;
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
        if (wbase + k * 64 + lane < n) s_vals[pos[k]] = val[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (dst[k] >= 0) vals_out[dst[k]] = s_vals[k * THREADS + tid];
}

// ------------------------------------------------------------ Alg. 4
//
// Alg. 4 runs in levels of blocks so that every compare-and-swap on `store`
// has all of its possible participants inside one workgroup and needs only
// workgroup-scope ordering (an agent-scope acquire-release CAS per tree
// level would write back and invalidate the XCD's L2 every time):
//   level 0   block b takes the kChunk leaves [A, B) = [b*kChunk, ...):
//             leaf records, then the climb with `store` and every box of
//             the chunk in LDS;
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

// delta*(i): rank of the highest differing bit of the augmented keys
// (code, sorted position) of leaves i and i+1; codes that differ rank
// above any index bit.  Out of range (i = -1 or n-1) is +inf (255).
template <typename K>
__device__ __forceinline__ int delta_rank(const K *__restrict__ codes, int i, int n)
{
    if (i < 0 || i >= n - 1) return 255;
    const K x = codes[i] ^ codes[i + 1];
    if (x) return 64 + highest_bit(x);
    return highest_bit((uint32_t)(i ^ (i + 1)));
}

__device__ __forceinline__ void store_node(float4 *nodes, int id, const float lo[3], int left,
                                           const float hi[3], int rope)
{
    float4 *p = nodes + 2 * (int64_t)id;
    p[0] = make_float4(lo[0], lo[1], lo[2], __int_as_float(left));
    p[1] = make_float4(hi[0], hi[1], hi[2], __int_as_float(rope));
}

// A path has at most one node per distinct delta* rank (<= 64 + 31), so a
// climb ends well within this cap; it only guards against corrupted input.
constexpr int kMaxDepth = 256;

template <int KIND, typename K>
__global__ __launch_bounds__(kBU0Threads) void k_bottomup_l0(const K *__restrict__ codes,
                                                             const int32_t *__restrict__ perm,
                                                             const float *__restrict__ prims,
                                                             int n, int32_t *__restrict__ store,
                                                             float4 *__restrict__ nodes,
                                                             int4 *__restrict__ pend,
                                                             uint32_t *err)
{
    __shared__ K s_codes[kChunk + 3];        // codes[A-1 .. B+1]
    __shared__ int32_t s_store[kChunk];      // store[A .. B-1]
    __shared__ float s_box[6][2 * kChunk];   // internal A.. then leaves A..
    __shared__ int4 s_pend[2];

    const int A = blockIdx.x * kChunk;
    const int B = min(A + kChunk, n);
    const int cn = B - A;
    const int leaf0 = n - 1;

    for (int t = threadIdx.x; t < cn + 3; t += kBU0Threads) {
        const int g = A - 1 + t;
        s_codes[t] = (g >= 0 && g < n) ? codes[g] : (K)0;
    }
    for (int t = threadIdx.x; t < kChunk; t += kBU0Threads) s_store[t] = -1;
    if (threadIdx.x < 2) s_pend[threadIdx.x] = make_int4(-1, 0, 0, 0);
    __syncthreads();

    // delta*(g) for g in [A-1, B]
    auto delta = [&](int g) -> int {
        if (g < 0 || g >= n - 1) return 255;
        const K x = s_codes[g - A + 1] ^ s_codes[g - A + 2];
        if (x) return 64 + highest_bit(x);
        return highest_bit((uint32_t)(g ^ (g + 1)));
    };

    // leaves: box, primitive id, rope (Alg. 2 on the range [i, i])
    for (int i = A + threadIdx.x; i < B; i += kBU0Threads) {
        const int prim = perm[i];
        float lo[3], hi[3];
        Prims<KIND>::one(prims, prim, lo, hi);
        const int dr = delta(i);
        const int rope = (i == n - 1) ? -1 : (dr < delta(i + 1) ? leaf0 + i + 1 : i + 1);
        store_node(nodes, leaf0 + i, lo, prim, hi, rope);
        const int sl = kChunk + (i - A);
#pragma unroll
        for (int a = 0; a < 3; ++a) { s_box[a][sl] = lo[a]; s_box[3 + a][sl] = hi[a]; }
    }
    __syncthreads();

    if (n > 1) {
        for (int i = A + threadIdx.x; i < B; i += kBU0Threads) {
            int rl = i, rr = i, cur = leaf0 + i;
            int dl = delta(i - 1), dr = delta(i);
            float lo[3], hi[3];
            const int sl = kChunk + (i - A);
#pragma unroll
            for (int a = 0; a < 3; ++a) { lo[a] = s_box[a][sl]; hi[a] = s_box[3 + a][sl]; }
            for (int level = 0;; ++level) {
                if (level == kMaxDepth) {
                    __hip_atomic_store(err, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                int p, sib;
                if (dr < dl) {                 // left child of its parent
                    p = rr;
                    if (p == B - 1) { s_pend[1] = make_int4(cur, rl, rr, 0); break; }
                    int other = -1;
                    if (__hip_atomic_compare_exchange_strong(&s_store[p - A], &other, rl,
                                                             __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP))
                        break;                 // first to arrive
                    rr = other;
                    dr = delta(rr);
                    sib = (p + 1 == rr) ? leaf0 + p + 1 : p + 1;
                } else {                       // right child of its parent
                    p = rl - 1;
                    if (p == A - 1) { s_pend[0] = make_int4(cur, rl, rr, 0); break; }
                    int other = -1;
                    if (__hip_atomic_compare_exchange_strong(&s_store[p - A], &other, rr,
                                                             __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP))
                        break;
                    rl = other;
                    dl = delta(rl - 1);
                    sib = (rl == p) ? leaf0 + p : p;
                }
                const int ss = sib >= leaf0 ? kChunk + (sib - leaf0 - A) : sib - A;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lo[a] = fminf(lo[a], s_box[a][ss]);
                    hi[a] = fmaxf(hi[a], s_box[3 + a][ss]);
                }
                const int q = dr < dl ? rr : rl;   // Karras index of the parent
                const int left = (rl == p) ? leaf0 + p : p;
                int qrope;
                if (rr == n - 1) qrope = -1;
                else qrope = dr < delta(rr + 1) ? leaf0 + rr + 1 : rr + 1;
                store_node(nodes, q, lo, left, hi, qrope);
                const int qs = q - A;
#pragma unroll
                for (int a = 0; a < 3; ++a) { s_box[a][qs] = lo[a]; s_box[3 + a][qs] = hi[a]; }
                cur = q;
                if (q == 0) break;
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cn; t += kBU0Threads) store[A + t] = s_store[t];
    if (threadIdx.x < 2) pend[2 * blockIdx.x + threadIdx.x] = s_pend[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kBUThreads) void k_bottomup_up(const K *__restrict__ codes, int n,
                                                            int64_t child_span, int64_t span,
                                                            int32_t *store, float4 *nodes,
                                                            const int4 *__restrict__ pend_in,
                                                            int4 *__restrict__ pend_out,
                                                            uint32_t *err)
{
    __shared__ int4 s_pend[2];
    const int64_t A = (int64_t)blockIdx.x * span;
    const int64_t B = A + span < n ? A + span : n;
    const int64_t j0 = A / child_span, j1 = (B + child_span - 1) / child_span;
    const int leaf0 = n - 1;
    if (threadIdx.x < 2) s_pend[threadIdx.x] = make_int4(-1, 0, 0, 0);
    __syncthreads();

    for (int64_t slot = 2 * j0 + threadIdx.x; slot < 2 * j1; slot += kBUThreads) {
        const int4 P = pend_in[slot];
        if (P.x < 0) continue;
        int cur = P.x, rl = P.y, rr = P.z;
        const float4 *own = nodes + 2 * (int64_t)cur;
        const float4 o0 = own[0], o1 = own[1];
        float lo[3] = {o0.x, o0.y, o0.z}, hi[3] = {o1.x, o1.y, o1.z};
        int dl = delta_rank(codes, rl - 1, n), dr = delta_rank(codes, rr, n);
        for (int level = 0;; ++level) {
            if (level == kMaxDepth) {
                __hip_atomic_store(err, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            int p, sib;
            if (dr < dl) {
                p = rr;
                if (p == B - 1) { s_pend[1] = make_int4(cur, rl, rr, 0); break; }
                int other = -1;
                if (__hip_atomic_compare_exchange_strong(&store[p], &other, rl, __ATOMIC_ACQ_REL,
                                                         __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                rr = other;
                dr = delta_rank(codes, rr, n);
                sib = (p + 1 == rr) ? leaf0 + p + 1 : p + 1;
            } else {
                p = rl - 1;
                if (p == A - 1) { s_pend[0] = make_int4(cur, rl, rr, 0); break; }
                int other = -1;
                if (__hip_atomic_compare_exchange_strong(&store[p], &other, rr, __ATOMIC_ACQ_REL,
                                                         __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                rl = other;
                dl = delta_rank(codes, rl - 1, n);
                sib = (rl == p) ? leaf0 + p : p;
            }
            const float4 *sp = nodes + 2 * (int64_t)sib;
            const float4 s0 = sp[0], s1 = sp[1];
            lo[0] = fminf(lo[0], s0.x); lo[1] = fminf(lo[1], s0.y); lo[2] = fminf(lo[2], s0.z);
            hi[0] = fmaxf(hi[0], s1.x); hi[1] = fmaxf(hi[1], s1.y); hi[2] = fmaxf(hi[2], s1.z);
            const int q = dr < dl ? rr : rl;
            const int left = (rl == p) ? leaf0 + p : p;
            int qrope;
            if (rr == n - 1) qrope = -1;
            else qrope = dr < delta_rank(codes, rr + 1, n) ? leaf0 + rr + 1 : rr + 1;
            store_node(nodes, q, lo, left, hi, qrope);
            cur = q;
            if (q == 0) break;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2) pend_out[2 * blockIdx.x + threadIdx.x] = s_pend[threadIdx.x];
}

// Tile shapes of the radix pass (threads x keys per thread); the tuning
// knob "sort_variant" picks one (see lbvh_tune).
struct SortShape { int threads, items; };
constexpr SortShape kSortShapes[] = {{256, 16}, {256, 8}, {256, 24}, {512, 8}, {512, 16}, {1024, 8}};
constexpr int kSortShapeCount = sizeof(kSortShapes) / sizeof(kSortShapes[0]);

template <typename K>
int sort_variant()
{
    const int64_t v = tune_get(sizeof(K) == 4 ? TUNE_SORT_VARIANT32 : TUNE_SORT_VARIANT64);
    return (v >= 0 && v < kSortShapeCount) ? (int)v : 0;
}

template <typename K, int T, int I>
void launch_one(const K *kin, K *kout, const int32_t *vin, int32_t *vout, int n, int shift,
                const uint32_t *hist, uint32_t *st, uint32_t *st_next, uint32_t *ctr, uint32_t *err,
                hipStream_t s)
{
    const unsigned tiles = (unsigned)(((int64_t)n + T * I - 1) / (T * I));
    hipLaunchKernelGGL((k_onesweep<K, T, I>), dim3(tiles), dim3(T), 0, s, kin, kout, vin, vout, n,
                       shift, hist, st, st_next, ctr, err);
}

template <typename K>
void launch_onesweep(int variant, const K *kin, K *kout, const int32_t *vin, int32_t *vout, int n,
                     int shift, const uint32_t *hist, uint32_t *st, uint32_t *st_next, uint32_t *ctr,
                     uint32_t *err, hipStream_t s)
{
    switch (variant) {
    case 1: launch_one<K, 256, 8>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    case 2: launch_one<K, 256, 24>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    case 3: launch_one<K, 512, 8>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    case 4: launch_one<K, 512, 16>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    case 5: launch_one<K, 1024, 8>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    default: launch_one<K, 256, 16>(kin, kout, vin, vout, n, shift, hist, st, st_next, ctr, err, s); break;
    }
}

template <int KIND, typename K>
hipError_t run_build(const float *prims, int n, int code_bits, lbvh_node *nodes_, K *codes,
                     int32_t *leaf_perm, char *ws, const BuildLayout &L, hipStream_t s)
{
    using P = Prims<KIND>;
    float *partials = reinterpret_cast<float *>(ws + L.partials);
    float4 *scene = reinterpret_cast<float4 *>(ws + L.scene);
    uint32_t *ctrl = reinterpret_cast<uint32_t *>(ws + L.ctrl);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *status[2] = {reinterpret_cast<uint32_t *>(ws + L.status[0]),
                           reinterpret_cast<uint32_t *>(ws + L.status[1])};
    K *keys_alt = reinterpret_cast<K *>(ws + L.keys_alt);
    int32_t *vals[2] = {reinterpret_cast<int32_t *>(ws + L.vals[0]),
                        reinterpret_cast<int32_t *>(ws + L.vals[1])};
    int32_t *store = reinterpret_cast<int32_t *>(ws + L.store);
    float4 *nodes = reinterpret_cast<float4 *>(nodes_);
    const int passes = L.passes;

    const int64_t groups = (int64_t)n / P::G;
    int nb = (int)((groups + 4 * kBlock - 1) / (4 * kBlock));
    nb = nb < 1 ? 1 : (nb > kBoundsBlocksMax ? kBoundsBlocksMax : nb);
    prof_begin(K_BOUNDS, s);
    hipLaunchKernelGGL((k_bounds<KIND>), dim3(nb), dim3(kBlock), 0, s, prims, n, partials);
    prof_end(K_BOUNDS, s);
    prof_begin(K_BOUNDS_FINAL, s);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBlock), 0, s, partials, nb, code_bits / 3,
                       scene, ctrl, hist, passes * kRadix);
    prof_end(K_BOUNDS_FINAL, s);

    int nm = (int)((groups + 4 * kBlock - 1) / (4 * kBlock));
    nm = nm < 1 ? 1 : (nm > kMortonBlocksMax ? kMortonBlocksMax : nm);
    prof_begin(K_MORTON, s);
    hipLaunchKernelGGL((k_morton<KIND, K>), dim3(nm), dim3(kBlock), 0, s, prims, n, scene, codes,
                       hist, passes, status[0], L.ntiles * kRadix);
    prof_end(K_MORTON, s);

    // ping-pong: even passes read tree->codes, odd passes write it back;
    // the pass count is even for both code widths, so the sorted codes end
    // in tree->codes; the last pass writes the permutation to leaf_perm
    for (int p = 0; p < passes; ++p) {
        const K *kin = (p & 1) ? keys_alt : codes;
        K *kout = (p & 1) ? codes : keys_alt;
        const int32_t *vin = p == 0 ? nullptr : vals[(p - 1) & 1];
        int32_t *vout = p + 1 == passes ? leaf_perm : vals[p & 1];
        uint32_t *st_next = (p + 1 < passes) ? status[(p + 1) & 1] : nullptr;
        prof_begin(K_SORT, s);
        launch_onesweep<K>(sort_variant<K>(), kin, kout, vin, vout, n, p * kRadixBits,
                           hist + p * kRadix, status[p & 1], st_next, ctrl + kCtrlTileCounter + p,
                           ctrl + kCtrlError, s);
        prof_end(K_SORT, s);
    }

    prof_begin(K_BOTTOMUP, s);
    int4 *pend[2] = {reinterpret_cast<int4 *>(ws + L.pend[0]), reinterpret_cast<int4 *>(ws + L.pend[1])};
    int nbu = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL((k_bottomup_l0<KIND, K>), dim3(nbu), dim3(kBU0Threads), 0, s, codes,
                       leaf_perm, prims, n, store, nodes, pend[0], ctrl + kCtrlError);
    prof_end(K_BOTTOMUP, s);
    int64_t span = kChunk;
    int in = 0;
    while (nbu > 1) {
        const int64_t next = span * kFanout;
        const int nbn = (int)((n + next - 1) / next);
        prof_begin(K_BOTTOMUP_UP, s);
        hipLaunchKernelGGL((k_bottomup_up<K>), dim3(nbn), dim3(kBUThreads), 0, s, codes, n, span,
                           next, store, nodes, pend[in], pend[in ^ 1], ctrl + kCtrlError);
        prof_end(K_BOTTOMUP_UP, s);
        in ^= 1;
        span = next;
        nbu = nbn;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_build(int kind, const float *prims, int n, int code_bits, lbvh_node *nodes,
                        void *codes, int32_t *leaf_perm, char *ws, const BuildLayout &L,
                        hipStream_t s)
{
    if (code_bits == 30) {
        if (kind == LBVH_POINTS)
            return run_build<LBVH_POINTS, uint32_t>(prims, n, code_bits, nodes,
                                                    static_cast<uint32_t *>(codes), leaf_perm, ws,
                                                    L, s);
        return run_build<LBVH_BOXES, uint32_t>(prims, n, code_bits, nodes,
                                               static_cast<uint32_t *>(codes), leaf_perm, ws, L, s);
    }
    if (kind == LBVH_POINTS)
        return run_build<LBVH_POINTS, uint64_t>(prims, n, code_bits, nodes,
                                                static_cast<uint64_t *>(codes), leaf_perm, ws, L,
                                                s);
    return run_build<LBVH_BOXES, uint64_t>(prims, n, code_bits, nodes,
                                           static_cast<uint64_t *>(codes), leaf_perm, ws, L, s);
}

}  // namespace lbvh
