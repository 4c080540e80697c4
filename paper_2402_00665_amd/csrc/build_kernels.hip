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

#include "bottomup.hpp"
#include "device_common.hpp"
#include "radix_sort.hpp"

namespace lbvh {
namespace {

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

// Codes in input order, LDS digit histograms of every radix pass (BITS-wide
// digits) folded into the global ones, and one side job that must precede
// the sort: clear the look-back status of the first sort pass.  With
// `reverse` the grid sweeps the primitives from the end of the array to its
// start, the opposite of the scene-box pass just before it, so its first
// reads find the lines that pass touched last (still in the last-level
// cache when the array is larger than that cache); the codes are the same.
template <int KIND, typename K, int BITS>
__global__ __launch_bounds__(kBlock) void k_morton(const float *__restrict__ prims, int n,
                                                   const float4 *__restrict__ scene,
                                                   K *__restrict__ codes, uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ status0,
                                                   int64_t status_words, int reverse)
{
    using P = Prims<KIND>;
    constexpr int R = 1 << BITS;
    constexpr int PASSES = ((sizeof(K) == 4 ? 30 : 63) + BITS - 1) / BITS;
    __shared__ uint32_t lh[PASSES * R];
    for (int j = threadIdx.x; j < PASSES * R; j += kBlock) lh[j] = 0u;

    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t j = tid; j < status_words; j += stride) status0[j] = 0u;
    __syncthreads();

    const float4 slo = scene[0], sc = scene[2];
    const int64_t ng = n / P::G;
    for (int64_t g0 = tid; g0 < ng; g0 += stride) {
        const int64_t g = reverse ? ng - 1 - g0 : g0;
        float lo[P::G][3], hi[P::G][3];
        P::group(prims, g, lo, hi);
        K c[P::G];
#pragma unroll
        for (int k = 0; k < P::G; ++k) {
            c[k] = code_of<KIND, K>(lo[k], hi[k], slo, sc);
#pragma unroll
            for (int p = 0; p < PASSES; ++p)
                atomicAdd(&lh[p * R + (uint32_t)((c[k] >> (p * BITS)) & (R - 1))], 1u);
        }
#pragma unroll
        for (int k = 0; k < P::G; ++k) codes[g * P::G + k] = c[k];
    }
    if (blockIdx.x == 0) {
        for (int64_t i = ng * P::G + threadIdx.x; i < n; i += kBlock) {
            float lo[3], hi[3];
            P::one(prims, i, lo, hi);
            K c = code_of<KIND, K>(lo, hi, slo, sc);
#pragma unroll
            for (int p = 0; p < PASSES; ++p)
                atomicAdd(&lh[p * R + (uint32_t)((c >> (p * BITS)) & (R - 1))], 1u);
            codes[i] = c;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < PASSES * R; j += kBlock)
        if (lh[j]) atomicAdd(&hist[j], lh[j]);
}

// ------------------------------------------------------ launchers

// Tile shapes of the radix pass (threads x keys per thread); the tuning
// knob "sort_variant" picks one (see lbvh_tune).  A shape whose tile is
// below the digit width's minimum, or whose digit tables and key buffer
// exceed the LDS, is replaced by the width's default shape.
struct SortShape { int threads, items; };
constexpr SortShape kSortShapes[] = {{256, 16}, {256, 8}, {256, 24}, {512, 8}, {512, 16}, {1024, 8},
                                     {768, 16}, {1024, 16}, {512, 24}};
constexpr int kSortShapeCount = sizeof(kSortShapes) / sizeof(kSortShapes[0]);

constexpr size_t sort_lds_bytes(int key_bytes, int threads, int items, int bits)
{
    return (size_t)(threads / 64) * ((bits <= 9 ? 4u : 2u) << bits) + (8u << bits) +
           (size_t)threads * items * key_bytes;
}

template <typename K>
int sort_variant(int bits)
{
    const int64_t v = tune_get(sizeof(K) == 4 ? TUNE_SORT_VARIANT32 : TUNE_SORT_VARIANT64);
    const int var = (v >= 0 && v < kSortShapeCount) ? (int)v : 0;
    const SortShape sh = kSortShapes[var];
    const bool fits = sh.threads * sh.items >= radix_min_tile(bits) &&
                      sort_lds_bytes(sizeof(K), sh.threads, sh.items, bits) <= 150 * 1024;
    return fits ? var : (sizeof(K) == 4 ? 4 : 3);   // 512 x 16 / 512 x 8 fit every width
}

// One radix pass: the onesweep kernel alone, or (toff given: the
// reduce-then-scan form) the count kernel over chunks of tiles and then the
// scatter, which reads its tiles' offsets from toff.  `st` is the pass's
// look-back table (per tile, or per chunk), `st_next` the next pass's,
// cleared by this pass's scatter.
template <typename K, int T, int I, int B>
void launch_one(const K *kin, K *kout, const int32_t *vin, int32_t *vout, int n, int shift, int nbits,
                const uint32_t *hist, uint32_t *st, uint32_t *st_next, uint32_t *ctr, uint32_t *err,
                uint32_t *toff, hipStream_t s)
{
    if constexpr (sort_lds_bytes(sizeof(K), T, I, B) > 150 * 1024) {
        return;   // never selected (sort_variant)
    } else {
        const unsigned tiles = (unsigned)(((int64_t)n + T * I - 1) / (T * I));
        const SortSegs one{nullptr, nullptr, 1, 0};
        if (toff) {
            const unsigned chunks = (tiles + kCountChunk - 1) / kCountChunk;
            hipLaunchKernelGGL((k_radix_count<K, B, T * I>), dim3(chunks), dim3(kCountThreads), 0, s, kin,
                               (int64_t)n, shift, hist, st, toff, ctr, err);
            hipLaunchKernelGGL((k_onesweep<K, T, I, B>), dim3(tiles), dim3(T), 0, s, kin, kout, vin, vout,
                               (int64_t)n, one, shift, nbits, hist, st, st_next, chunks, ctr, err,
                               (const uint32_t *)toff);
        } else {
            hipLaunchKernelGGL((k_onesweep<K, T, I, B>), dim3(tiles), dim3(T), 0, s, kin, kout, vin, vout,
                               (int64_t)n, one, shift, nbits, hist, st, st_next, tiles, ctr, err,
                               (const uint32_t *)nullptr);
        }
    }
}

template <typename K, int B>
void launch_onesweep_b(int variant, const K *kin, K *kout, const int32_t *vin, int32_t *vout, int n,
                       int shift, int nbits, const uint32_t *hist, uint32_t *st, uint32_t *st_next,
                       uint32_t *ctr, uint32_t *err, uint32_t *toff, hipStream_t s)
{
#define LBVH_SORT_ARGS kin, kout, vin, vout, n, shift, nbits, hist, st, st_next, ctr, err, toff, s
    switch (variant) {
    case 1: launch_one<K, 256, 8, B>(LBVH_SORT_ARGS); break;
    case 2: launch_one<K, 256, 24, B>(LBVH_SORT_ARGS); break;
    case 3: launch_one<K, 512, 8, B>(LBVH_SORT_ARGS); break;
    case 4: launch_one<K, 512, 16, B>(LBVH_SORT_ARGS); break;
    case 5: launch_one<K, 1024, 8, B>(LBVH_SORT_ARGS); break;
    case 6: launch_one<K, 768, 16, B>(LBVH_SORT_ARGS); break;
    case 7: launch_one<K, 1024, 16, B>(LBVH_SORT_ARGS); break;
    case 8: launch_one<K, 512, 24, B>(LBVH_SORT_ARGS); break;
    default: launch_one<K, 256, 16, B>(LBVH_SORT_ARGS); break;
    }
#undef LBVH_SORT_ARGS
}

// The digit width's Morton kernel and radix passes.  Ping-pong: the Morton
// kernel writes the codes to the buffer that makes the last pass end in
// tree->codes (keys_alt for an odd number of passes); the last pass writes
// the permutation to leaf_perm.  Look-back tables: the two status buffers
// in turn (onesweep), or status[0] for the chunks of every pass and
// status[1] for the tiles' offsets (reduce-then-scan, "radix_mode" 1).
template <int KIND, typename K, int B>
void run_sort(const float *prims, int n, int code_bits, K *codes, int32_t *leaf_perm,
              const float4 *scene, uint32_t *ctrl, uint32_t *hist, uint32_t *status[2], K *keys_alt,
              int32_t *vals[2], hipStream_t s)
{
    using P = Prims<KIND>;
    const int passes = radix_passes(code_bits, B);
    const int variant = sort_variant<K>(B);
    const int tile = kSortShapes[variant].threads * kSortShapes[variant].items;
    const int64_t tiles = ((int64_t)n + tile - 1) / tile;
    K *first = (passes & 1) ? keys_alt : codes;
    K *second = (passes & 1) ? codes : keys_alt;

    const int64_t groups = (int64_t)n / P::G;
    int nm = (int)((groups + 4 * kBlock - 1) / (4 * kBlock));
    // fewer, longer blocks for wide digits: each block adds its whole
    // histogram table to the global one
    const int nm_max = B <= 8 ? kMortonBlocksMax : (B <= 10 ? kMortonBlocksMax / 2 : kMortonBlocksMax / 4);
    nm = nm < 1 ? 1 : (nm > nm_max ? nm_max : nm);
    prof_begin(K_MORTON, s);
    hipLaunchKernelGGL((k_morton<KIND, K, B>), dim3(nm), dim3(kBlock), 0, s, prims, n, scene, first,
                       hist, status[0], tiles << B, (int)tune_get(TUNE_MORTON_ORDER));
    prof_end(K_MORTON, s);

    const bool rts = tune_get(TUNE_RADIX_MODE) == 1;
    for (int p = 0; p < passes; ++p) {
        const K *kin = (p & 1) ? second : first;
        K *kout = (p & 1) ? first : second;
        const int32_t *vin = p == 0 ? nullptr : vals[(p - 1) & 1];
        int32_t *vout = p + 1 == passes ? leaf_perm : vals[p & 1];
        uint32_t *st = rts ? status[0] : status[p & 1];
        uint32_t *st_next = (p + 1 < passes) ? (rts ? status[0] : status[(p + 1) & 1]) : nullptr;
        const int nbits = std::min(B, code_bits - p * B);
        prof_begin(K_SORT, s);
        launch_onesweep_b<K, B>(variant, kin, kout, vin, vout, n, p * B, nbits, hist + ((int64_t)p << B),
                                st, st_next, ctrl + kCtrlTileCounter + p, ctrl + kCtrlError,
                                rts ? status[1] : nullptr, s);
        prof_end(K_SORT, s);
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
    const int bits = radix_bits(code_bits);

    const int64_t groups = (int64_t)n / P::G;
    int nb = (int)((groups + 4 * kBlock - 1) / (4 * kBlock));
    nb = nb < 1 ? 1 : (nb > kBoundsBlocksMax ? kBoundsBlocksMax : nb);
    prof_begin(K_BOUNDS, s);
    hipLaunchKernelGGL((k_bounds<KIND>), dim3(nb), dim3(kBlock), 0, s, prims, n, partials);
    prof_end(K_BOUNDS, s);
    prof_begin(K_BOUNDS_FINAL, s);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBlock), 0, s, partials, nb, code_bits / 3,
                       scene, ctrl, hist, (int)((int64_t)radix_passes(code_bits, bits) << bits));
    prof_end(K_BOUNDS_FINAL, s);

    if constexpr (sizeof(K) == 4) {
        if (bits == 10)
            run_sort<KIND, K, 10>(prims, n, code_bits, codes, leaf_perm, scene, ctrl, hist, status,
                                  keys_alt, vals, s);
        else
            run_sort<KIND, K, 8>(prims, n, code_bits, codes, leaf_perm, scene, ctrl, hist, status,
                                 keys_alt, vals, s);
    } else {
        if (bits == 11)
            run_sort<KIND, K, 11>(prims, n, code_bits, codes, leaf_perm, scene, ctrl, hist, status,
                                  keys_alt, vals, s);
        else if (bits == 9)
            run_sort<KIND, K, 9>(prims, n, code_bits, codes, leaf_perm, scene, ctrl, hist, status,
                                 keys_alt, vals, s);
        else
            run_sort<KIND, K, 8>(prims, n, code_bits, codes, leaf_perm, scene, ctrl, hist, status,
                                 keys_alt, vals, s);
    }

    prof_begin(K_BOTTOMUP, s);
    Climb *pend[2] = {reinterpret_cast<Climb *>(ws + L.pend[0]), reinterpret_cast<Climb *>(ws + L.pend[1])};
    int nbu = (n + kChunk - 1) / kChunk;
    BatchLevel one{nullptr, nullptr, nullptr, 1, nbu == 1};
    // delta* bytes for the upper levels of a tree too large for packed
    // store words: in the sort's other key buffer, free now
    uint8_t *dstar = reinterpret_cast<uint8_t *>(keys_alt);
    const bool packed = n <= kPackedMaxN;
    if (packed)
        hipLaunchKernelGGL((k_bottomup_l0<KIND, K, true>), dim3(nbu), dim3(kBU0Threads), 0, s, codes,
                           leaf_perm, prims, n, store, nodes, pend[0], one, dstar, ctrl + kCtrlError);
    else
        hipLaunchKernelGGL((k_bottomup_l0<KIND, K, false>), dim3(nbu), dim3(kBU0Threads), 0, s, codes,
                           leaf_perm, prims, n, store, nodes, pend[0], one, dstar, ctrl + kCtrlError);
    prof_end(K_BOTTOMUP, s);
    int64_t span = kChunk;
    int in = 0;
    while (nbu > 1) {
        const int64_t next = span * kFanout;
        const int nbn = (int)((n + next - 1) / next);
        one.last = nbn == 1;
        prof_begin(K_BOTTOMUP_UP, s);
        if (packed)
            hipLaunchKernelGGL(k_bottomup_up<true>, dim3(nbn), dim3(kBUThreads), 0, s, dstar, n, span,
                               next, store, nodes, pend[in], pend[in ^ 1], one, ctrl + kCtrlError);
        else
            hipLaunchKernelGGL(k_bottomup_up<false>, dim3(nbn), dim3(kBUThreads), 0, s, dstar, n, span,
                               next, store, nodes, pend[in], pend[in ^ 1], one, ctrl + kCtrlError);
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
