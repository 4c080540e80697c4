// Device helpers shared by the library's HIP translation units: primitive
// loads, Morton encoding, block scans and reductions, delta* and node
// records.  Everything here is inline device code with internal linkage.
#pragma once
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
template <int THREADS = kBlock>
__device__ __forceinline__ void block_minmax6(float v[6], float *sh /* [THREADS/64][6] */)
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
        for (int w = 1; w < THREADS / 64; ++w)
            for (int a = 0; a < 3; ++a) {
                v[a] = fminf(v[a], sh[w * 6 + a]);
                v[3 + a] = fmaxf(v[3 + a], sh[w * 6 + 3 + a]);
            }
    }
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

// --------------------------------------------------------------- scans

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

// ---------------------------------------------------------- Alg. 4 bits

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

}  // namespace
}  // namespace lbvh
