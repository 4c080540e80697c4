// Stackless range queries on gfx950 (Alg. 1) and the CSR offset scan.
//
// One thread per query walks the tree from the root: a node whose box
// passes the test sends the walk to its left child (internal node) or
// reports the primitive (leaf) and follows the rope; a node that fails sends
// it along the rope.  The walk ends at the sentinel -1.  The same walk runs
// twice: the count pass stores hits per query, a three-kernel scan turns the
// counts into int64 offsets, the fill pass writes the primitive indices.
// No contraction: the sphere test is evaluated exactly as written.
#pragma clang fp contract(off)

#include "lbvh_internal.hpp"

namespace lbvh {
namespace {

struct Sphere {
    float cx, cy, cz, r2;
    __device__ void load(const float *q, int j)
    {
        const float4 v = reinterpret_cast<const float4 *>(q)[j];
        cx = v.x; cy = v.y; cz = v.z; r2 = v.w * v.w;
    }
    __device__ bool test(float4 lo, float4 hi) const
    {
        const float dx = fmaxf(fmaxf(lo.x - cx, cx - hi.x), 0.0f);
        const float dy = fmaxf(fmaxf(lo.y - cy, cy - hi.y), 0.0f);
        const float dz = fmaxf(fmaxf(lo.z - cz, cz - hi.z), 0.0f);
        return (dx * dx + dy * dy) + dz * dz <= r2;
    }
};

struct QBox {
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
};

template <class Q, bool FILL>
__global__ __launch_bounds__(kBlock) void k_query(const float4 *__restrict__ nodes, int n,
                                                  const float *__restrict__ queries, int m,
                                                  int32_t *__restrict__ counts,
                                                  const int64_t *__restrict__ offsets,
                                                  int32_t *__restrict__ out)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    Q q;
    q.load(queries, j);
    const int first_leaf = n - 1;
    int64_t pos = FILL ? offsets[j] : 0;
    int cnt = 0;
    int id = 0;
    // ropes only point forward in preorder, so a walk visits each of the
    // 2n-1 nodes at most once; the cap only guards against a corrupt tree
    int64_t budget = 2 * (int64_t)n;
    do {
        if (--budget < 0) break;
        const float4 a = nodes[2 * (int64_t)id];
        const float4 b = nodes[2 * (int64_t)id + 1];
        const bool hit = q.test(a, b);
        const int left = __float_as_int(a.w);
        const int rope = __float_as_int(b.w);
        const bool leaf = id >= first_leaf;
        if (hit && leaf) {
            if (FILL) out[pos++] = left;   // a leaf's `left` is its primitive
            else ++cnt;
        }
        id = (hit && !leaf) ? left : rope;
    } while (id != -1);
    if (!FILL) counts[j] = cnt;
}

__global__ void k_zero_i64(int64_t *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = 0;
}

// -------------------------------------------------------------- scan

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *sh /* [kBlock/64] */, T *block_total)
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

// Sum of each tile of kScanTile counts.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ counts, int m,
                                                        int64_t *__restrict__ partials)
{
    __shared__ int64_t sh[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += counts[base + k];
    int64_t total;
    block_excl_scan<int64_t>(s, sh, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Exclusive scan of the tile sums, in place, by one block.
__global__ __launch_bounds__(kBlock) void k_scan_partials(int64_t *partials, int nb)
{
    __shared__ int64_t sh[kBlock / 64];
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kBlock) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < nb ? partials[b] : 0;
        int64_t total;
        const int64_t e = block_excl_scan<int64_t>(v, sh, &total);
        if (b < nb) partials[b] = carry + e;
        carry += total;
        __syncthreads();
    }
}

// offsets[j] = sum of counts before j; offsets[m] = total.
__global__ __launch_bounds__(kBlock) void k_scan_final(const int32_t *__restrict__ counts, int m,
                                                       const int64_t *__restrict__ partials,
                                                       int64_t *__restrict__ offsets)
{
    __shared__ int64_t sh[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t c[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        c[k] = base + k < m ? counts[base + k] : 0;
        s += c[k];
    }
    int64_t total;
    int64_t run = partials[blockIdx.x] + block_excl_scan<int64_t>(s, sh, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) offsets[base + k] = run;
        run += c[k];
        if (base + k == m - 1) offsets[m] = run;
    }
}

template <class Q>
hipError_t run_query(const lbvh_node *nodes_, int n, const float *q, int m, int64_t *offsets,
                     int32_t *indices, bool fill, char *ws, const QueryLayout &L, hipStream_t s)
{
    const float4 *nodes = reinterpret_cast<const float4 *>(nodes_);
    int32_t *counts = reinterpret_cast<int32_t *>(ws + L.counts);
    int64_t *partials = reinterpret_cast<int64_t *>(ws + L.partials);
    const unsigned gq = (unsigned)((m + kBlock - 1) / kBlock);
    if (fill) {
        if (n == 0 || m == 0) return hipSuccess;
        prof_begin(K_QFILL, s);
        hipLaunchKernelGGL((k_query<Q, true>), dim3(gq), dim3(kBlock), 0, s, nodes, n, q, m, nullptr,
                           offsets, indices);
        prof_end(K_QFILL, s);
        return hipGetLastError();
    }
    if (n == 0 || m == 0) {
        const int64_t cnt = (int64_t)m + 1;
        hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, offsets, cnt);
        return hipGetLastError();
    }
    prof_begin(K_QCOUNT, s);
    hipLaunchKernelGGL((k_query<Q, false>), dim3(gq), dim3(kBlock), 0, s, nodes, n, q, m, counts,
                       nullptr, nullptr);
    prof_end(K_QCOUNT, s);
    const int nb = (int)((m + kScanTile - 1) / kScanTile);
    prof_begin(K_SCAN, s);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, counts, m, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kBlock), 0, s, counts, m, partials, offsets);
    prof_end(K_SCAN, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_query(int qkind, const lbvh_node *nodes, int n, const float *q, int m,
                        int64_t *offsets, int32_t *indices, bool fill, char *ws,
                        const QueryLayout &L, hipStream_t s)
{
    if (qkind == 0) return run_query<Sphere>(nodes, n, q, m, offsets, indices, fill, ws, L, s);
    return run_query<QBox>(nodes, n, q, m, offsets, indices, fill, ws, L, s);
}

}  // namespace lbvh
