// C ABI of the rope-LBVH library: argument checks, workspace layout,
// launch sequencing on the caller's stream, per-kernel event timing.
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "lbvh_internal.hpp"

namespace lbvh {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

BuildLayout build_layout(int64_t n, int code_bits)
{
    BuildLayout L{};
    const size_t kb = (size_t)key_bytes(code_bits);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    L.scene = take(3 * sizeof(float4));
    L.partials = take((size_t)kBoundsBlocksMax * 8 * sizeof(float));
    L.ctrl = take(kCtrlWords * sizeof(uint32_t));
    L.hist = take((size_t)radix_hist_words(code_bits) * sizeof(uint32_t));
    const size_t status_words = (size_t)radix_status_words(n, code_bits, 0);
    L.status[0] = take(status_words * sizeof(uint32_t));
    L.status[1] = take(status_words * sizeof(uint32_t));
    L.keys_alt = take((size_t)n * kb);
    L.vals[0] = take((size_t)n * sizeof(int32_t));
    L.vals[1] = take((size_t)n * sizeof(int32_t));
    L.store = take((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    const int64_t nb0 = (n + kChunk - 1) / kChunk;
    const int64_t nb1 = (n + (int64_t)kChunk * kFanout - 1) / ((int64_t)kChunk * kFanout);
    L.pend[0] = take((size_t)(2 * nb0 + 2) * kClimbBytes);
    L.pend[1] = take((size_t)(2 * nb1 + 2) * kClimbBytes);
    L.total = off;
    return L;
}

QueryLayout query_layout(int64_t m)
{
    QueryLayout L{};
    L.cap1 = 2 * m + 1024;
    L.cap2 = 6 * m + 4096;
    L.out1 = L.cap1 + m;        // an unsplit query adds one piece
    L.out2 = L.cap2 + L.out1;   // an unsplit level-1 piece adds one
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    L.cnt1 = take((size_t)(m + 1) * sizeof(int32_t));
    L.off1 = take((size_t)(m + 1) * sizeof(int64_t));
    L.items1 = take((size_t)L.out1 * 16);
    L.cnt2 = take((size_t)L.out1 * sizeof(int32_t));
    L.off2 = take((size_t)(L.out1 + 1) * sizeof(int64_t));
    L.items2 = take((size_t)L.out2 * 16);
    L.app_piece = take((size_t)L.cap2 * 16);   // shared by both levels (cap2 >= cap1)
    L.app_item = take((size_t)L.cap2 * sizeof(int64_t));
    L.app_rank = take((size_t)L.cap2 * sizeof(int32_t));
    L.hcnt = take((size_t)L.out2 * sizeof(int32_t));
    L.hmask = take((size_t)L.out2 * kMaskWords * sizeof(uint64_t));
    L.hoff = take((size_t)(L.out2 + 1) * sizeof(int64_t));
    L.partials = take((size_t)((L.out2 + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t));
    L.ctrl = take(128);
    L.qsorted = take((size_t)m * 8 * sizeof(float));   // widest query: a ray
    L.qperm = take((size_t)m * sizeof(int32_t));
    L.qoff = take((size_t)(m + 1) * sizeof(int64_t));
    L.total = off;
    // the query-order sort's buffers live in `hmask`, which is first
    // written by the leaf level, after the sort is done with them
    const size_t qtiles = (size_t)((m + kQOrderTile - 1) / kQOrderTile);
    size_t q = L.hmask;
    auto inner = [&](size_t bytes) { size_t at = q; q = align256(q + bytes); return at; };
    L.qkeys[0] = inner((size_t)m * sizeof(uint32_t));
    L.qkeys[1] = inner((size_t)m * sizeof(uint32_t));
    L.qvals = inner((size_t)m * sizeof(int32_t));
    L.qstatus[0] = inner(qtiles * kRadix * sizeof(uint32_t));
    L.qstatus[1] = inner(qtiles * kRadix * sizeof(uint32_t));
    L.qhist = inner((size_t)kQOrderPasses * kRadix * sizeof(uint32_t));
    // hmask holds 32 * out2 >= 288 m + 163840 bytes: more than the above
    return L;
}

QueryLayout batch_query_layout(int64_t m)
{
    QueryLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    L.cnt1 = take((size_t)(m + 1) * sizeof(int32_t));
    L.hcache = take((size_t)m * 64 * sizeof(int32_t));   // first 64 hits of each query
    L.partials = take((size_t)((m + kScanTile - 1) / kScanTile + 1) * sizeof(int64_t));
    L.ctrl = take(128);
    L.total = off;
    return L;
}

int batch_levels(int64_t max_scene)
{
    int levels = 0;
    for (int64_t span = kChunk; span < max_scene; span *= kFanout) ++levels;
    return levels;
}

BatchLayout batch_layout(int64_t N, int S, int64_t max_scene, int code_bits)
{
    BatchLayout L{};
    const size_t kb = (size_t)key_bytes(code_bits);
    L.levels = batch_levels(max_scene);
    int64_t span = kChunk;
    for (int lv = 0; lv <= L.levels; ++lv, span *= kFanout) L.blocks_max[lv] = (N + span - 1) / span + S;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
    L.ctrl = take(kCtrlWords * sizeof(uint32_t));
    L.scene_box = take((size_t)S * 3 * sizeof(float4));
    L.tile_off = take((size_t)(S + 1) * sizeof(int32_t));
    L.order = take((size_t)(S > 0 ? S : 1) * sizeof(int32_t));
    L.blk_off = take((size_t)(L.levels + 1) * (S + 1) * sizeof(int32_t));
    L.hist = take((size_t)S * radix_hist_words(code_bits) * sizeof(uint32_t));
    const size_t status_words = (size_t)radix_status_words(N, code_bits, S);
    L.status[0] = take(status_words * sizeof(uint32_t));
    L.status[1] = take(status_words * sizeof(uint32_t));
    L.keys_alt = take((size_t)N * kb);
    L.vals[0] = take((size_t)N * sizeof(int32_t));
    L.vals[1] = take((size_t)N * sizeof(int32_t));
    L.store = take((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    L.pend[0] = take((size_t)2 * L.blocks_max[0] * kClimbBytes);
    L.pend[1] = take((size_t)2 * L.blocks_max[0] * kClimbBytes);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- tuning

namespace {
// defaults measured on MI355X: 8-bit digits and 512 x 16 tiles for 30-bit
// keys, 9-bit digits and 768 x 16 tiles for 63-bit keys; the Morton kernel
// sweeping backwards
std::atomic<int64_t> g_tune[TUNE_NUM] = {{4}, {6}, {0}, {kSplit1}, {kSplit2}, {0}, {0}, {8}, {9}, {0},
                                         {1}, {0}, {0}};
const char *kTuneNames[TUNE_NUM] = {"sort_variant32", "sort_variant64", "batch_sort_variant",
                                    "query_split1", "query_split2", "query_leaf_mode",
                                    "query_order", "radix_bits32", "radix_bits64",
                                    "query_walk_budget", "morton_order", "batch_sort_mode",
                                    "radix_mode"};
const int64_t kTuneMin[TUNE_NUM] = {0, 0, 0, 2, 2, 0, 0, 8, 8, 0, 0, 0, 0};   // accepted values: min .. max
const int64_t kTuneMax[TUNE_NUM] = {8, 8, 3, 24, 24, 1, 1, 10, 11, INT32_MAX, 1, 1, 1};
}  // namespace

int64_t tune_get(int knob) { return g_tune[knob].load(std::memory_order_relaxed); }

int radix_bits(int code_bits)
{
    const int b = (int)tune_get(code_bits <= 32 ? TUNE_RADIX_BITS32 : TUNE_RADIX_BITS64);
    return radix_bits_ok(code_bits, b) ? b : 8;
}

// ---------------------------------------------------------------- timing

namespace {
struct Profiler {
    std::mutex mu;
    bool on = false;
    hipEvent_t open[K_NUM] = {};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[K_NUM];
    double ms[K_NUM] = {};
    int64_t launches[K_NUM] = {};
    std::vector<hipEvent_t> pool;

    hipEvent_t get()
    {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void drain(int id)
    {
        for (auto &pr : pending[id]) {
            float t = 0.0f;
            if (hipEventSynchronize(pr.second) == hipSuccess &&
                hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
                ms[id] += t;
                launches[id] += 1;
            }
            pool.push_back(pr.first);
            pool.push_back(pr.second);
        }
        pending[id].clear();
    }
};
Profiler &prof()
{
    static Profiler p;
    return p;
}
const char *kNames[K_NUM] = {"bounds", "bounds_final", "morton", "sort_pass", "bottomup",
                             "query_count", "query_fill", "scan", "query_split", "bottomup_up",
                             "batch_prep", "query_order"};
}  // namespace

void prof_begin(int id, hipStream_t s)
{
    Profiler &P = prof();
    if (!P.on) return;
    std::lock_guard<std::mutex> g(P.mu);
    hipEvent_t e = P.get();
    if (e && hipEventRecord(e, s) == hipSuccess) P.open[id] = e;
}

void prof_end(int id, hipStream_t s)
{
    Profiler &P = prof();
    if (!P.on) return;
    std::lock_guard<std::mutex> g(P.mu);
    hipEvent_t e = P.get();
    if (!e || !P.open[id]) return;
    if (hipEventRecord(e, s) == hipSuccess) P.pending[id].push_back({P.open[id], e});
    P.open[id] = nullptr;
}

}  // namespace lbvh

using namespace lbvh;

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ------------------------------------------------ allocation-free build
//
// Scratch of lbvh_build_noalloc: a fixed array in device memory, one copy
// per GPU at its own address, held until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: the device
// address is taken once per device, with that device current, through
// hipGetSymbolAddress, and only that address is ever handed to kernels.
static __device__ __align__(256) char scratch[LBVH_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

// the current device's scratch address (looked up on its first use)
hipError_t noalloc_scratch(char **out)
{
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)); e != hipSuccess) return e;
        g_scratch_addr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

// the build's error word to the caller's flag
__global__ void k_copy_word(const uint32_t *src, uint32_t *dst) { *dst = *src; }
}  // namespace

// HIP error behind the last LBVH_EHIP returned on this thread.
static thread_local hipError_t t_last_hip = hipSuccess;

static int hip_status(hipError_t e)
{
    if (e == hipSuccess) return LBVH_OK;
    t_last_hip = e;
    return LBVH_EHIP;
}

extern "C" {

const char *lbvh_strerror(int status)
{
    switch (status) {
    case LBVH_OK: return "ok";
    case LBVH_EINVAL: return "invalid argument";
    case LBVH_ENOSPACE: return "workspace too small";
    case LBVH_EHIP: return "HIP launch or runtime error";
    case LBVH_EDEVICE: return "device-side error flagged by a kernel";
    case LBVH_ELIMIT: return "n exceeds the allocation-free build's fixed scratch (LBVH_NOALLOC_MAX_PRIMS)";
    default: return "unknown status";
    }
}

int64_t lbvh_build_workspace_bytes(int64_t n, int32_t code_bits, int32_t kind)
{
    if (n < 0 || n > LBVH_MAX_PRIMS || (code_bits != 30 && code_bits != 63) ||
        (kind != LBVH_POINTS && kind != LBVH_BOXES))
        return LBVH_EINVAL;
    return (int64_t)build_layout(n, code_bits).total;
}

int lbvh_build(int32_t kind, const float *prims, int64_t n, int32_t code_bits, lbvh_tree *tree,
               void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!tree || n < 0 || n > LBVH_MAX_PRIMS || (code_bits != 30 && code_bits != 63) ||
        (kind != LBVH_POINTS && kind != LBVH_BOXES))
        return LBVH_EINVAL;
    if (n == 0) {
        tree->n = 0;
        tree->code_bits = code_bits;
        tree->kind = kind;
        return LBVH_OK;
    }
    if (!prims || !tree->nodes || !tree->codes || !tree->leaf_perm || !workspace ||
        !aligned(prims, 16) || !aligned(tree->nodes, 16) || !aligned(tree->codes, 16) ||
        !aligned(tree->leaf_perm, 16) || !aligned(workspace, 256))
        return LBVH_EINVAL;
    const BuildLayout L = build_layout(n, code_bits);
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    tree->n = n;
    tree->code_bits = code_bits;
    tree->kind = kind;
    hipError_t e = launch_build(kind, prims, (int)n, code_bits, tree->nodes, tree->codes,
                                tree->leaf_perm, static_cast<char *>(workspace), L,
                                (hipStream_t)stream);
    return hip_status(e);
}

int lbvh_build_noalloc(int32_t kind, const float *prims, int64_t n, int32_t code_bits,
                       lbvh_tree *tree, uint32_t *error_out, void *stream)
{
    if (!tree || n < 0 || n > LBVH_MAX_PRIMS || (code_bits != 30 && code_bits != 63) ||
        (kind != LBVH_POINTS && kind != LBVH_BOXES))
        return LBVH_EINVAL;
    if (n > LBVH_NOALLOC_MAX_PRIMS) return LBVH_ELIMIT;
    if (error_out && !aligned(error_out, 4)) return LBVH_EINVAL;
    if (n == 0) {
        tree->n = 0;
        tree->code_bits = code_bits;
        tree->kind = kind;
        return LBVH_OK;
    }
    if (!prims || !tree->nodes || !tree->codes || !tree->leaf_perm || !aligned(prims, 16) ||
        !aligned(tree->nodes, 16) || !aligned(tree->codes, 16) || !aligned(tree->leaf_perm, 16))
        return LBVH_EINVAL;
    const BuildLayout L = build_layout(n, code_bits);
    if ((int64_t)L.total > LBVH_NOALLOC_SCRATCH_BYTES) return LBVH_ELIMIT;   // not for n within the limit
    char *ws = nullptr;
    if (hipError_t e = noalloc_scratch(&ws); e != hipSuccess) return hip_status(e);
    tree->n = n;
    tree->code_bits = code_bits;
    tree->kind = kind;
    hipError_t e = launch_build(kind, prims, (int)n, code_bits, tree->nodes, tree->codes,
                                tree->leaf_perm, ws, L, (hipStream_t)stream);
    if (e == hipSuccess && error_out) {
        hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(1), 0, (hipStream_t)stream,
                           reinterpret_cast<const uint32_t *>(ws + L.ctrl) + kCtrlError, error_out);
        e = hipGetLastError();
    }
    return hip_status(e);
}

int lbvh_build_points(const float *xyz, int64_t n, int32_t code_bits, lbvh_tree *tree,
                      void *workspace, int64_t workspace_bytes, void *stream)
{
    return lbvh_build(LBVH_POINTS, xyz, n, code_bits, tree, workspace, workspace_bytes, stream);
}

int lbvh_build_boxes(const float *lohi, int64_t n, int32_t code_bits, lbvh_tree *tree,
                     void *workspace, int64_t workspace_bytes, void *stream)
{
    return lbvh_build(LBVH_BOXES, lohi, n, code_bits, tree, workspace, workspace_bytes, stream);
}

int lbvh_build_check(const void *workspace, int64_t n, int32_t code_bits, int32_t kind,
                     void *stream)
{
    if (lbvh_build_workspace_bytes(n, code_bits, kind) < 0 || !workspace) return LBVH_EINVAL;
    if (hipError_t e = hipStreamSynchronize((hipStream_t)stream); e != hipSuccess) return hip_status(e);
    if (n == 0) return LBVH_OK;
    const BuildLayout L = build_layout(n, code_bits);
    uint32_t flag = 0;
    if (hipError_t e = hipMemcpy(&flag,
                                 static_cast<const char *>(workspace) + L.ctrl +
                                     kCtrlError * sizeof(uint32_t),
                                 sizeof(flag), hipMemcpyDeviceToHost);
        e != hipSuccess)
        return hip_status(e);
    return flag ? LBVH_EDEVICE : LBVH_OK;
}

// ------------------------------------------------------------- batched

static bool batch_args_ok(int64_t N, int32_t S, int64_t max_scene, int32_t code_bits, int32_t kind)
{
    return N >= 0 && N <= LBVH_MAX_PRIMS && S >= 0 && max_scene >= 0 &&
           max_scene <= LBVH_MAX_PRIMS && (code_bits == 30 || code_bits == 63) &&
           (kind == LBVH_POINTS || kind == LBVH_BOXES);
}

int64_t lbvh_build_batched_workspace_bytes(int64_t total_n, int32_t num_scenes, int64_t max_scene,
                                           int32_t code_bits, int32_t kind)
{
    if (!batch_args_ok(total_n, num_scenes, max_scene, code_bits, kind)) return LBVH_EINVAL;
    return (int64_t)batch_layout(total_n, num_scenes, max_scene, code_bits).total;
}

int lbvh_build_batched(int32_t kind, const float *prims, lbvh_batch *b, void *workspace,
                       int64_t workspace_bytes, void *stream)
{
    if (!b || !batch_args_ok(b->total_n, b->num_scenes, b->max_scene, b->code_bits, kind))
        return LBVH_EINVAL;
    b->kind = kind;
    if (b->num_scenes == 0 || b->total_n == 0) return LBVH_OK;
    if (!prims || !b->seg_off || !b->nodes || !b->codes || !b->leaf_perm || !workspace ||
        !aligned(prims, 8) || !aligned(b->seg_off, 8) || !aligned(b->nodes, 16) ||
        !aligned(b->codes, 16) || !aligned(b->leaf_perm, 16) || !aligned(workspace, 256))
        return LBVH_EINVAL;
    const BatchLayout L = batch_layout(b->total_n, b->num_scenes, b->max_scene, b->code_bits);
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    hipError_t e = launch_build_batched(kind, prims, b, L.levels, static_cast<char *>(workspace), L,
                                        (hipStream_t)stream);
    return hip_status(e);
}

int lbvh_build_batched_check(const void *workspace, const lbvh_batch *b, void *stream)
{
    if (!b || !workspace) return LBVH_EINVAL;
    if (hipError_t e = hipStreamSynchronize((hipStream_t)stream); e != hipSuccess) return hip_status(e);
    if (b->num_scenes == 0 || b->total_n == 0) return LBVH_OK;
    const BatchLayout L = batch_layout(b->total_n, b->num_scenes, b->max_scene, b->code_bits);
    uint32_t flag = 0;
    if (hipError_t e = hipMemcpy(&flag,
                                 static_cast<const char *>(workspace) + L.ctrl +
                                     kCtrlError * sizeof(uint32_t),
                                 sizeof(flag), hipMemcpyDeviceToHost);
        e != hipSuccess)
        return hip_status(e);
    return flag ? LBVH_EDEVICE : LBVH_OK;
}

int lbvh_build_batched_status_async(const void *workspace, const lbvh_batch *b,
                                    uint32_t *flag_out, void *stream)
{
    if (!b || !workspace || !flag_out) return LBVH_EINVAL;
    if (!batch_args_ok(b->total_n, b->num_scenes, b->max_scene, b->code_bits, LBVH_POINTS))
        return LBVH_EINVAL;
    if (b->num_scenes == 0 || b->total_n == 0) return LBVH_OK;   // nothing built, flag untouched
    const BatchLayout L = batch_layout(b->total_n, b->num_scenes, b->max_scene, b->code_bits);
    const hipError_t e = hipMemcpyAsync(flag_out,
                                        static_cast<const char *>(workspace) + L.ctrl +
                                            kCtrlError * sizeof(uint32_t),
                                        sizeof(uint32_t), hipMemcpyDefault, (hipStream_t)stream);
    return e == hipSuccess ? LBVH_OK : hip_status(e);
}

int64_t lbvh_query_batched_workspace_bytes(int64_t m)
{
    if (m < 0 || m > INT32_MAX) return LBVH_EINVAL;
    return (int64_t)batch_query_layout(m).total;
}

static int batched_query(int qkind, const lbvh_batch *b, const float *q, const int64_t *qseg_off,
                         int64_t m, int64_t *offsets, int32_t *indices, bool fill, void *workspace,
                         int64_t workspace_bytes, void *stream)
{
    if (!b || m < 0 || m > INT32_MAX || !offsets || !aligned(offsets, 8)) return LBVH_EINVAL;
    if (m > 0 && (!q || !aligned(q, 16) || !qseg_off || b->num_scenes < 1 || !b->seg_off ||
                  !b->nodes || !b->leaf_perm || !aligned(b->nodes, 16)))
        return LBVH_EINVAL;
    if (fill && m > 0 && !indices) return LBVH_EINVAL;
    const QueryLayout L = batch_query_layout(m);
    if (!workspace || !aligned(workspace, 256)) return LBVH_EINVAL;
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    hipError_t e = launch_query_batched(qkind, b, q, qseg_off, m, offsets, indices, fill,
                                        static_cast<char *>(workspace), L, (hipStream_t)stream);
    return hip_status(e);
}

int lbvh_query_batched_spheres_count(const lbvh_batch *b, const float *xyzr, const int64_t *qseg_off,
                                     int64_t m, int64_t *offsets, void *workspace,
                                     int64_t workspace_bytes, void *stream)
{
    return batched_query(0, b, xyzr, qseg_off, m, offsets, nullptr, false, workspace,
                         workspace_bytes, stream);
}

int lbvh_query_batched_boxes_count(const lbvh_batch *b, const float *lohi, const int64_t *qseg_off,
                                   int64_t m, int64_t *offsets, void *workspace,
                                   int64_t workspace_bytes, void *stream)
{
    return batched_query(1, b, lohi, qseg_off, m, offsets, nullptr, false, workspace,
                         workspace_bytes, stream);
}

int lbvh_query_batched_spheres_fill(const lbvh_batch *b, const float *xyzr, const int64_t *qseg_off,
                                    int64_t m, const int64_t *offsets, int32_t *indices,
                                    const void *workspace, int64_t workspace_bytes, void *stream)
{
    return batched_query(0, b, xyzr, qseg_off, m, const_cast<int64_t *>(offsets), indices, true,
                         const_cast<void *>(workspace), workspace_bytes, stream);
}

int lbvh_query_batched_boxes_fill(const lbvh_batch *b, const float *lohi, const int64_t *qseg_off,
                                  int64_t m, const int64_t *offsets, int32_t *indices,
                                  const void *workspace, int64_t workspace_bytes, void *stream)
{
    return batched_query(1, b, lohi, qseg_off, m, const_cast<int64_t *>(offsets), indices, true,
                         const_cast<void *>(workspace), workspace_bytes, stream);
}

int64_t lbvh_query_workspace_bytes(int64_t m)
{
    if (m < 0 || m > INT32_MAX) return LBVH_EINVAL;
    return (int64_t)query_layout(m).total;
}

static int query_count(int qkind, const lbvh_tree *tree, const float *q, int64_t m, int64_t *offsets,
                       void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!tree || m < 0 || m > INT32_MAX || tree->n < 0 || tree->n > LBVH_MAX_PRIMS || !offsets ||
        !aligned(offsets, 8))
        return LBVH_EINVAL;
    if (m > 0 && (!q || !aligned(q, 16))) return LBVH_EINVAL;
    if (tree->n > 0 && (!tree->nodes || !tree->leaf_perm || !aligned(tree->nodes, 16)))
        return LBVH_EINVAL;
    const QueryLayout L = query_layout(m);
    if (!workspace || !aligned(workspace, 256)) return LBVH_EINVAL;
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    hipError_t e = launch_query(qkind, tree->kind, tree->nodes, tree->leaf_perm, (int)tree->n, q, (int)m,
                                offsets, nullptr, false,
                                static_cast<char *>(workspace), L, (hipStream_t)stream);
    return hip_status(e);
}

static int query_fill(int qkind, const lbvh_tree *tree, const float *q, int64_t m, int32_t *indices,
                      const void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!tree || m < 0 || m > INT32_MAX || tree->n < 0 || tree->n > LBVH_MAX_PRIMS)
        return LBVH_EINVAL;
    if (m > 0 && (!q || !aligned(q, 16))) return LBVH_EINVAL;
    if (tree->n > 0 && m > 0 &&
        (!tree->nodes || !tree->leaf_perm || !indices || !aligned(tree->nodes, 16)))
        return LBVH_EINVAL;
    const QueryLayout L = query_layout(m);
    if (!workspace || !aligned(workspace, 256)) return LBVH_EINVAL;
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    hipError_t e = launch_query(qkind, tree->kind, tree->nodes, tree->leaf_perm, (int)tree->n, q, (int)m,
                                nullptr, indices, true,
                                static_cast<char *>(const_cast<void *>(workspace)), L,
                                (hipStream_t)stream);
    return hip_status(e);
}

int lbvh_query_spheres_count(const lbvh_tree *tree, const float *xyzr, int64_t m, int64_t *offsets,
                             void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_count(0, tree, xyzr, m, offsets, workspace, workspace_bytes, stream);
}

int lbvh_query_boxes_count(const lbvh_tree *tree, const float *lohi, int64_t m, int64_t *offsets,
                           void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_count(1, tree, lohi, m, offsets, workspace, workspace_bytes, stream);
}

int lbvh_query_spheres_fill(const lbvh_tree *tree, const float *xyzr, int64_t m, int32_t *indices,
                            const void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_fill(0, tree, xyzr, m, indices, workspace, workspace_bytes, stream);
}

int lbvh_query_boxes_fill(const lbvh_tree *tree, const float *lohi, int64_t m, int32_t *indices,
                          const void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_fill(1, tree, lohi, m, indices, workspace, workspace_bytes, stream);
}

int lbvh_query_rays_count(const lbvh_tree *tree, const float *rays, int64_t m, int64_t *offsets,
                          void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_count(2, tree, rays, m, offsets, workspace, workspace_bytes, stream);
}

int lbvh_query_rays_fill(const lbvh_tree *tree, const float *rays, int64_t m, int32_t *indices,
                         const void *workspace, int64_t workspace_bytes, void *stream)
{
    return query_fill(2, tree, rays, m, indices, workspace, workspace_bytes, stream);
}

int lbvh_query_rays_first(const lbvh_tree *tree, const float *rays, int64_t m, int32_t *hit,
                          float *t, void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!tree || m < 0 || m > INT32_MAX || tree->n < 0 || tree->n > LBVH_MAX_PRIMS) return LBVH_EINVAL;
    if (m == 0) return LBVH_OK;
    if (!rays || !aligned(rays, 16) || !hit || !t || !aligned(hit, 4) || !aligned(t, 4))
        return LBVH_EINVAL;
    if (tree->n > 0 && (!tree->nodes || !aligned(tree->nodes, 16))) return LBVH_EINVAL;
    const QueryLayout L = query_layout(m);
    if (!workspace || !aligned(workspace, 256)) return LBVH_EINVAL;
    if (workspace_bytes < (int64_t)L.total) return LBVH_ENOSPACE;
    hipError_t e;
    if (tree->n == 0) {
        // nothing to meet: hit -1, t = +inf, and a cleared error word
        e = launch_ray_none(m, hit, t, static_cast<char *>(workspace), L, (hipStream_t)stream);
    } else {
        e = launch_ray_first(tree->nodes, (int)tree->n, rays, (int)m, hit, t,
                             static_cast<char *>(workspace), L, (hipStream_t)stream);
    }
    return hip_status(e);
}

static int query_check(const void *workspace, size_t ctrl, void *stream)
{
    if (hipError_t e = hipStreamSynchronize((hipStream_t)stream); e != hipSuccess) return hip_status(e);
    uint32_t flag = 0;
    if (hipError_t e = hipMemcpy(&flag, static_cast<const char *>(workspace) + ctrl + kQueryErrorByte,
                                 sizeof(flag), hipMemcpyDeviceToHost);
        e != hipSuccess)
        return hip_status(e);
    return flag ? LBVH_EDEVICE : LBVH_OK;
}

int lbvh_query_check(const void *workspace, int64_t m, void *stream)
{
    if (!workspace || m < 0 || m > INT32_MAX) return LBVH_EINVAL;
    return query_check(workspace, query_layout(m).ctrl, stream);
}

int lbvh_query_batched_check(const void *workspace, int64_t m, void *stream)
{
    if (!workspace || m < 0 || m > INT32_MAX) return LBVH_EINVAL;
    return query_check(workspace, batch_query_layout(m).ctrl, stream);
}

const char *lbvh_last_hip_error(void) { return hipGetErrorString(t_last_hip); }

int64_t lbvh_tune(const char *name, int64_t value)
{
    if (!name) return LBVH_EINVAL;
    for (int k = 0; k < TUNE_NUM; ++k) {
        if (strcmp(name, kTuneNames[k]) == 0) {
            if (value < 0) return g_tune[k].load();
            if (value < kTuneMin[k] || value > kTuneMax[k]) return LBVH_EINVAL;
            if (k == TUNE_RADIX_BITS32 && !radix_bits_ok(30, (int)value)) return LBVH_EINVAL;
            if (k == TUNE_RADIX_BITS64 && !radix_bits_ok(63, (int)value)) return LBVH_EINVAL;
            return g_tune[k].exchange(value);
        }
    }
    return LBVH_EINVAL;
}

int lbvh_profile_enable(int32_t on)
{
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = on != 0;
    return LBVH_OK;
}

int lbvh_profile_reset(void)
{
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (int k = 0; k < K_NUM; ++k) {
        P.drain(k);
        P.ms[k] = 0.0;
        P.launches[k] = 0;
    }
    return LBVH_OK;
}

int lbvh_profile_read(const char *kernel, double *total_ms, int64_t *launches)
{
    if (!kernel) return LBVH_EINVAL;
    Profiler &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (int k = 0; k < K_NUM; ++k) {
        if (strcmp(kernel, kNames[k]) == 0) {
            P.drain(k);
            if (total_ms) *total_ms = P.ms[k];
            if (launches) *launches = P.launches[k];
            return LBVH_OK;
        }
    }
    return LBVH_EINVAL;
}

}  // extern "C"
