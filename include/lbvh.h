/*
 * lbvh.h - C ABI of the MI355X (gfx950) rope-LBVH library.
 *
 * Builds the linear bounding volume hierarchy of Prokopenko & Lebrun-Grandie,
 * "Revising Apetrei's bounding volume hierarchy construction algorithm to
 * allow stackless traversal" (arXiv 2402.00665), and answers range queries
 * with the stackless traversal that its skip-connections ("ropes") enable.
 *
 * Memory and ownership
 *   Every array argument is a DEVICE pointer owned by the caller, except the
 *   lbvh_tree descriptor itself, which is host memory.  The library never
 *   allocates device memory: scratch space comes in through a caller-owned
 *   workspace whose size the *_workspace_bytes functions return (that size
 *   is also the build's exact device-memory footprint beyond inputs and
 *   outputs).  All work is enqueued asynchronously on the given HIP stream
 *   (a hipStream_t passed as void*; NULL means the null stream).  Inputs must
 *   stay alive and unmodified, and outputs untouched, until the stream has
 *   passed the call.  Two calls that share a workspace must be ordered on
 *   one stream.
 *
 * Errors
 *   Functions return LBVH_OK (0) or a negative status; lbvh_strerror()
 *   names it.  Arguments are validated before anything is enqueued, so a
 *   call that returns LBVH_EINVAL or LBVH_ENOSPACE has no effect.
 *   LBVH_EHIP reports a failed kernel launch.  Faults inside kernels
 *   surface, as usual for HIP, at the next synchronising call.
 *
 * Node ids
 *   A tree over n >= 1 primitives has n-1 internal nodes and n leaves,
 *   stored in one array of 2n-1 lbvh_node records: internal node k (Karras
 *   order) is record k, leaf k (k-th primitive in Morton order) is record
 *   n-1+k, and -1 is the sentinel that ends a traversal.  Record 0 is the
 *   root (for n = 1 it is the single leaf).
 */
#ifndef LBVH_H
#define LBVH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ constants */

#define LBVH_OK 0
#define LBVH_EINVAL (-1)     /* bad argument: null pointer, size, code_bits */
#define LBVH_ENOSPACE (-2)   /* workspace smaller than *_workspace_bytes */
#define LBVH_EHIP (-3)       /* a HIP launch or runtime call failed */
#define LBVH_EDEVICE (-4)    /* a kernel flagged an internal error */
#define LBVH_ELIMIT (-5)     /* n above what lbvh_build_noalloc's fixed scratch holds */

#define LBVH_POINTS 0        /* primitives: float [n][3] = x, y, z */
#define LBVH_BOXES 1         /* primitives: float [n][6] = lo.xyz, hi.xyz */

#define LBVH_MAX_PRIMS ((int64_t)(1 << 30) - 1)

/* --------------------------------------------------------------- types */

/* One node of the hierarchy, 32 bytes, 16-byte aligned.
 *   lo, hi : the node's axis-aligned bounding box.  A leaf holds its
 *            primitive's box (a point p gives lo = hi = p); an internal node
 *            holds the componentwise min of its children's lo and max of
 *            their hi, exact in binary32.
 *   left   : internal node: id of its left child (Karras order: the children
 *            of a node split at gamma are gamma and gamma+1, Sec. 3.1);
 *            leaf: index of its primitive in the caller's input array.
 *   rope   : skip-connection (escape index, Sec. 2): where a traversal goes
 *            when this node's test fails or after a leaf; -1 = sentinel. */
typedef struct lbvh_node {
    float lo[3];
    int32_t left;
    float hi[3];
    int32_t rope;
} lbvh_node;

/* A built tree.  The caller allocates the arrays and sets the pointers;
 * the build fills n, code_bits and kind and writes the arrays.
 *   nodes     : device, 2n-1 records (nothing for n = 0).
 *   codes     : device, n Morton codes in ascending order (uint32 for 30-bit
 *               codes, uint64 for 63-bit); the build also uses it as sort
 *               scratch.  Queries do not read it.
 *   leaf_perm : device, int32 [n]: leaf k -> input index of its primitive
 *               (the same values as the leaves' `left` fields, contiguous). */
typedef struct lbvh_tree {
    int64_t n;
    int32_t code_bits;
    int32_t kind;
    lbvh_node *nodes;
    void *codes;
    int32_t *leaf_perm;
} lbvh_tree;

/* ---------------------------------------------------------------- build */

/* Workspace bytes that lbvh_build needs for n primitives of the given kind
 * (LBVH_POINTS / LBVH_BOXES) and code_bits (30 or 63).  Returns a negative
 * status for invalid arguments. */
int64_t lbvh_build_workspace_bytes(int64_t n, int32_t code_bits, int32_t kind);

/* Build the rope-LBVH of n primitives.
 *   Steps (Sec. 3.1 and Alg. 4): scene box (min/max of all primitive
 *   boxes); Morton code of each centroid (b = code_bits/3 bits per axis,
 *   x in the most significant bit of each 3-bit group); stable radix sort of
 *   (code, input index); one bottom-up pass that merges ranges with a
 *   compare-and-swap per internal node, names each parent by its Karras
 *   index, and writes its left child, rope and box.
 *   prims      : device, float [n][3] (points) or [n][6] (boxes), finite,
 *                lo <= hi per axis for boxes.  Non-finite coordinates are
 *                not rejected: the tree is still well formed (leaf_perm a
 *                permutation, every child and rope a valid node id, no
 *                access outside the arrays), but its boxes, and the
 *                answers of queries against it, are unspecified.
 *   n          : 0 <= n <= LBVH_MAX_PRIMS.  n = 0 gives an empty tree.
 *   code_bits  : 30 (uint32 codes) or 63 (uint64 codes).
 *   tree       : host descriptor with nodes, codes and leaf_perm set
 *                (non-NULL if n > 0).
 *   workspace  : device, at least lbvh_build_workspace_bytes(...) bytes,
 *                256-byte aligned; contents on entry are ignored.
 * Equal Morton codes are ordered by input index and the keys are made
 * distinct by the sorted position, so the tree is unique. */
int lbvh_build(int32_t kind, const float *prims, int64_t n, int32_t code_bits,
               lbvh_tree *tree, void *workspace, int64_t workspace_bytes,
               void *stream);

/* lbvh_build with kind = LBVH_POINTS; xyz is float [n][3]. */
int lbvh_build_points(const float *xyz, int64_t n, int32_t code_bits,
                      lbvh_tree *tree, void *workspace, int64_t workspace_bytes,
                      void *stream);

/* lbvh_build with kind = LBVH_BOXES; lohi is float [n][6]. */
int lbvh_build_boxes(const float *lohi, int64_t n, int32_t code_bits,
                     lbvh_tree *tree, void *workspace, int64_t workspace_bytes,
                     void *stream);

/* Synchronise the stream and report an internal error that a build's
 * kernels flagged in the workspace (LBVH_EDEVICE), else LBVH_OK.  For tests
 * and debugging; the build itself never synchronises. */
int lbvh_build_check(const void *workspace, int64_t n, int32_t code_bits,
                     int32_t kind, void *stream);

/* lbvh_build for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops or harnesses that forbid hipMalloc):
 * the same build, with no workspace argument.  Its scratch is a fixed
 * array of LBVH_NOALLOC_SCRATCH_BYTES bytes in device memory, one per GPU,
 * which each GPU the library runs on holds until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the caller still allocates the tree's arrays.
 *   n         : 0 <= n <= LBVH_NOALLOC_MAX_PRIMS; a larger n returns
 *               LBVH_ELIMIT and enqueues nothing.
 *   error_out : NULL, or caller-owned device or pinned host memory (4-byte
 *               aligned) that receives the build's error word once the
 *               stream has passed the call: nonzero means what
 *               lbvh_build_check reports as LBVH_EDEVICE.  Nothing is
 *               written for n = 0.
 * Other arguments, results and errors as lbvh_build.  The current device
 * (hipSetDevice) must be the stream's.  Every call on one GPU shares that
 * GPU's scratch, and each call overwrites it: calls that overlap on one GPU
 * (different streams or host threads) race, so the caller orders them. */
#define LBVH_NOALLOC_MAX_PRIMS ((int64_t)1 << 20)
#define LBVH_NOALLOC_SCRATCH_BYTES ((int64_t)25 << 20)
int lbvh_build_noalloc(int32_t kind, const float *prims, int64_t n, int32_t code_bits,
                       lbvh_tree *tree, uint32_t *error_out, void *stream);


/* ------------------------------------------------------------- queries */

/* Workspace bytes for the count and fill calls over m queries. */
int64_t lbvh_query_workspace_bytes(int64_t m);

/* Range queries, first of two calls: Alg. 1 per query, counting hits.
 * The tree descriptor is the one its build filled in (its kind included:
 * for LBVH_POINTS every leaf box has hi == lo, so the leaf test reads only
 * the lower corner of each leaf record).
 * Sphere j is xyzr[j] = (x, y, z, r), r >= 0: a node or primitive box B
 * matches if d = per-axis max(B.lo - c, c - B.hi, 0) gives
 * (dx*dx + dy*dy) + dz*dz <= r*r in binary32 (closed ball, no fused
 * multiply-add).  Box j is lohi[j] = (lo.xyz, hi.xyz): B matches if
 * lo <= B.hi and B.lo <= hi on every axis (closed boxes).
 * Each query's walk is run as independent pieces over aligned blocks of
 * leaves (same nodes, same order); the pieces, a hit mask per piece and
 * the hit offsets are kept in the workspace for the fill call, which tests
 * no box again for pieces of at most 256 leaves.  With the "query_order"
 * knob the walks run in a Morton order of the queries; the workspace then
 * also keeps the reordered queries and each one's shift to its output
 * slot.
 *   xyzr / lohi : device, float [m][4] / [m][6], 16-byte aligned.
 *   offsets     : device int64 [m+1]; receives the CSR offsets,
 *                 offsets[0] = 0 and offsets[m] = total number of hits.
 *   workspace   : device, at least lbvh_query_workspace_bytes(m) bytes,
 *                 256-byte aligned.
 * The caller reads offsets[m] (the one device-to-host copy), allocates the
 * index array and calls the matching *_fill with the same workspace. */
int lbvh_query_spheres_count(const lbvh_tree *tree, const float *xyzr, int64_t m,
                             int64_t *offsets, void *workspace,
                             int64_t workspace_bytes, void *stream);
int lbvh_query_boxes_count(const lbvh_tree *tree, const float *lohi, int64_t m,
                           int64_t *offsets, void *workspace,
                           int64_t workspace_bytes, void *stream);

/* Second call: write, for query j, the input indices of the matching
 * primitives into indices[offsets[j] .. offsets[j+1]) in traversal order
 * (ascending Morton-order position): the hits Alg. 1 reports, stored as
 * its "store the result" step leaves open (Sec. 2).  A fill never writes
 * more than the count call counted for a query, whatever the knobs.
 *   indices   : device int32 [offsets[m]] (non-NULL even when empty).
 *   workspace : the workspace of the preceding count call on the same tree
 *               and queries, untouched since (enqueue both on one stream or
 *               order the streams). */
int lbvh_query_spheres_fill(const lbvh_tree *tree, const float *xyzr, int64_t m,
                            int32_t *indices, const void *workspace,
                            int64_t workspace_bytes, void *stream);
int lbvh_query_boxes_fill(const lbvh_tree *tree, const float *lohi, int64_t m,
                          int32_t *indices, const void *workspace,
                          int64_t workspace_bytes, void *stream);

/* Rays and segments (Sec. 1 lists the primitives a ray meets among the
 * range searches a hierarchy answers; Alg. 1 walks them like any other
 * query).  Ray j is rays[j] = (o.x, o.y, o.z, tmin, d.x, d.y, d.z, tmax):
 * the points o + t*d with tmin <= t <= tmax.  A segment from a to b is
 * o = a, d = b - a, [0, 1]; a ray has tmax = +inf.  Closed slab test in
 * binary32, no fused multiply-add: per axis inv = 1/d (correctly rounded);
 * an axis with d = 0, or whose inv overflows, passes iff lo <= o <= hi;
 * otherwise t1 = (lo - o)*inv and t2 = (hi - o)*inv.  The entry parameter
 * is the largest of tmin and the per-axis min(t1, t2), the exit the
 * smallest of tmax and the per-axis max(t1, t2); a box B matches iff every
 * parallel axis passes and entry <= exit.
 *   rays : device, float [m][8], 16-byte aligned.
 * All hits: the count and fill calls behave as the sphere and box calls
 * (same workspace, CSR offsets, hits in ascending Morton-order position). */
int lbvh_query_rays_count(const lbvh_tree *tree, const float *rays, int64_t m,
                          int64_t *offsets, void *workspace,
                          int64_t workspace_bytes, void *stream);
int lbvh_query_rays_fill(const lbvh_tree *tree, const float *rays, int64_t m,
                         int32_t *indices, const void *workspace,
                         int64_t workspace_bytes, void *stream);

/* First hit of each ray: among the primitives it matches, the one with the
 * smallest entry parameter, ties to the smallest Morton-order position.
 * One pruned Alg. 1 walk per ray: a node is entered only if the ray meets
 * its box with an entry parameter below the best hit so far (a box inside
 * another never has a smaller entry parameter, so nothing is lost).
 *   hit       : device int32 [m]: input index of the primitive, -1 if none.
 *   t         : device float [m]: its entry parameter, +inf if none.
 *   workspace : device, at least lbvh_query_workspace_bytes(m) bytes,
 *               256-byte aligned; only its error word is used, and
 *               lbvh_query_check reads it as after a count call.
 * m = 0 enqueues nothing. */
int lbvh_query_rays_first(const lbvh_tree *tree, const float *rays, int64_t m,
                          int32_t *hit, float *t, void *workspace,
                          int64_t workspace_bytes, void *stream);

/* Synchronise the stream and report an error that the last count call over
 * m queries flagged in `workspace` (LBVH_EDEVICE), else LBVH_OK.  Flagged:
 * a walk that spent its node-visit budget before the sentinel (never for a
 * tree this library built, unless the "query_walk_budget" knob caps it), or
 * a failed query-order sort.  The offsets and indices of such a call are
 * then not Alg. 1's.  Each count call clears the word first.  For tests and
 * debugging; the count call itself never synchronises. */
int lbvh_query_check(const void *workspace, int64_t m, void *stream);

/* ------------------------------------------------------------- batched */

/* Many independent scenes built together.  Scene s owns primitives
 * [seg_off[s], seg_off[s+1]) of the concatenated input; its tree is exactly
 * the tree lbvh_build gives for those primitives alone (own scene box,
 * Morton codes, sort, node ids, primitive ids local to the scene), stored at
 * record 2*seg_off[s] of `nodes` (2n_s-1 records; n_s = 0 gives none).
 * The caller allocates every array and fills the descriptor except kind.
 *   seg_off   : device int64 [num_scenes+1], seg_off[0] = 0, non-decreasing,
 *               seg_off[num_scenes] = total_n.
 *   max_scene : an upper bound of every scene's size (host value).  It sets
 *               how many bottom-up levels run: the least L >= 0 with
 *               256 * 256^L >= max_scene, which covers scenes of up to
 *               256 * 256^L primitives.  A scene beyond that cover is
 *               reported by the check call (LBVH_EDEVICE) and its tree is
 *               not valid; a scene above max_scene but within the cover is
 *               built exactly.
 *   nodes     : device, 2*total_n records.
 *   codes     : device, total_n codes, ascending within each scene.
 *   leaf_perm : device int32 [total_n]: leaf k of scene s (entry
 *               seg_off[s]+k) -> index of its primitive within the scene. */
typedef struct lbvh_batch {
    int32_t num_scenes;
    int32_t code_bits;
    int32_t kind;
    int32_t reserved;
    int64_t total_n;
    int64_t max_scene;
    const int64_t *seg_off;
    lbvh_node *nodes;
    void *codes;
    int32_t *leaf_perm;
} lbvh_batch;

/* Workspace bytes for lbvh_build_batched. */
int64_t lbvh_build_batched_workspace_bytes(int64_t total_n, int32_t num_scenes,
                                           int64_t max_scene, int32_t code_bits,
                                           int32_t kind);

/* Build every scene's rope-LBVH (the steps of lbvh_build, Sec. 3.1 and
 * Alg. 4) with one launch sequence for all scenes: per-scene boxes and
 * codes (one block per scene), segmented radix passes (tiles never cross
 * scenes), and the bottom-up pass with blocks that never cross scenes.
 * Only kernel launches are enqueued (no memsets, no host synchronisation),
 * so the call can be captured in a HIP graph and replayed.
 *   prims     : device, float [total_n][3] or [total_n][6], 8-byte aligned.
 *   workspace : device, lbvh_build_batched_workspace_bytes(...) bytes,
 *               256-byte aligned. */
int lbvh_build_batched(int32_t kind, const float *prims, lbvh_batch *batch,
                       void *workspace, int64_t workspace_bytes, void *stream);

/* Synchronise and report an error flagged by a batched build's kernels
 * (LBVH_EDEVICE), e.g. a scene larger than max_scene. */
int lbvh_build_batched_check(const void *workspace, const lbvh_batch *batch,
                             void *stream);

/* Asynchronous form of lbvh_build_batched_check, for callers that must not
 * block (a request loop): enqueues on `stream` a 4-byte copy of the batched
 * build's error word from `workspace` to `flag_out` (pinned host or device
 * memory, caller-owned, 4-byte aligned).  Once the stream has passed that
 * copy, a nonzero *flag_out means the build failed as lbvh_build_batched_check
 * would report it (LBVH_EDEVICE).  A batch with no primitives builds nothing:
 * then nothing is enqueued and *flag_out is left as it was, so callers zero
 * it first.  Returns LBVH_EINVAL for null or invalid arguments, LBVH_EHIP if
 * the copy cannot be enqueued. */
int lbvh_build_batched_status_async(const void *workspace, const lbvh_batch *batch,
                                    uint32_t *flag_out, void *stream);

/* Workspace bytes for a batched count call over m queries. */
int64_t lbvh_query_batched_workspace_bytes(int64_t m);

/* lbvh_query_check for the batched count call's workspace (m queries). */
int lbvh_query_batched_check(const void *workspace, int64_t m, void *stream);

/* Range queries on a batch: query j belongs to the scene s with
 * qseg_off[s] <= j < qseg_off[s+1] (device int64 [num_scenes+1]) and walks
 * that scene's tree (Alg. 1; same predicates and order as the single-tree
 * calls).  Indices are primitive ids local to the scene.  The count call
 * writes CSR offsets [m+1] and keeps each query's first hits in the
 * workspace; the fill call, given the same workspace (unchanged since the
 * count call of the same queries), copies those for queries with few hits
 * and repeats the walk for the others, writing the ids at the offsets. */
int lbvh_query_batched_spheres_count(const lbvh_batch *batch, const float *xyzr,
                                     const int64_t *qseg_off, int64_t m,
                                     int64_t *offsets, void *workspace,
                                     int64_t workspace_bytes, void *stream);
int lbvh_query_batched_boxes_count(const lbvh_batch *batch, const float *lohi,
                                   const int64_t *qseg_off, int64_t m,
                                   int64_t *offsets, void *workspace,
                                   int64_t workspace_bytes, void *stream);
int lbvh_query_batched_spheres_fill(const lbvh_batch *batch, const float *xyzr,
                                    const int64_t *qseg_off, int64_t m,
                                    const int64_t *offsets, int32_t *indices,
                                    const void *workspace, int64_t workspace_bytes,
                                    void *stream);
int lbvh_query_batched_boxes_fill(const lbvh_batch *batch, const float *lohi,
                                  const int64_t *qseg_off, int64_t m,
                                  const int64_t *offsets, int32_t *indices,
                                  const void *workspace, int64_t workspace_bytes,
                                  void *stream);

/* ------------------------------------------------------------ utilities */

/* Human-readable name of a status code (static string). */
const char *lbvh_strerror(int status);

/* The HIP runtime's description of the error behind the last LBVH_EHIP
 * returned on the calling thread ("no error" if none). */
const char *lbvh_last_hip_error(void);

/* Launch-shape tuning, process-wide (for autotuners and benchmarks).
 * Sets knob `name` to `value` and returns the previous value; a negative
 * `value` only reads the knob.  Returns LBVH_EINVAL for an unknown name or
 * a value out of range.  Knobs:
 *   "radix_bits32", "radix_bits64": digit width of the radix sort (single
 *       and batched builds) for 30-bit / 63-bit codes: 8 or 10 bits
 *       (4 or 3 passes; default 8) and 8, 9 or 11 bits (8, 7 or 6 passes;
 *       default 9).  Other values are refused.
 *   "sort_variant32", "sort_variant64": tile shape of the radix passes for
 *       30-bit / 63-bit codes: 0 = 256 threads x 16 keys, 1 = 256 x 8,
 *       2 = 256 x 24, 3 = 512 x 8, 4 = 512 x 16, 5 = 1024 x 8, 6 = 768 x 16,
 *       7 = 1024 x 16, 8 = 512 x 24 (defaults 4 and 6).  A shape whose tile
 *       holds fewer keys than the digit width needs (4096 for 11-bit digits) or whose tables do not
 *       fit the LDS runs as 512 x 16 (30-bit) or 512 x 8 (63-bit).
 *   "batch_sort_variant": tile shape of the batched build's segmented
 *       radix passes: 0 = 256 x 16 (default), 1 = 256 x 8, 2 = 512 x 8,
 *       3 = 512 x 16 (1 runs as 0 with 11-bit digits).
 *   "batch_sort_mode": how the batched build sorts: 0 = segmented radix
 *       passes over all scenes (default), 1 = one block per scene, which
 *       computes the scene's box and codes and runs every pass over the
 *       scene itself (no look-back between blocks); in this mode
 *       "batch_sort_variant" picks the block: 0 = 256 x 16, 1 = 512 x 8,
 *       2 = 1024 x 8, 3 = 512 x 16 (a block whose tables do not fit the LDS
 *       runs as 256 x 16).  Mode 1 applies to batches whose largest scene
 *       has at most 262144 primitives; larger batches run mode 0.
 *   "query_split1", "query_split2": the single-tree count call cuts each
 *       query's Alg. 1 walk into pieces at aligned blocks of 2^split1
 *       leaves, then cuts those at blocks of 2^split2 leaves, and walks the
 *       pieces in parallel; values 2 .. 24 (defaults 12 and 7).  The fill
 *       call reuses the count call's pieces.
 *   "query_leaf_mode": how the single-tree count and fill calls handle the
 *       finest pieces: 0 = one wave tests a piece's leaves 64 at a time
 *       (default; best when queries hit many leaves), 1 = pieces whose
 *       start-node box lies mostly outside the query are walked with Alg. 1
 *       by one lane, the rest as in 0 (best for sparse queries).  Both
 *       record the same per-piece hit masks, and the fill call reads those
 *       whatever the knobs are when it is enqueued.
 *   "query_order": 1 = the single-tree count call first sorts the queries
 *       by a 16-bit Morton key of their centres (in the root's box) and
 *       walks them in that order, so that neighbouring threads walk
 *       neighbouring parts of the tree; offsets and indices still come out
 *       in the caller's query order.  0 = the caller's order (default).
 *       The count call records which it did in the workspace, and the fill
 *       call follows that whatever the knob is when it is enqueued.
 *   "query_walk_budget": for tests of the error path: caps the node visits
 *       of each walk of a count call (0 = no cap beyond 2n, the default).
 *       A walk that hits the cap stops; lbvh_query_check then reports it.
 *   "morton_order": 1 = the single-tree build's Morton-code kernel sweeps
 *       the primitives from the end of the array to its start, the
 *       opposite of the scene-box pass before it, so its first reads find
 *       that pass's last lines in the last-level cache (default); 0 = from
 *       the start.
 *   "radix_mode": how the single-tree build runs each radix pass: 0 = one
 *       onesweep kernel whose tiles find their output positions by a
 *       decoupled look-back over the earlier tiles (default); 1 = a count
 *       kernel over chunks of 8 tiles (the look-back runs over the
 *       chunks' totals) and then the scatter kernel, which reads each
 *       tile's positions and waits for no other tile.
 * Results never depend on the knobs other than query_walk_budget; only
 * speed does.  Calls already enqueued keep the shapes they were enqueued
 * with. */
int64_t lbvh_tune(const char *name, int64_t value);

/* Per-kernel timing.  While enabled, every launch the library makes is
 * bracketed by HIP events recorded on the launch's own stream.
 * lbvh_profile_read synchronises those events and returns, for the kernel
 * named `kernel`, the summed duration in milliseconds and the number of
 * launches since the last reset.  Names: "bounds", "bounds_final",
 * "morton", "sort_pass", "bottomup" (level 0 of the bottom-up pass),
 * "bottomup_up" (its upper levels), "batch_prep" (batched plan and
 * per-scene codes), "query_order" (the query sort and the mapping back to
 * the caller's order), "query_split",
 * "query_count", "query_fill", "scan" (scans and offset bookkeeping).
 * Returns LBVH_EINVAL for an unknown name. */
int lbvh_profile_enable(int32_t on);
int lbvh_profile_reset(void);
int lbvh_profile_read(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* LBVH_H */
