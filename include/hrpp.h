/*
 * hrpp.h -- C ABI of the MI355X (gfx950) Hash-Based Ray Path Prediction library.
 *
 * Method: Demoullin, Gubran and Aamodt, "Hash-Based Ray Path Prediction:
 * Skipping BVH Traversal Computation by Exploiting Ray Locality".  Before a
 * ray enters the BVH its origin and direction are hashed into a predictor
 * table that maps the hash to leaf nodes reached by earlier similar rays
 * (section "Overview").  The predicted leaves are tested first; if that
 * yields a valid intersection the interior traversal is skipped, otherwise
 * the ray traverses normally (section "Precision and Recall").  A traversed
 * ray inserts its leaf into its entry unless already present (section "HRPP
 * Hash Function").  Hit-any and hit-all rays use separate predictors
 * (section "Limit Study").
 *
 * Conventions for every entry point:
 *  - Pointers prefixed d_ are device (HBM) pointers, h_ host pointers.
 *  - The caller owns all device memory: rays, results, stats, and the
 *    backing stores of BVHs and predictors, sized by *_required_bytes.
 *    The library owns only the opaque handle structs (host heap).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued and the call returns; nothing synchronises unless stated.
 *  - Arguments are validated on the host before anything is enqueued; an
 *    invalid argument returns HRPP_EINVAL and enqueues nothing.
 *  - Handles are not thread-safe.  Calls that use one predictor must be
 *    issued on one stream or ordered by the caller.
 *  - Floating point: binary32, round to nearest even, no contraction, no
 *    flush-to-zero, correctly rounded division.
 */
#ifndef HRPP_H
#define HRPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRPP_OK = 0,
    HRPP_EINVAL = 1,   /* bad argument or descriptor */
    HRPP_ENOMEM = 2,   /* caller buffer too small, or host allocation failed */
    HRPP_EDEVICE = 3,  /* a HIP runtime call failed */
    HRPP_EDEPTH = 4,   /* the BVH would exceed max_depth */
    HRPP_EBUSY = 5     /* serving queue full / budget exhausted */
} hrpp_status;

/* A ray: origin, interval start, direction (need not be unit), interval end.
 * 32 bytes, 16-byte aligned arrays.  Hits are accepted for tmin < t < tmax.
 * A ray is invalid (reported as a miss, counted in `invalid`, never hashed
 * or traversed) if o or d has a non-finite component, d is the zero
 * vector, a bound is NaN, or !(tmin < tmax).  tmax may be +inf. */
typedef struct { float ox, oy, oz, tmin, dx, dy, dz, tmax; } hrpp_ray;

/* Closest-hit result: distance, barycentrics of v1 and v2, original
 * primitive index.  A miss is t = +inf, u = v = 0, prim = 0xFFFFFFFF. */
typedef struct { float t, u, v; uint32_t prim; } hrpp_hit;

/* BVH build parameters (the paper takes the binary BVH as given; this
 * library builds a deterministic binned-SAH tree).  leaf_max in [1, 8]
 * (4 by default), sah_bins in [2, 256] (32), max_depth in [1, 64] (64).
 * treelet_passes in [0, 8] (0): passes of treelet restructuring applied
 * to the built tree (the host SAH tree or the device linear BVH; see
 * hrpp_build_bvh_device): interior nodes rearranged to lower the sum of
 * their surface areas, leaves unchanged. */
typedef struct { uint32_t leaf_max, sah_bins, max_depth, treelet_passes; } hrpp_bvh_desc;

/* Predictor parameters.
 *  log2_entries  T: table of 2^T entries, T in [1, 26]
 *  ways          W: leaf slots per entry, 1..8 (entry = 32 B for W <= 4, 64 B otherwise)
 *  origin_bits   q_o: origin cells per axis = 2^q_o over the scene bounds, 1..10
 *  dir_bits      q_d: octahedral direction bins per axis = 2^q_d, 1..10
 *  epoch_rays    E: rays per epoch; rays of epoch k see the table as it stood
 *                after epoch k-1 (batch-synchronous update), 1..2^22
 *  hash_mode     0 = grid origin cells (q_o bits per axis over the scene bounds)
 *                    + octahedral direction bins (q_d bits per axis);
 *                1 = the bit-field hash of section "HRPP Hash Function": per
 *                    binary32 value of origin and direction the sign, the p
 *                    leading exponent and p leading mantissa bits, fields
 *                    o.x^d.z, o.y^d.y, o.z^d.x packed at a stride of 8 bits
 *                    (p <= 3) or 16 bits (p >= 4); p = origin_bits in 1..7
 *                    and dir_bits must equal origin_bits.  The scene bounds
 *                    play no part in this mode.
 *                Both modes fold the key into the index with
 *                (key * 0x9E3779B97F4A7C15) >> (64 - T) and store it as the tag.
 *  go_up_level   g in [0, 64] (section "Go Up Level"): 0 predicts leaves;
 *                g >= 1 predicts the node g levels above the leaf a ray
 *                reached (the root if the leaf is shallower), and a
 *                positive ray walks that node's subtree with the ordinary
 *                traversal rules after testing its box
 *  inline_lanes  scheduling only (results do not depend on it): a 64-lane
 *                wave of the prediction kernel in which at least this many
 *                rays must still traverse traverses them at once; other
 *                waves append theirs to the epoch's compacted fallback
 *                queue.  1..64; 65 = always queue; 0 = the default (48).
 *  replace_policy  0 = no eviction (the paper has no replacement policy,
 *                section "Precision and Recall": ids that do not fit a full
 *                entry are dropped; a new owner key replaces the tag);
 *                bit 0 = FIFO within an entry: the oldest slots make room for
 *                up to `ways` new ids; bit 1 = the resident tag keeps its
 *                entry: records of another key are conflicts and only empty
 *                entries are claimed.  0..3.
 *  first_epoch_rays  length of each call's first epoch (0 = epoch_rays,
 *                otherwise 1..epoch_rays); the other epochs keep epoch_rays.
 *                A short first epoch fills the table early: when the rays
 *                are ordered so that it samples the whole view, the rest of
 *                the call sees a table that covers it. */
typedef struct {
    uint32_t log2_entries, ways, origin_bits, dir_bits, epoch_rays, hash_mode, go_up_level, inline_lanes,
             replace_policy, first_epoch_rays;
} hrpp_predictor_desc;

/* Work counters, accumulated (added to) by every trace call that is given
 * a stats pointer.  Definitions (section "Precision and Recall" names the
 * outcomes; the counting rules are this library's):
 *  rays, invalid, hits          rays seen / invalid / with a hit
 *  lookups, positives           table probes / probes whose entry holds the key
 *  pred_hits, false_pos         positives that did / did not succeed in the
 *                               predicted leaves or subtrees (EXACT: final hit
 *                               in one of them or not)
 *  traversals                   full stack traversals run (subtree walks of
 *                               predicted nodes are not counted here)
 *  nodes_visited                interior + leaf visits (predicted ones included)
 *  interior_visited, leaf_visited, box_tests, tri_tests
 *  nodes_skipped                sum over prediction successes of the
 *                               interior-ancestor count of the predicted leaf
 *                               or node that produced the result
 *  records                      update records emitted (traversed rays with a hit)
 *  tag_claims, leaf_inserts     entries (re)claimed / ids written
 *  dropped                      owner-key records whose id is not in the final entry
 *  conflicts                    records discarded because another key owns the entry
 *  pred_leaf_visited, pred_tri_tests, pred_box_tests
 *                               the part of leaf_visited / tri_tests / box_tests
 *                               spent on predictions (a predicted leaf's or
 *                               node's box is tested first; its triangles or
 *                               subtree only if it is hit)
 *  evictions                    ids evicted by FIFO replacement
 *  queue_traversals, queue_interior_visited, queue_tri_tests, queue_records
 *                               schedule counters, not part of the method: the
 *                               part of traversals / interior_visited /
 *                               tri_tests / records done by the fallback-queue
 *                               kernel (the rest of the fallback work runs
 *                               inside the prediction kernel; the split
 *                               follows inline_lanes)
 *  empty_lookups                schedule counter: lookups answered without
 *                               reading the table, in the first epoch after a
 *                               reset (the table is known to be empty)
 *  empty_rays, empty_interior_visited, empty_tri_tests, empty_records
 *                               schedule counters: the part of rays /
 *                               interior_visited / tri_tests / records in
 *                               that first epoch (its own kernel) */
#define HRPP_STATS_SLOTS 32
typedef struct {
    uint64_t rays, invalid, hits, lookups, positives, pred_hits, false_pos, traversals,
             nodes_visited, interior_visited, leaf_visited, box_tests, tri_tests, nodes_skipped,
             records, tag_claims, leaf_inserts, dropped, conflicts, pred_leaf_visited, pred_tri_tests,
             pred_box_tests, evictions, queue_traversals, queue_interior_visited, queue_tri_tests,
             queue_records, empty_lookups, empty_rays, empty_interior_visited, empty_tri_tests,
             empty_records;
} hrpp_stats;

enum { HRPP_CLOSEST_PAPER = 0, HRPP_CLOSEST_EXACT = 1 };

typedef struct hrpp_bvh hrpp_bvh;
typedef struct hrpp_predictor hrpp_predictor;

/* Canonical (device-independent) form of a built BVH: nodes in depth-first
 * pre-order, left child = next node.  Arrays are caller-owned host buffers
 * of num_nodes entries (box: 6 floats per node, min xyz then max xyz) and
 * num_tris entries (tri_perm: BVH position -> original primitive id). */
typedef struct {
    float *box;
    uint32_t *right;      /* right child id; 0xFFFFFFFF for a leaf */
    uint32_t *first_tri;  /* leaf: first BVH-ordered triangle; interior: 0 */
    uint32_t *count;      /* leaf: triangle count; interior: 0 */
    uint32_t *depth;      /* interior ancestors */
    uint32_t *tri_perm;
} hrpp_bvh_canon;

/* Upper bound of the device bytes a BVH over num_tris triangles needs. */
size_t hrpp_bvh_required_bytes(uint32_t num_tris, const hrpp_bvh_desc *desc);

/* Build a BVH on the host from h_verts (9 floats per triangle: v0 v1 v2,
 * original order = primitive id) and upload its GPU layout into d_buf
 * (bytes >= hrpp_bvh_required_bytes, 256-byte aligned) on `stream`.
 * h_verts may be freed when the call returns.  Errors: EINVAL (null
 * pointers, num_tris == 0 or >= 2^28, non-finite vertex, bad desc),
 * ENOMEM (bytes too small), EDEPTH (tree deeper than max_depth), EDEVICE. */
hrpp_status hrpp_build_bvh(const float *h_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                           void *d_buf, size_t bytes, void *stream, hrpp_bvh **out);

/* The two halves of hrpp_build_bvh, for callers that build on a host
 * thread and upload later: build the tree only (host memory, no HIP call;
 * the handle can be exported but not traced until uploaded) ... */
hrpp_status hrpp_bvh_build_host(const float *h_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                hrpp_bvh **out);

/* ... exact device bytes of its GPU layout ... */
size_t hrpp_bvh_device_bytes(const hrpp_bvh *bvh);

/* ... and write the GPU layout into d_buf (256-byte aligned, bytes >=
 * hrpp_bvh_device_bytes).  Synchronises `stream`.  Uploading again to
 * another buffer moves the BVH there (predictors stay bound to it). */
hrpp_status hrpp_bvh_upload(hrpp_bvh *bvh, void *d_buf, size_t bytes, void *stream);

/* Device build (a GPU builder for callers that take new scenes while they
 * run, such as the serving loop; the paper takes the BVH as given,
 * "Overview").  Builds a linear BVH entirely on the GPU: the binary radix
 * tree over 63-bit Morton codes of the triangle centres on a grid of cubic
 * cells (Karras, HPG 2012),
 * triangles ordered by (code, primitive id), every subtree over at most
 * leaf_max triangles kept as one leaf, exact boxes, DFS pre-order -- a
 * different tree from the host builder's SAH tree, with the same query
 * results.  With desc->treelet_passes >= 1 the interior nodes are then
 * rearranged by that many passes of treelet restructuring (Karras and Aila,
 * HPG 2013): in each pass every interior node, after all interior nodes
 * below it, gathers a treelet of up to 7 subtrees (repeatedly opening the
 * interior one of largest surface area) and takes the topology over them
 * that minimises the sum of its interior nodes' surface areas, when that
 * sum is below the current one; the leaves stay as they are.
 *
 * Scratch bytes the build needs for num_tris triangles, about 157 per
 * triangle (0 when num_tris is 0 or >= 2^28). */
size_t hrpp_bvh_device_build_scratch_bytes(uint32_t num_tris);

/* d_verts: device array of 9 floats per triangle (original order =
 * primitive id), 4-byte aligned, read only.  d_scratch (>= the bytes above)
 * and d_buf (>= hrpp_bvh_required_bytes) are caller-owned, 256-byte aligned;
 * the scratch is free again when the call returns, d_buf holds the BVH.
 * desc->sah_bins is ignored.  Enqueues the build on `stream` and
 * synchronises it.  Errors: EINVAL (null pointers, misalignment, num_tris
 * == 0 or >= 2^28, bad desc, a non-finite vertex), ENOMEM (a buffer too
 * small), EDEPTH (a leaf deeper than desc->max_depth), EDEVICE.  The handle
 * can be traced, used by predictors, batches and the server, and exported
 * (hrpp_bvh_export then copies the tree back); it has no 4-wide tree
 * (hrpp_trace_wide_* return EINVAL) and cannot be uploaded again. */
hrpp_status hrpp_build_bvh_device(const float *d_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                  void *d_scratch, size_t scratch_bytes, void *d_buf, size_t bytes, void *stream,
                                  hrpp_bvh **out);

/* The device build for callers that cannot allocate device memory (code
 * under hipGraph capture, serving loops that take new scenes, harnesses that
 * forbid hipMalloc): as hrpp_build_bvh_device, but the build scratch is a
 * static device array of 64 MiB inside the library (one per GPU, held until
 * the process ends) instead of a caller buffer.  The call allocates nothing:
 * no hipMalloc, no hipFree, no allocating library routine.  The caller still
 * passes the vertices and d_buf (>= hrpp_bvh_required_bytes, 256-byte
 * aligned), which holds the BVH.  The scratch is free again when the call
 * returns, so handles built by earlier calls stay valid; but every call on
 * one GPU uses that GPU's one array, so calls that overlap on one GPU (from
 * several host threads) race and must be serialised by the caller.  Errors
 * as hrpp_build_bvh_device, plus ENOMEM when the build needs more than the
 * static 64 MiB (hrpp_bvh_device_build_scratch_bytes(num_tris) > 64 MiB:
 * from about 427,000 triangles on; then nothing is enqueued). */
hrpp_status hrpp_build_bvh_device_static(const float *d_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                         void *d_buf, size_t bytes, void *stream, hrpp_bvh **out);

/* Node count, triangle count and maximum leaf depth of a built BVH. */
hrpp_status hrpp_bvh_info(const hrpp_bvh *bvh, uint32_t *num_nodes, uint32_t *num_tris,
                          uint32_t *max_depth);

/* Copy the canonical form of the tree into caller-owned host arrays
 * (sized from hrpp_bvh_info).  Synchronous: host only for a host-built
 * tree; a device-built tree is copied back from device memory. */
hrpp_status hrpp_bvh_export(const hrpp_bvh *bvh, hrpp_bvh_canon *h_out);

/* Release the handle (the caller's device buffer is not touched). */
void hrpp_bvh_destroy(hrpp_bvh *bvh);

/* Device bytes a predictor needs: the table (2^T entries of 32/64 B), one
 * reset mark per 16 entries and per-epoch scratch (fallback queue, update
 * records, fresh-id lists). */
size_t hrpp_predictor_required_bytes(const hrpp_predictor_desc *desc);

/* Bytes of the table alone (what hrpp_predictor_export copies). */
size_t hrpp_predictor_table_bytes(const hrpp_predictor_desc *desc);

/* Create a predictor bound to `bvh` (its hash grid spans the BVH's root
 * box) in d_buf (256-byte aligned), and enqueue its reset on `stream`.
 * The predictor is the table of section "Overview" that maps a ray's hash
 * to the leaf nodes earlier rays of that hash reached; its entries are
 * filled as section "HRPP Hash Function" describes (a traversed ray's leaf
 * joins its entry unless already there), here with the finite table, slot
 * count and batch-synchronous epochs set by desc.  Section "Limit Study"
 * keeps one such table per query type: create one for any-hit and one for
 * closest-hit rays.
 * Errors: EINVAL (bad desc, hash_mode above 1 or a mode-1 precision out of
 * range, go_up_level above 64),
 * ENOMEM (bytes too small). */
hrpp_status hrpp_predictor_create(const hrpp_bvh *bvh, const hrpp_predictor_desc *desc, void *d_buf,
                                  size_t bytes, void *stream, hrpp_predictor **out);

/* Enqueue a reset: every entry empty (all bytes 0xFF), the state in which
 * the predictor of section "Overview" starts, before any ray has reached a
 * leaf (section "Limit Study" measures from such an empty table).  Ray
 * queries that keep learning across calls (the frames or samples of one
 * render) simply do not reset between them.  The update marks
 * each group of 16 entries in which it tags an empty entry, so a reset
 * rewrites only the marked groups (the whole table after creation, an import
 * or a failed launch).  The per-epoch scratch (fallback queue, records,
 * fresh-id lists) is left cleared by every epoch, so it is cleared here only
 * after creation or a failed launch. */
hrpp_status hrpp_predictor_reset(hrpp_predictor *pred, void *stream);

/* Copy the table to host memory after the work on `stream` (synchronises
 * the stream): the predictor's contents (section "HRPP Hash Function": per
 * hash value, the leaf nodes recorded for it; the table's size is what
 * section "Limit Study" reports in megabytes).  Layout per entry: uint64 tag (all-ones = empty), then
 * `ways` uint32 slots (0xFFFFFFFF = empty; at go-up level 0 a leaf id
 * (first_tri << 3) | (count - 1), at level g >= 1 the canonical depth-first
 * index of the node g levels above the leaf), then a uint32 claim word
 * (0xFFFFFFFF between calls) and 0xFF padding up to the entry size (32 B
 * for ways <= 4, else 64 B). */
hrpp_status hrpp_predictor_export(const hrpp_predictor *pred, void *h_dst, size_t bytes, void *stream);

/* Overwrite the table from host memory (same layout as export); for
 * checkpoint/restore.  Synchronises the stream.  EINVAL if a claim word is
 * not 0xFFFFFFFF or a slot lies outside the predictor's BVH (a leaf id whose
 * triangle range passes the triangle count, or a node index >= the node
 * count); nothing is copied then. */
hrpp_status hrpp_predictor_import(hrpp_predictor *pred, const void *h_src, size_t bytes, void *stream);

void hrpp_predictor_destroy(hrpp_predictor *pred);

/* Any-hit (shadow / hit-any) query for n rays d_rays[0..n).  d_occluded[i]
 * = 1 if some triangle is hit inside (tmin, tmax), else 0.  pred NULL =
 * plain traversal; otherwise rays are processed in epochs of epoch_rays in
 * index order (the first one first_epoch_rays long): hash, lookup, test the
 * predicted leaves (stop at the first hit), traverse the rest, then update
 * the table -- the direct flow of section "Overview"; section "Precision
 * and Recall" defines the outcomes: a hit in a predicted leaf is a true
 * positive and ends the ray, any other positive and every negative traverse
 * as usual.  Any hit is a valid answer for this query, so the flag does not
 * depend on the predictor.  d_stats (may be NULL) is accumulated.  n == 0 is a
 * no-op.  Errors: EINVAL (null arrays with n > 0, n >= 2^31, predictor
 * built for another BVH, or a predictor whose last trace failed to launch
 * and that has not been reset since). */
hrpp_status hrpp_trace_anyhit(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint32_t n,
                              uint8_t *d_occluded, hrpp_stats *d_stats, void *stream);

/* Closest-hit (hit-all) query.  mode HRPP_CLOSEST_PAPER: a positive ray
 * whose predicted leaves hold a hit returns the best hit among them and
 * skips traversal (the paper's semantics, section "Precision and Recall":
 * a hit-all ray accepts a valid intersection in a predicted leaf, which may
 * not be the closest one).
 * HRPP_CLOSEST_EXACT: the best predicted hit only seeds the traversal's
 * interval, so the result is always the closest hit (ties: smaller prim).
 * Other arguments as for hrpp_trace_anyhit. */
hrpp_status hrpp_trace_closest(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint32_t n,
                               uint32_t mode, hrpp_hit *d_hits, hrpp_stats *d_stats, void *stream);

/* ------------------------------------------------------------------------
 * Plain-traversal baseline on a 4-wide BVH, collapsed on the host from the
 * binary tree (a stronger plain baseline than binary traversal; the paper
 * traverses a binary BVH, section "Overview").  Collapse: a wide node starts
 * from the two children of a binary interior node and, while it has fewer
 * than four, replaces its interior child of largest surface area by that
 * child's two children; leaves are the binary leaves.  A node's hit children
 * are visited nearest first.  Results equal the binary traversal's (any-hit
 * flags; the exact closest hit, ties to the smaller prim); the visit counts
 * in d_stats are the wide tree's own.  No predictor.
 * ------------------------------------------------------------------------ */

/* The wide tree of a BVH: node count, root reference (node 0, or bit 31 |
 * leaf id for a one-leaf tree), the largest stack it can need, its depth. */
hrpp_status hrpp_bvh_wide_info(const hrpp_bvh *bvh, uint32_t *num_nodes, uint32_t *root_ref, uint32_t *stack_need,
                               uint32_t *depth);

/* Copy the wide nodes to host memory: 32 uint32 words (128 B) per node:
 * [0..3] min x of children 0..3, [4..7] max x, [8..11] min y, [12..15]
 * max y, [16..19] min z, [20..23] max z (binary32 bits), [24..27] child
 * references (wide node index, bit 31 | leaf id, or 0xFFFFFFFF for no
 * child), [28..31] zero.  EINVAL if `words` is too small. */
hrpp_status hrpp_bvh_wide_export(const hrpp_bvh *bvh, uint32_t *h_words, size_t words);

/* Any-hit and exact closest-hit queries on the wide tree (arguments and
 * errors as for hrpp_trace_anyhit / hrpp_trace_closest without a
 * predictor); EINVAL for a BVH not uploaded. */
hrpp_status hrpp_trace_wide_anyhit(const hrpp_bvh *bvh, const hrpp_ray *d_rays, uint32_t n, uint8_t *d_occluded,
                                   hrpp_stats *d_stats, void *stream);
hrpp_status hrpp_trace_wide_closest(const hrpp_bvh *bvh, const hrpp_ray *d_rays, uint32_t n, hrpp_hit *d_hits,
                                    hrpp_stats *d_stats, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent jobs (each its own BVH, predictor or none, rays
 * and outputs) executed together.  Round r runs epoch r of every job (round
 * 0: each job's first epoch) in one launch per kernel, so scenes of uneven
 * size fill the GPU together; the
 * whole sequence can be captured once into a hipGraph and replayed.  Each
 * job computes exactly what its own hrpp_trace_* call would (results,
 * counters and table), because jobs share nothing and each job's epochs
 * stay in order.  Predictors must be distinct across the jobs of a batch.
 * The device pointers of the jobs are baked into the batch: to trace new
 * rays, write them into the same buffers and launch again.
 * ------------------------------------------------------------------------ */
typedef struct {
    const hrpp_bvh *bvh;
    hrpp_predictor *pred;      /* NULL = plain traversal */
    const hrpp_ray *d_rays;
    uint32_t n;
    uint32_t query;            /* 0 any-hit, 1 closest-hit */
    uint32_t mode;             /* closest-hit: HRPP_CLOSEST_PAPER or HRPP_CLOSEST_EXACT */
    void *d_out;               /* uint8_t[n] occlusion flags or hrpp_hit[n] */
    hrpp_stats *d_stats;       /* may be NULL */
} hrpp_batch_job;

typedef struct hrpp_batch hrpp_batch;

/* Device bytes of the job table, job ids and launch-grid offsets of a batch of
   njobs jobs (a buffer of this size, 256-byte aligned, for hrpp_batch_create). */
size_t hrpp_batch_required_bytes(uint32_t njobs);

/* Validate the jobs (as the trace calls do; EINVAL also for a predictor used
 * twice) and upload the job table into d_buf (256-byte aligned).
 * Synchronises `stream`. */
hrpp_status hrpp_batch_create(const hrpp_batch_job *jobs, uint32_t njobs, void *d_buf, size_t bytes,
                              void *stream, hrpp_batch **out);

/* Enqueue every job of the batch on `stream`.  use_graph != 0 captures the
 * launch sequence into a hipGraph on the first call and replays it later
 * (the kernels contain no memset, so the graph is replay-safe); 0 issues
 * the launches directly.  Predictors are not reset by the batch. */
hrpp_status hrpp_batch_launch(hrpp_batch *batch, uint32_t use_graph, void *stream);

void hrpp_batch_destroy(hrpp_batch *batch);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of ray-query requests against resident
 * scenes.  A scheduler thread admits queued requests (arrival order; a
 * request waiting only for a busy predictor does not hold back the requests
 * behind it, one waiting for pool space does) when
 *   - its rays and results fit in the device pool (the HBM budget for
 *     in-flight requests, caller-owned, 256-byte aligned),
 *   - one of `slots` streams is free, and
 *   - one of the scene's predictor replicas for the query kind is free;
 * it then copies the rays in, traces them and copies the results back on
 * the slot's stream.  Requests on different slots run concurrently, and new
 * requests are admitted as slots and pool space free up.  Predictors keep
 * their tables across requests.  Only any-hit and EXACT closest-hit are
 * served, whose results do not depend on the tables: a request's results
 * are the same alone and in any mix.
 * ------------------------------------------------------------------------ */
typedef struct {
    const hrpp_bvh *bvh;
    hrpp_predictor *const *any_preds;      /* replicas for any-hit requests (>= 1) */
    uint32_t n_any;
    hrpp_predictor *const *closest_preds;  /* replicas for closest-hit requests (>= 1) */
    uint32_t n_closest;
} hrpp_serve_scene;

typedef struct {
    uint32_t state;          /* 0 queued, 1 running, 2 done */
    hrpp_status status;
    double queue_ms;         /* submit -> admission */
    double service_ms;       /* admission -> results in host memory */
    double latency_ms;       /* submit -> results in host memory */
} hrpp_request_info;

typedef struct hrpp_server hrpp_server;

/* Start a server over `nscenes` scenes (each predictor may appear once). */
hrpp_status hrpp_serve_create(const hrpp_serve_scene *scenes, uint32_t nscenes, uint32_t slots, void *d_pool,
                              size_t pool_bytes, hrpp_server **out);

/* Add a scene to a running server (a scene that arrives while it serves,
 * e.g. one just built with hrpp_build_bvh_device).  The BVH and predictors
 * must be ready: their build and creation have completed (the device build
 * synchronises; predictor creation is ordered on its own stream, so
 * synchronise it), and they outlive the server.  Its predictors must not
 * serve another scene.  *index receives the new scene's index for
 * hrpp_serve_submit; the scenes already served keep theirs.  EINVAL for a
 * bad description or a server being destroyed. */
hrpp_status hrpp_serve_add_scene(hrpp_server *server, const hrpp_serve_scene *scene, uint32_t *index);

/* Remove a scene from a running server (to free its BVH and tables, e.g. to
 * stay within an HBM budget).  New requests for it are refused (EINVAL);
 * the call blocks until its queued and running requests are done, after
 * which its BVH and predictors may be freed or added again with another
 * scene.  The other scenes keep their indices; the index is not reused.
 * EINVAL for an unknown or already removed scene. */
hrpp_status hrpp_serve_remove_scene(hrpp_server *server, uint32_t index);

/* Queue a request: n rays in host memory (pinned memory lets the copies run
 * asynchronously), results to h_out (uint8_t[n] for query 0 = any-hit,
 * hrpp_hit[n] for query 1 = EXACT closest-hit).  Both buffers must stay
 * valid until the request is done.  EBUSY if the request can never fit
 * the pool. */
hrpp_status hrpp_serve_submit(hrpp_server *server, uint32_t scene, uint32_t query, const hrpp_ray *h_rays,
                              uint32_t n, void *h_out, uint64_t *request_id);

/* Non-blocking state and timings of a request.  The poll that reports a
 * request done (state 2) is its final one: it retires the request, whose
 * record is freed and whose id is unknown afterwards (EINVAL), so a server
 * that runs for a long time holds only the requests not yet read. */
hrpp_status hrpp_serve_poll(hrpp_server *server, uint64_t request_id, hrpp_request_info *info);

/* Block until every submitted request is done; the first failed status
 * since the server was created, if any.  A failed request's slot and pool
 * region are reused only after its stream has drained, and its predictor
 * replica is reset if its trace did not launch. */
hrpp_status hrpp_serve_wait_all(hrpp_server *server);

/* Number of request records the server holds: queued, running, or done and
 * not yet retired by a final poll. */
hrpp_status hrpp_serve_held(hrpp_server *server, uint64_t *held);

/* Largest pool occupancy seen so far (never above pool_bytes). */
hrpp_status hrpp_serve_pool_peak(hrpp_server *server, size_t *peak_bytes);

/* Drain the queue, stop the scheduler, free the handle. */
void hrpp_serve_destroy(hrpp_server *server);

/* Per-kernel timing for measurement.  Between hrpp_profile_start() and
 * hrpp_profile_stop(), every kernel the library launches is bracketed by two
 * HIP events recorded on the launch stream.  Stop waits for those events and
 * writes one record per kernel kind that ran (up to `capacity`; *count gets
 * the number of kinds).  Process-global and not thread-safe; timing adds a
 * few microseconds per launch, so time throughput with profiling off. */
typedef struct { char name[32]; uint64_t launches; double total_ms; } hrpp_kernel_time;
hrpp_status hrpp_profile_start(void);
hrpp_status hrpp_profile_stop(hrpp_kernel_time *out, uint32_t capacity, uint32_t *count);

/* Measurement only: the distinct memory lines each kernel kind touches.
 * After this call, every trace on `bvh` with predictor `pred` (NULL = plain
 * traversal) that is given a stats pointer also marks, in the device bitmap
 * d_bits, each 128-byte line of the scene and table arrays its kernels read
 * or write (atomic ORs: counting runs become slower; traces without stats are
 * unchanged).  The caller zeroes d_bits.  h_layout (11 words) receives the
 * layout: [0] words per kernel-kind block; [1..5] word offsets, within a
 * block, of the regions of interior nodes (64 B each), triangles (48 B), leaf
 * boxes (32 B), table entries (32 or 64 B) and canonical node records
 * (48 B); [6..10] the line count of each region.  Blocks follow each other
 * in the order prediction kernel, first-epoch kernel, fallback-queue kernel,
 * plain traversal kernel.  EINVAL if `words` is under 4 blocks or pred is
 * bound to another BVH.  d_bits NULL switches the marking off (and, given
 * bvh and h_layout, still writes the layout, to size a bitmap).  Process-
 * global, not thread-safe. */
hrpp_status hrpp_profile_touch(const hrpp_bvh *bvh, const hrpp_predictor *pred, uint32_t *d_bits, size_t words,
                               uint32_t *h_layout);

/* Synchronise `stream`; report HRPP_EDEVICE if a HIP error is pending and
 * HRPP_EDEPTH if a kernel tracing `bvh` (may be NULL) found a traversal
 * stack too small (cannot happen for trees built by hrpp_build_bvh). */
hrpp_status hrpp_get_error(const hrpp_bvh *bvh, void *stream);

const char *hrpp_status_string(hrpp_status s);

#ifdef __cplusplus
}
#endif
#endif /* HRPP_H */
