// HIP kernels of the HRPP library for CDNA4 (gfx950, wave64).
//
// Per epoch (a call's first epoch F rays, the others E; rays of epoch k see the
// table after epoch k-1):
//   k_predict    one lane per ray: validate, hash, probe the table, test the
//                predicted leaves (or walk the predicted subtrees, go-up
//                level >= 1); successes write their result; a wave with
//                enough failing rays traverses them in place, other waves
//                append theirs to the epoch's fallback queue (one atomic per
//                block on one of kSubQueues striped counters).
//   k_epoch_empty  the first epoch after a reset (empty table): every valid
//                ray traverses, one lane per ray, without reading the table.
//   k_traverse_queue  stack traversal of the queued rays.
//                A traversed ray with a hit emits one update record and
//                claims the record's entry with a 32-bit atomicMin on the ray
//                id (the smallest id owns it), wherever it traversed.
//   k_update_*   three passes over the epoch's records that turn the table
//                of epoch k-1 into the table of epoch k; an entry tagged
//                while empty marks its group for k_reset_table.
// Without a predictor:
//   k_traverse_plain  stack traversal of every ray (binary tree).
//   k_traverse_wide   the same on the 4-wide tree collapsed from it.
//
// Section references are to Demoullin, Gubran and Aamodt, "Hash-Based Ray
// Path Prediction".  Every floating-point expression below is written in
// the same operation order as the library's specification (binary32, no
// contraction: the file is compiled with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "hrpp_internal.h"
#include "hrpp_kernels.h"

namespace hrpp {

// ---------------------------------------------------------------------------
// Scalar building blocks
// ---------------------------------------------------------------------------

// Conservative far-distance factor 1 + 3 * 2^-23 (Ize, "Robust BVH Ray
// Traversal", JCGT 2013: >= 1 + 2 * gamma_3 covers rounding of the slab
// distances).
__device__ __forceinline__ float far_pad() { return __uint_as_float(0x3F800003u); }

__device__ __forceinline__ bool ray_is_valid(const float4 &a, const float4 &b) {
    bool fin = __builtin_isfinite(a.x) && __builtin_isfinite(a.y) && __builtin_isfinite(a.z) &&
               __builtin_isfinite(b.x) && __builtin_isfinite(b.y) && __builtin_isfinite(b.z);
    bool nonzero = !(b.x == 0.0f && b.y == 0.0f && b.z == 0.0f);
    bool interval = !__builtin_isnan(a.w) && !__builtin_isnan(b.w) && (a.w < b.w);
    return fin && nonzero && interval;
}

struct RayState {
    float ox, oy, oz, dx, dy, dz, ix, iy, iz, tmin, tmax;
};

// Slab test of one box against [tmin, tcur]; fminf/fmaxf ignore a NaN operand
// (IEEE minNum/maxNum, the gfx9 v_min/v_max behaviour in IEEE mode).
__device__ __forceinline__ bool slab(float x0, float y0, float z0, float x1, float y1, float z1,
                                     const RayState &r, float tcur, float &tnear) {
    float t0x = (x0 - r.ox) * r.ix, t1x = (x1 - r.ox) * r.ix;
    float t0y = (y0 - r.oy) * r.iy, t1y = (y1 - r.oy) * r.iy;
    float t0z = (z0 - r.oz) * r.iz, t1z = (z1 - r.oz) * r.iz;
    float lox = fminf(t0x, t1x), hix = fmaxf(t0x, t1x);
    float loy = fminf(t0y, t1y), hiy = fmaxf(t0y, t1y);
    float loz = fminf(t0z, t1z), hiz = fmaxf(t0z, t1z);
    tnear = fmaxf(fmaxf(fmaxf(lox, loy), loz), r.tmin);
    float tfar = fminf(fminf(fminf(hix, hiy), hiz), tcur) * far_pad();
    return tnear <= tfar;
}

// Moller-Trumbore on a stored triangle {v0, e1 = v1 - v0, e2 = v2 - v0}.
__device__ __forceinline__ bool intersect_tri(const float4 &A, const float4 &B, const float4 &C,
                                              const RayState &r, float &t, float &u, float &v) {
    const float e1x = B.x, e1y = B.y, e1z = B.z;
    const float e2x = C.x, e2y = C.y, e2z = C.z;
    float px = r.dy * e2z - r.dz * e2y;
    float py = r.dz * e2x - r.dx * e2z;
    float pz = r.dx * e2y - r.dy * e2x;
    float det = (e1x * px + e1y * py) + e1z * pz;
    if (det == 0.0f) return false;
    float inv = 1.0f / det;
    float sx = r.ox - A.x, sy = r.oy - A.y, sz = r.oz - A.z;
    u = ((sx * px + sy * py) + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    float qx = sy * e1z - sz * e1y;
    float qy = sz * e1x - sx * e1z;
    float qz = sx * e1y - sy * e1x;
    v = ((r.dx * qx + r.dy * qy) + r.dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
    return true;
}

__device__ __forceinline__ uint32_t quantize(float x, float maxcell) {
    float c = floorf(x);
    if (!(c >= 0.0f)) c = 0.0f;
    else if (c > maxcell) c = maxcell;
    return (uint32_t)c;
}

// Ray hash: origin cell on a 2^qo grid over the scene box, direction on a
// 2^qd x 2^qd octahedral map, packed into a key and folded into the table
// index by Fibonacci hashing (the section "HRPP Hash Function" asks for a
// hash that sends similar rays to the same entry).
// Mode 1 is the section's own encoding: per binary32 value the sign, the p
// leading exponent bits and the p leading mantissa bits (2p+1 bits, sign
// highest); origin and direction values are paired by XOR as (o.x, d.z),
// (o.y, d.y), (o.z, d.x) and the three fields packed at a stride of 8 or 16.
__device__ __forceinline__ uint32_t ieee_bits(float x, uint32_t p) {
    const uint32_t u = __float_as_uint(x);
    return ((u >> 31) << (2 * p)) | ((((u >> 23) & 0xFFu) >> (8 - p)) << p) | ((u & 0x7FFFFFu) >> (23 - p));
}

__device__ __forceinline__ void hash_ray(const HashArgs &h, const RayState &r, uint64_t &key, uint32_t &idx) {
    if (h.mode == 1) {
        const uint32_t p = h.qo;
        const uint64_t f0 = ieee_bits(r.ox, p) ^ ieee_bits(r.dz, p);
        const uint64_t f1 = ieee_bits(r.oy, p) ^ ieee_bits(r.dy, p);
        const uint64_t f2 = ieee_bits(r.oz, p) ^ ieee_bits(r.dx, p);
        key = f0 | (f1 << h.stride) | (f2 << (2 * h.stride));
        idx = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64u - h.log2n));
        return;
    }
    const float maxo = h.maxo, maxd = h.maxd, half = h.half;
    uint32_t cx = quantize((r.ox - h.bmin[0]) * h.scale[0], maxo);
    uint32_t cy = quantize((r.oy - h.bmin[1]) * h.scale[1], maxo);
    uint32_t cz = quantize((r.oz - h.bmin[2]) * h.scale[2], maxo);
    float l1 = (fabsf(r.dx) + fabsf(r.dy)) + fabsf(r.dz);
    float inv = 1.0f / l1;
    float px = r.dx * inv, py = r.dy * inv;
    if (r.dz < 0.0f) {
        float fx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
        float fy = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
        px = fx;
        py = fy;
    }
    uint32_t bu = quantize((px + 1.0f) * half, maxd);
    uint32_t bv = quantize((py + 1.0f) * half, maxd);
    const uint32_t qo = h.qo, qd = h.qd;
    key = (uint64_t)cx | ((uint64_t)cy << qo) | ((uint64_t)cz << (2 * qo)) | ((uint64_t)bu << (3 * qo)) |
          ((uint64_t)bv << (3 * qo + qd));
    idx = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64u - h.log2n));
}

// ---------------------------------------------------------------------------
// Counters: per-lane registers, reduced per block, one atomic per counter
// per block.
// ---------------------------------------------------------------------------
struct Counters {
    uint32_t v[kNumStats];
    uint32_t *touch;   // this kernel kind's block of the touch bitmap, or null
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < kNumStats; i++) v[i] = 0;
        touch = nullptr;
    }
};

// Measurement only: kernels with counters mark in a bitmap every 128-byte line
// of the scene and table arrays they read or write, when the caller asked for
// it (hrpp_profile_touch); without counters `touch` stays null and the marks
// compile away.
template <bool STATS>
__device__ __forceinline__ void bind_touch(Counters &c, const TraceArgs &a, int kind) {
    if constexpr (STATS)
        if (a.touch != nullptr) c.touch = a.touch + (size_t)kind * a.touch_kind_words;
}

__device__ __forceinline__ void touch(const TraceArgs &a, const Counters &c, int region, size_t off, uint32_t len) {
    if (c.touch == nullptr) return;
    const size_t l1 = (off + len - 1) >> 7;
    for (size_t l = off >> 7; l <= l1; l++) {
        const size_t bit = (size_t)a.touch_off[region] * 32 + l;
        atomicOr(&c.touch[bit >> 5], 1u << (bit & 31));
    }
}

template <bool STATS>
__device__ __forceinline__ void flush_counters(Counters &c, unsigned long long *stats) {
    if constexpr (STATS) {
        if (stats == nullptr) return;   // uniform per block: one block serves one job
        __shared__ unsigned long long red[kNumStats];
        if (threadIdx.x < kNumStats) red[threadIdx.x] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kNumStats; i++) {
            uint32_t x = c.v[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            if ((threadIdx.x & 63) == 0 && x) atomicAdd(&red[i], (unsigned long long)x);
        }
        __syncthreads();
        if (threadIdx.x < kNumStats && red[threadIdx.x]) atomicAdd(&stats[threadIdx.x], red[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// Leaf test (shared by prediction and traversal)
// ---------------------------------------------------------------------------
struct Best {
    float t, u, v;
    uint32_t prim, leaf;
};

// ANY: returns true at the first hit inside (tmin, tmax).  CLOSEST: keeps the
// lexicographically smallest (t, prim) and returns true if it changed.
template <bool ANY>
__device__ __forceinline__ bool test_leaf(const TraceArgs &a, uint32_t leaf, const RayState &r, Best &b,
                                          Counters &c) {
    const float4 *__restrict__ tris = (const float4 *)a.tris;
    const uint32_t first = leaf >> 3, cnt = (leaf & 7u) + 1u;
    touch(a, c, kTouchTris, (size_t)first * 48, cnt * 48);
    bool changed = false;
    for (uint32_t k = first; k < first + cnt; k++) {
        const float4 A = tris[3 * (size_t)k + 0];
        const float4 B = tris[3 * (size_t)k + 1];
        const float4 C = tris[3 * (size_t)k + 2];
        c.v[kTriTests]++;
        float t, u, v;
        if (!intersect_tri(A, B, C, r, t, u, v)) continue;
        if (!(r.tmin < t && t < r.tmax)) continue;
        const uint32_t prim = __float_as_uint(A.w);
        if constexpr (ANY) {
            b.t = t; b.u = u; b.v = v; b.prim = prim; b.leaf = leaf;
            return true;
        } else {
            if (t < b.t || (t == b.t && prim < b.prim)) {
                b.t = t; b.u = u; b.v = v; b.prim = prim; b.leaf = leaf;
                changed = true;
            }
        }
    }
    return changed;
}

// Traversal kernels run blocks of kTraceBlock lanes (BLK where a kernel runs
// larger blocks); the first entries of each lane's traversal stack live in
// LDS (walk()).  8 entries: for closest hit 4
// and 12 measured slower, for any hit 4 was slower and 12 or 16 no faster;
// 4 KB of LDS per block for any hit, 8 KB with the distances for closest hit.
constexpr uint32_t kTraceBlock = 128;
constexpr uint32_t kLdsStackAny = 8;
constexpr uint32_t kLdsStackClosest = 8;

// ---------------------------------------------------------------------------
// Stack traversal.  Fixed order: root box test; at an interior node both
// child boxes are tested against [tmin, tcur]; with both hit the nearer
// child (left on a tie) is taken and the other pushed with its entry
// distance; a popped node is visited only if its entry distance still passes
// against the current tcur; leaves test triangles in BVH order.
// Beyond its LDS entries the per-lane stack lives in private memory (the
// cached scratch path), sized to the deepest tree the library accepts; a
// whole stack in LDS limited closest-hit kernels to 3 waves per SIMD.
// Callers pass (pointer, stride 1, capacity = depth) for the private part.
// ---------------------------------------------------------------------------
// walk(): the subtree of `ref`, whose own box the caller has tested; from
// the root this is the whole traversal, from a predicted node (go-up level
// >= 1) the evaluation of that prediction.
template <bool ANY, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ bool walk(const TraceArgs &a, const RayState &r, Best &b, Counters &c, uint32_t ref,
                                     uint32_t *stk_node, float *stk_t, uint32_t stride, uint32_t cap) {
    const float4 *__restrict__ nodes = (const float4 *)a.nodes;
    float tcur = (!ANY && b.prim != kNone) ? b.t : r.tmax;
    bool found = (b.prim != kNone);
    // sp nodes are deferred: the newest (entry sp - 1) is held in registers
    // (top_ref, top_t), so a pop takes its node without waiting for memory and
    // the load of the next newest entry overlaps the work on the popped node.
    // The older entries: the first K in LDS, lane-interleaved (entry j of lane
    // l at word j * BLK + l: the 64 lanes of a wave touch 64
    // consecutive words), the rest in the private stack.  Closest hit keeps
    // each entry's distance beside it.
    uint32_t sp = 0, top_ref = 0;
    float top_t = 0.0f;
    constexpr uint32_t K = ANY ? kLdsStackAny : kLdsStackClosest;
    __shared__ uint32_t s_sn[K * BLK];
    __shared__ float s_st[ANY ? 1 : K * BLK];
    for (;;) {
        c.v[kNodesVisited]++;
        if (!(ref & kLeafFlag)) {
            c.v[kInteriorVisited]++;
            c.v[kBoxTests] += 2;
            touch(a, c, kTouchNodes, (size_t)ref * 64, 64);
            const float4 n0 = nodes[4 * (size_t)ref + 0];
            const float4 n1 = nodes[4 * (size_t)ref + 1];
            const float4 n2 = nodes[4 * (size_t)ref + 2];
            const uint4 n3 = ((const uint4 *)nodes)[4 * (size_t)ref + 3];
            float tl, tr;
            const bool hl = slab(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, r, tcur, tl);
            const bool hr = slab(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, r, tcur, tr);
            if (hl && hr) {
                uint32_t push_ref;
                float push_t;
                if (tr < tl) { push_ref = n3.x; push_t = tl; ref = n3.y; }
                else         { push_ref = n3.y; push_t = tr; ref = n3.x; }
                if (sp >= cap) { atomicOr(a.error, 1u); return found; }
                if (sp > 0) {
                    const uint32_t j = sp - 1;
                    if (j < K) {
                        s_sn[j * BLK + threadIdx.x] = top_ref;
                        if constexpr (!ANY) s_st[j * BLK + threadIdx.x] = top_t;
                    } else {
                        stk_node[(j - K) * stride] = top_ref;
                        if constexpr (!ANY) stk_t[(j - K) * stride] = top_t;
                    }
                }
                top_ref = push_ref;
                top_t = push_t;
                sp++;
                continue;
            }
            if (hl) { ref = n3.x; continue; }
            if (hr) { ref = n3.y; continue; }
        } else {
            c.v[kLeafVisited]++;
            if (test_leaf<ANY>(a, ref & ~kLeafFlag, r, b, c)) {
                found = true;
                if constexpr (ANY) return true;
                tcur = b.t;
            }
        }
        // pop
        for (;;) {
            if (sp == 0) return found;
            sp--;
            const uint32_t pref = top_ref;
            const float pt = top_t;
            if (sp > 0) {
                const uint32_t j = sp - 1;
                if (j < K) {
                    top_ref = s_sn[j * BLK + threadIdx.x];
                    if constexpr (!ANY) top_t = s_st[j * BLK + threadIdx.x];
                } else {
                    top_ref = stk_node[(j - K) * stride];
                    if constexpr (!ANY) top_t = stk_t[(j - K) * stride];
                }
            }
            if (ANY || pt <= tcur * far_pad()) {
                ref = pref;
                break;
            }
        }
    }
}

template <bool ANY, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ bool traverse(const TraceArgs &a, const RayState &r, Best &b, Counters &c,
                                         uint32_t *stk_node, float *stk_t, uint32_t stride, uint32_t cap) {
    const float tcur = (!ANY && b.prim != kNone) ? b.t : r.tmax;
    float tn;
    c.v[kTraversals]++;
    c.v[kBoxTests]++;
    if (!slab(a.root_box[0], a.root_box[1], a.root_box[2], a.root_box[3], a.root_box[4], a.root_box[5], r, tcur, tn))
        return b.prim != kNone;
    return walk<ANY, BLK>(a, r, b, c, a.root_ref, stk_node, stk_t, stride, cap);
}

// Canonical node record: min xyz, max x | max yz, reference, depth | parent,
// subtree triangle range [lo, hi), 0.
__device__ __forceinline__ const uint32_t *cnode_ptr(const TraceArgs &a, uint32_t node) {
    return (const uint32_t *)a.cnode + 12 * (size_t)node;
}

// The node a record names: the result leaf (go-up level 0), or its ancestor
// go_up levels up, stopping at the root.
__device__ __forceinline__ uint32_t record_node(const TraceArgs &a, const Counters &c, uint32_t leaf) {
    if (a.go_up == 0) return leaf;
    touch(a, c, kTouchLeafbox, (size_t)(leaf >> 3) * 32, 32);
    const float4 b1 = ((const float4 *)a.leafbox)[2 * (size_t)(leaf >> 3) + 1];
    uint32_t node = __float_as_uint(b1.w);
    for (uint32_t k = 0; k < a.go_up; k++) {
        touch(a, c, kTouchCnode, (size_t)node * 48, 48);
        const uint32_t p = cnode_ptr(a, node)[8];
        if (p == kNone) break;
        node = p;
    }
    return node;
}

__device__ __forceinline__ RayState load_ray(const float4 *rays, uint32_t rid, float4 &a, float4 &b) {
    a = rays[2 * (size_t)rid + 0];
    b = rays[2 * (size_t)rid + 1];
    RayState r;
    r.ox = a.x; r.oy = a.y; r.oz = a.z; r.tmin = a.w;
    r.dx = b.x; r.dy = b.y; r.dz = b.z; r.tmax = b.w;
    r.ix = 0.0f; r.iy = 0.0f; r.iz = 0.0f;
    return r;
}

// Reciprocal direction (three correctly rounded binary32 divisions), needed
// only by box tests.
__device__ __forceinline__ void set_inverse(RayState &r) {
    r.ix = 1.0f / r.dx; r.iy = 1.0f / r.dy; r.iz = 1.0f / r.dz;
}

template <bool ANY>
__device__ __forceinline__ void write_result(const TraceArgs &a, uint32_t rid, bool hit, const Best &b) {
    if constexpr (ANY) {
        a.occluded[rid] = hit ? 1 : 0;
    } else {
        float4 h;
        if (hit) { h.x = b.t; h.y = b.u; h.z = b.v; h.w = __uint_as_float(b.prim); }
        else     { h.x = __builtin_inff(); h.y = 0.0f; h.z = 0.0f; h.w = __uint_as_float(kNone); }
        ((float4 *)a.hits)[rid] = h;
    }
}

// Table entry access.  Entry: u64 tag | u32 slot[W] | u32 claim | padding.
__device__ __forceinline__ const uint32_t *entry_ptr(const TraceArgs &a, uint32_t idx) {
    return (const uint32_t *)((const char *)a.table + (size_t)idx * a.entry_bytes);
}

// ---------------------------------------------------------------------------
// Per-ray phases
// ---------------------------------------------------------------------------

// Prediction for ray `rid` ("Overview": hash, look up, evaluate the predicted
// leaves or, at go-up level >= 1, walk the predicted subtrees).  Returns true
// if the ray must still traverse; then *seed_leaf is the leaf of the best
// predicted hit (EXACT) or kNone.
template <bool ANY, bool EXACT, bool SUBTREE, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ bool predict_one(const TraceArgs &a, uint32_t rid, Counters &c, uint32_t &seed_leaf,
                                            uint32_t *stk_node, float *stk_t, uint32_t stride, uint32_t cap) {
    float4 ra, rb;
    RayState r = load_ray((const float4 *)a.rays, rid, ra, rb);
    seed_leaf = kNone;
    c.v[kRays]++;
    if (!ray_is_valid(ra, rb)) {
        c.v[kInvalid]++;
        write_result<ANY>(a, rid, false, Best{});
        return false;
    }
    uint64_t key;
    uint32_t idx;
    hash_ray(a.hash, r, key, idx);
    c.v[kLookups]++;
    touch(a, c, kTouchEntries, (size_t)idx * a.entry_bytes, a.entry_bytes);
    const uint32_t *e = entry_ptr(a, idx);
    const uint64_t tag = *(const uint64_t *)e;
    const uint32_t W = a.ways;
    Best b;
    b.t = __builtin_inff(); b.u = 0.0f; b.v = 0.0f; b.prim = kNone; b.leaf = kNone;
    const bool positive = (tag == key) && (e[2] != kNone);
    bool hit = false;
    uint32_t skip_depth = 0;
    if (SUBTREE && positive) {
        c.v[kPositives]++;
        set_inverse(r);
        const uint32_t box0 = c.v[kBoxTests], leaf0 = c.v[kLeafVisited], tri0 = c.v[kTriTests];
        // predicted nodes in slot order: the node's box against [tmin, tcur],
        // then a walk of its subtree; the interior nodes above the node that
        // produced the result are the ones skipped
        for (uint32_t s = 0; s < W; s++) {
            const uint32_t node = e[2 + s];
            if (node == kNone) break;
            touch(a, c, kTouchCnode, (size_t)node * 48, 48);
            const float4 *nb = (const float4 *)cnode_ptr(a, node);
            const float4 n0 = nb[0], n1 = nb[1];
            const float tcur = (!ANY && b.prim != kNone) ? b.t : r.tmax;
            float tn;
            c.v[kBoxTests]++;
            if (!slab(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, r, tcur, tn)) continue;
            const float bt = b.t;
            const uint32_t bp = b.prim;
            const bool f = walk<ANY, BLK>(a, r, b, c, __float_as_uint(n1.z), stk_node, stk_t, stride, cap);
            if (b.prim != bp || b.t != bt) skip_depth = __float_as_uint(n1.w);
            if (f) {
                hit = true;
                if (ANY) break;
            }
        }
        c.v[kPredBoxTests] += c.v[kBoxTests] - box0;
        c.v[kPredLeafVisited] += c.v[kLeafVisited] - leaf0;
        c.v[kPredTriTests] += c.v[kTriTests] - tri0;
    } else if (positive) {
        c.v[kPositives]++;
        set_inverse(r);
        const float4 *__restrict__ lbox = (const float4 *)a.leafbox;
        // predicted leaves in slot order: the leaf's box against [tmin, tcur]
        // (tcur = tmax, or the best hit so far for closest hit), then its
        // triangles if the box is hit
        for (uint32_t s = 0; s < W; s++) {
            const uint32_t leaf = e[2 + s];
            if (leaf == kNone) break;
            touch(a, c, kTouchLeafbox, (size_t)(leaf >> 3) * 32, 32);
            const float4 b0 = lbox[2 * (size_t)(leaf >> 3) + 0];
            const float4 b1 = lbox[2 * (size_t)(leaf >> 3) + 1];
            const float tcur = (!ANY && b.prim != kNone) ? b.t : r.tmax;
            float tn;
            c.v[kBoxTests]++;
            c.v[kPredBoxTests]++;
            if (!slab(b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, r, tcur, tn)) continue;
            c.v[kNodesVisited]++;
            c.v[kLeafVisited]++;
            c.v[kPredLeafVisited]++;
            const uint32_t before = c.v[kTriTests];
            const bool h = test_leaf<ANY>(a, leaf, r, b, c);
            c.v[kPredTriTests] += c.v[kTriTests] - before;
            if (h) {
                hit = true;
                if (ANY) break;
            }
        }
    }
    if (EXACT) {
        // every valid ray traverses; the best predicted hit seeds its interval
        if (!ANY) {
            float4 h;
            h.x = b.t; h.y = b.u; h.z = b.v; h.w = __uint_as_float(b.prim);
            ((float4 *)a.hits)[rid] = h;
        }
        seed_leaf = b.leaf;
        return true;
    }
    if (positive && hit) {
        c.v[kPredHits]++;
        c.v[kHits]++;
        if (SUBTREE) {
            c.v[kNodesSkipped] += skip_depth;
        } else {
            // the leaf's interior-ancestor count is stored with its box
            touch(a, c, kTouchLeafbox, (size_t)(b.leaf >> 3) * 32, 32);
            const float4 b1 = ((const float4 *)a.leafbox)[2 * (size_t)(b.leaf >> 3) + 1];
            c.v[kNodesSkipped] += __float_as_uint(b1.z);
        }
        write_result<ANY>(a, rid, true, b);
        return false;
    }
    if (positive) c.v[kFalsePos]++;
    return true;   // back to the pool of rays to traverse (section "Precision and Recall")
}

// Full traversal of ray `rid`.  HRPP: a fallback ray (already validated and
// counted by the prediction step, from the queue, in place, or in the first
// epoch after a reset); emit its update record and claim the entry.  PLAIN:
// validate and count here.
template <bool ANY, bool EXACT, bool HRPP, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ void traverse_one(const TraceArgs &a, uint32_t base, uint32_t rid, uint32_t seed_leaf,
                                             Counters &c, uint32_t *stk_node, float *stk_t, uint32_t stride,
                                             uint32_t cap) {
    float4 ra, rb;
    RayState r = load_ray((const float4 *)a.rays, rid, ra, rb);
    if (!HRPP) {
        c.v[kRays]++;
        if (!ray_is_valid(ra, rb)) {
            c.v[kInvalid]++;
            write_result<ANY>(a, rid, false, Best{});
            return;
        }
    }
    set_inverse(r);
    Best b;
    b.t = __builtin_inff(); b.u = 0.0f; b.v = 0.0f; b.prim = kNone; b.leaf = kNone;
    if (!ANY && EXACT && HRPP) {
        const float4 s = ((const float4 *)a.hits)[rid];
        b.t = s.x; b.u = s.y; b.v = s.z; b.prim = __float_as_uint(s.w); b.leaf = seed_leaf;
    }
    const bool hit = traverse<ANY, BLK>(a, r, b, c, stk_node, stk_t, stride, cap);
    write_result<ANY>(a, rid, hit, b);
    if (hit) c.v[kHits]++;
    if (HRPP) {
        // the key is needed by a record (a hit) and by the EXACT positive check
        uint64_t key = 0;
        uint32_t idx = 0;
        if (hit || (!ANY && EXACT)) hash_ray(a.hash, r, key, idx);
        if (!ANY && EXACT) {
            touch(a, c, kTouchEntries, (size_t)idx * a.entry_bytes, a.entry_bytes);
            const uint32_t *e = entry_ptr(a, idx);
            const bool positive = (*(const uint64_t *)e == key) && (e[2] != kNone);
            if (positive) {
                // the final best lies in a predicted leaf, or in the
                // subtree of a predicted node
                bool in_pred = false;
                for (uint32_t s = 0; s < a.ways; s++) {
                    const uint32_t l = e[2 + s];
                    if (l == kNone) break;
                    if (!hit) continue;
                    if (a.go_up == 0) {
                        if (l == b.leaf) in_pred = true;
                    } else {
                        touch(a, c, kTouchCnode, (size_t)l * 48, 48);
                        const uint32_t *cn = cnode_ptr(a, l);
                        const uint32_t first = b.leaf >> 3;
                        if (cn[9] <= first && first < cn[10]) in_pred = true;
                    }
                }
                if (in_pred) c.v[kPredHits]++;
                else c.v[kFalsePos]++;
            }
        }
        if (hit) {
            const uint32_t slot = rid - base;
            a.rec_key[slot] = key;
            a.rec_idx[slot] = idx;
            a.rec_leaf[slot] = record_node(a, c, b.leaf);
            touch(a, c, kTouchEntries, (size_t)idx * a.entry_bytes, a.entry_bytes);
            uint32_t *e = (uint32_t *)entry_ptr(a, idx);
            // the smallest ray id claims the entry (with the resident policy only
            // a record of the resident key, or any record for an empty entry;
            // the table does not change during an epoch); claims only decrease
            // within an epoch, so a coherent read that is already <= rid spares
            // the atomic
            const uint64_t tag = *(const uint64_t *)e;
            if (!(a.policy & 2u) || tag == kEmptyTag || tag == key) {
                const uint32_t seen = __hip_atomic_load(&e[2 + a.ways], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seen > rid) atomicMin(&e[2 + a.ways], rid);
            }
            c.v[kRecords]++;
        }
    }
}

// ---------------------------------------------------------------------------
// Plain traversal of the 4-wide tree (the stronger plain baseline).  A node's
// up to four child boxes are tested against [tmin, tcur]; the hit children
// are ordered by entry distance (ties to the lower child slot), the nearest
// is visited and the others are pushed farthest first; popping and leaf
// tests follow the binary traversal.  The closest hit is the exact one
// (lexicographic (t, prim) minimum), so its results equal the binary
// traversal's; its visit counts are its own.
// ---------------------------------------------------------------------------
template <bool ANY>
__device__ __forceinline__ bool traverse_wide(const TraceArgs &a, const RayState &r, Best &b, Counters &c,
                                              uint32_t *stk_node, float *stk_t, uint32_t stride, uint32_t cap) {
    const float4 *__restrict__ wn = (const float4 *)a.wide;
    float tcur = (!ANY && b.prim != kNone) ? b.t : r.tmax;
    bool found = (b.prim != kNone);
    float tn;
    c.v[kTraversals]++;
    c.v[kBoxTests]++;
    if (!slab(a.root_box[0], a.root_box[1], a.root_box[2], a.root_box[3], a.root_box[4], a.root_box[5], r, tcur, tn))
        return found;
    uint32_t ref = a.wide_root;
    uint32_t sp = 0;
    for (;;) {
        c.v[kNodesVisited]++;
        if (!(ref & kLeafFlag)) {
            c.v[kInteriorVisited]++;
            const float4 *q = wn + 8 * (size_t)ref;
            const float4 x0 = q[0], x1 = q[1], y0 = q[2], y1 = q[3], z0 = q[4], z1 = q[5];
            const uint4 rf = ((const uint4 *)q)[6];
            // one sort key per child slot: miss flag, entry distance in an
            // order-preserving encoding, slot index (ties keep slot order);
            // sorted by a 5-comparator network, all in registers
            uint64_t key[4];
            float tk[4];
            uint32_t nh = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const float mnx = k == 0 ? x0.x : k == 1 ? x0.y : k == 2 ? x0.z : x0.w;
                const float mxx = k == 0 ? x1.x : k == 1 ? x1.y : k == 2 ? x1.z : x1.w;
                const float mny = k == 0 ? y0.x : k == 1 ? y0.y : k == 2 ? y0.z : y0.w;
                const float mxy = k == 0 ? y1.x : k == 1 ? y1.y : k == 2 ? y1.z : y1.w;
                const float mnz = k == 0 ? z0.x : k == 1 ? z0.y : k == 2 ? z0.z : z0.w;
                const float mxz = k == 0 ? z1.x : k == 1 ? z1.y : k == 2 ? z1.z : z1.w;
                const uint32_t rk = k == 0 ? rf.x : k == 1 ? rf.y : k == 2 ? rf.z : rf.w;
                bool h = false;
                float t = 0.0f;
                if (rk != kNone) {
                    c.v[kBoxTests]++;
                    h = slab(mnx, mny, mnz, mxx, mxy, mxz, r, tcur, t);
                }
                const uint32_t u = __float_as_uint(t);
                const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
                key[k] = ((uint64_t)(h ? 0u : 1u) << 40) | ((uint64_t)ord << 2) | (uint64_t)k;
                tk[k] = t;
                nh += h ? 1u : 0u;
            }
#define HRPP_CSWAP(i, j) { const uint64_t lo_ = key[i] < key[j] ? key[i] : key[j]; \
                           const uint64_t hi_ = key[i] < key[j] ? key[j] : key[i]; key[i] = lo_; key[j] = hi_; }
            HRPP_CSWAP(0, 1) HRPP_CSWAP(2, 3) HRPP_CSWAP(0, 2) HRPP_CSWAP(1, 3) HRPP_CSWAP(1, 2)
#undef HRPP_CSWAP
            if (nh > 0) {
                if (sp + nh - 1 > cap) { atomicOr(a.error, 1u); return found; }
                // push the hit children farthest first; visit the nearest
#pragma unroll
                for (int j = 3; j >= 0; j--) {
                    const uint32_t k = (uint32_t)(key[j] & 3u);
                    const uint32_t rk = k == 0 ? rf.x : k == 1 ? rf.y : k == 2 ? rf.z : rf.w;
                    const float t = k == 0 ? tk[0] : k == 1 ? tk[1] : k == 2 ? tk[2] : tk[3];
                    if ((uint32_t)j >= nh) continue;
                    if (j == 0) {
                        ref = rk;
                    } else {
                        stk_node[sp * stride] = rk;
                        if constexpr (!ANY) stk_t[sp * stride] = t;
                        sp++;
                    }
                }
                continue;
            }
        } else {
            c.v[kLeafVisited]++;
            if (test_leaf<ANY>(a, ref & ~kLeafFlag, r, b, c)) {
                found = true;
                if constexpr (ANY) return true;
                tcur = b.t;
            }
        }
        for (;;) {
            if (sp == 0) return found;
            sp--;
            if constexpr (ANY) break;
            else if (stk_t[sp * stride] <= tcur * far_pad()) break;
        }
        ref = stk_node[sp * stride];
    }
}

// PRIV: the stack in per-lane private memory (backed by the cached scratch
// path) instead of LDS, so that the wide tree's deep worst-case stack does
// not limit occupancy; used when the stack need fits kWidePrivStack.
constexpr uint32_t kWidePrivStack = 48;

template <bool ANY, bool STATS, bool PRIV>
__global__ __launch_bounds__(128) void k_traverse_wide(TraceArgs a, uint32_t count) {
    extern __shared__ uint32_t lds[];
    uint32_t pn[PRIV ? kWidePrivStack : 1];
    float pt[PRIV ? kWidePrivStack : 1];
    const uint32_t stride = PRIV ? 1u : blockDim.x;
    const uint32_t cap = PRIV ? kWidePrivStack : a.stack_cap;
    uint32_t *stk_node = PRIV ? pn : lds + threadIdx.x;
    float *stk_t = PRIV ? pt : (float *)(lds + cap * stride + threadIdx.x);
    Counters c;
    c.zero();
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += step) {
        float4 ra, rb;
        RayState r = load_ray((const float4 *)a.rays, i, ra, rb);
        c.v[kRays]++;
        if (!ray_is_valid(ra, rb)) {
            c.v[kInvalid]++;
            write_result<ANY>(a, i, false, Best{});
            continue;
        }
        set_inverse(r);
        Best b;
        b.t = __builtin_inff(); b.u = 0.0f; b.v = 0.0f; b.prim = kNone; b.leaf = kNone;
        const bool hit = traverse_wide<ANY>(a, r, b, c, stk_node, stk_t, stride, cap);
        write_result<ANY>(a, i, hit, b);
        if (hit) c.v[kHits]++;
    }
    flush_counters<STATS>(c, a.stats);
}

// ---------------------------------------------------------------------------
// Plain traversal: every ray of [0, count), grid-stride loop (the single call
// launches one lane per ray; the batch kernel shares a grid among jobs).
// ---------------------------------------------------------------------------
template <bool ANY, bool STATS>
__device__ __forceinline__ void body_traverse_plain(const TraceArgs &a, uint32_t count, uint32_t bx, uint32_t gx) {
    uint32_t stk_node[kMaxDepth];                // per-lane stack in private memory
    float stk_t[ANY ? 1 : kMaxDepth];
    const uint32_t stride = 1;
    const uint32_t cap = a.stack_cap;            // the tree's depth, <= kMaxDepth
    Counters c;
    c.zero();
    bind_touch<STATS>(c, a, kTouchPlain);
    const uint32_t step = gx * blockDim.x;
    for (uint32_t i = bx * blockDim.x + threadIdx.x; i < count; i += step)
        traverse_one<ANY, false, false>(a, 0, i, kNone, c, stk_node, stk_t, stride, cap);
    flush_counters<STATS>(c, a.stats);
}

template <bool ANY, bool STATS>
__global__ __launch_bounds__(128) void k_traverse_plain(TraceArgs a, uint32_t count) {
    body_traverse_plain<ANY, STATS>(a, count, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Prediction for one epoch: one lane per ray.  A wave in which at least
// inline_min rays must still traverse traverses them at once (their lanes
// would mostly be busy anyway); other waves append theirs to the epoch's
// compacted fallback queue.  Either way a ray runs the same traversal and
// emits the same record, so results do not depend on the split.
// ---------------------------------------------------------------------------
template <bool ANY, bool EXACT, bool STATS, bool SUBTREE, bool INLINE, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ void body_predict(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    // SUBTREE (go-up level >= 1) walks predicted nodes and INLINE traverses
    // failing rays in place, both with a traversal stack; without either the
    // stack is unused
    uint32_t stk_node[kMaxDepth];                // per-lane stack in private memory
    float stk_t[ANY ? 1 : kMaxDepth];
    const uint32_t stride = 1;
    const uint32_t cap = a.stack_cap;            // the tree's depth, <= kMaxDepth
    Counters c;
    c.zero();
    bind_touch<STATS>(c, a, kTouchPredict);
    const uint32_t i = bx * blockDim.x + threadIdx.x;
    bool enq = false;
    uint32_t seed_leaf = kNone;
    if (i < count) enq = predict_one<ANY, EXACT, SUBTREE, BLK>(a, base + i, c, seed_leaf, stk_node, stk_t, stride, cap);
    const bool inline_wave = INLINE && (uint32_t)__popcll(__ballot(enq)) >= a.inline_min;   // uniform per wave
    const bool now = enq && inline_wave;
    enq = enq && !inline_wave;
    // append to the fallback queue: lanes are counted per wave (ballot), waves
    // per block (LDS atomic), and each block takes its range with one global
    // atomic on one of kSubQueues striped counters, so no single counter sees
    // more than one atomic per kSubQueues blocks
    __shared__ uint32_t s_count, s_base;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    const uint64_t mask = __ballot(enq);
    const uint32_t lane = __lane_id();
    uint32_t wave_off = 0;
    if (lane == 0 && mask) wave_off = atomicAdd(&s_count, (uint32_t)__popcll(mask));
    wave_off = __shfl(wave_off, 0);
    __syncthreads();
    const uint32_t sub = bx % kSubQueues;
    if (threadIdx.x == 0 && s_count) s_base = atomicAdd(&a.ctrl[sub], s_count);
    __syncthreads();
    if (enq) {
        const uint32_t pos = s_base + wave_off + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        a.queue[(size_t)sub * a.queue_subcap + pos] = (uint64_t)(base + i) | ((uint64_t)seed_leaf << 32);
    }
    if (INLINE && now) traverse_one<ANY, EXACT, true, BLK>(a, base, base + i, seed_leaf, c, stk_node, stk_t, stride, cap);
    flush_counters<STATS>(c, a.stats);
}

template <bool ANY, bool EXACT, bool STATS, bool SUBTREE, bool INLINE>
__global__ __launch_bounds__(256) void k_predict(TraceArgs a, uint32_t base, uint32_t count) {
    body_predict<ANY, EXACT, STATS, SUBTREE, INLINE>(a, base, count, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// The first epoch after a reset: the table is empty, so every valid ray's
// lookup is negative and every valid ray traverses.  Same counts, records
// and claims as the prediction kernel followed by the queue, without the
// entry reads and the queue; a grid-stride loop like plain traversal,
// launched with one lane per ray.
// ---------------------------------------------------------------------------
template <bool ANY, bool EXACT, bool STATS, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ void body_epoch_empty(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    uint32_t stk_node[kMaxDepth];                // per-lane stack in private memory
    float stk_t[ANY ? 1 : kMaxDepth];
    const uint32_t stride = 1;
    const uint32_t cap = a.stack_cap;            // the tree's depth, <= kMaxDepth
    Counters c;
    c.zero();
    bind_touch<STATS>(c, a, kTouchEmpty);
    const uint32_t step = gx * blockDim.x;
    for (uint32_t i = bx * blockDim.x + threadIdx.x; i < count; i += step) {
        const uint32_t rid = base + i;
        float4 ra, rb;
        load_ray((const float4 *)a.rays, rid, ra, rb);
        c.v[kRays]++;
        if (!ray_is_valid(ra, rb)) {
            c.v[kInvalid]++;
            write_result<ANY>(a, rid, false, Best{});
            continue;
        }
        c.v[kLookups]++;
        c.v[kEmptyLookups]++;
        if (!ANY && EXACT) {
            // no predicted hit seeds the interval
            float4 h;
            h.x = __builtin_inff(); h.y = 0.0f; h.z = 0.0f; h.w = __uint_as_float(kNone);
            ((float4 *)a.hits)[rid] = h;
        }
        traverse_one<ANY, EXACT, true, BLK>(a, base, rid, kNone, c, stk_node, stk_t, stride, cap);
    }
    // schedule counters: all of this kernel's work is first-epoch work
    c.v[kEmptyRays] = c.v[kRays];
    c.v[kEmptyInteriorVisited] = c.v[kInteriorVisited];
    c.v[kEmptyTriTests] = c.v[kTriTests];
    c.v[kEmptyRecords] = c.v[kRecords];
    flush_counters<STATS>(c, a.stats);
}

template <bool ANY, bool EXACT, bool STATS>
__global__ __launch_bounds__(128) void k_epoch_empty(TraceArgs a, uint32_t base, uint32_t count) {
    body_epoch_empty<ANY, EXACT, STATS>(a, base, count, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Traversal of the epoch's fallback queue (its length is read on the device;
// the grid covers the epoch, lanes past the queue's end exit at once).
// ---------------------------------------------------------------------------
template <bool ANY, bool EXACT, bool STATS, uint32_t BLK = kTraceBlock>
__device__ __forceinline__ void body_traverse_queue(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    uint32_t stk_node[kMaxDepth];                // per-lane stack in private memory
    float stk_t[ANY ? 1 : kMaxDepth];
    const uint32_t stride = 1;
    const uint32_t cap = a.stack_cap;            // the tree's depth, <= kMaxDepth
    Counters c;
    c.zero();
    bind_touch<STATS>(c, a, kTouchQueue);
    // the sub-queue counts are final when this kernel starts (the prediction
    // kernel before it wrote them): one uniform read per wave
    static_assert(kSubQueues == 8, "the counts are read as two uint4");
    uint32_t cnt[kSubQueues];
    uint32_t total = 0;
    const uint4 c0 = *(const uint4 *)&a.ctrl[0], c1 = *(const uint4 *)&a.ctrl[4];
    cnt[0] = __builtin_amdgcn_readfirstlane(c0.x); cnt[1] = __builtin_amdgcn_readfirstlane(c0.y);
    cnt[2] = __builtin_amdgcn_readfirstlane(c0.z); cnt[3] = __builtin_amdgcn_readfirstlane(c0.w);
    cnt[4] = __builtin_amdgcn_readfirstlane(c1.x); cnt[5] = __builtin_amdgcn_readfirstlane(c1.y);
    cnt[6] = __builtin_amdgcn_readfirstlane(c1.z); cnt[7] = __builtin_amdgcn_readfirstlane(c1.w);
#pragma unroll
    for (uint32_t k = 0; k < kSubQueues; k++) total += cnt[k];
    const uint32_t step = gx * blockDim.x;
    for (uint32_t i = bx * blockDim.x + threadIdx.x; i < total; i += step) {
        // work item i -> (sub-queue, offset)
        uint32_t sub = 0, off = i;
        bool found = false;
#pragma unroll
        for (uint32_t k = 0; k < kSubQueues; k++) {
            if (!found) {
                if (off < cnt[k]) found = true;
                else { off -= cnt[k]; sub++; }
            }
        }
        const uint64_t q = a.queue[(size_t)sub * a.queue_subcap + off];
        traverse_one<ANY, EXACT, true, BLK>(a, base, (uint32_t)q, (uint32_t)(q >> 32), c, stk_node, stk_t, stride, cap);
    }
    // schedule counters: all of this kernel's work is queued fallback work
    c.v[kQueueTraversals] = c.v[kTraversals];
    c.v[kQueueInteriorVisited] = c.v[kInteriorVisited];
    c.v[kQueueTriTests] = c.v[kTriTests];
    c.v[kQueueRecords] = c.v[kRecords];
    flush_counters<STATS>(c, a.stats);
}

template <bool ANY, bool EXACT, bool STATS>
__global__ __launch_bounds__(128) void k_traverse_queue(TraceArgs a, uint32_t base, uint32_t count) {
    body_traverse_queue<ANY, EXACT, STATS>(a, base, count, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// K3: epoch-end update (section "HRPP Hash Function": a conflicting ray's
// leaf is inserted into the existing entry unless already present; the paper
// has no replacement policy, section "Precision and Recall").  Deterministic
// batch form in which the smallest ray id wins every conflict: the key of the
// smallest claiming ray id owns an entry touched this epoch (with the
// resident policy only the resident key's records, or any record for an
// empty entry, claim); the owner's new ids enter the free slots in the order
// of the smallest ray id that recorded each, and the rest are dropped, or,
// with FIFO eviction, the first W of them enter at the back and the oldest
// slots make room.
//   U1 classify (records): classify each record against the claim winner; a
//       fresh (owner, id) pair enters the epoch's pair set, which keeps the
//       smallest ray id that recorded it (64-bit compare-and-swap on the pair,
//       32-bit atomicMin on its ray id).
//   U2 rank (records): the record holding its pair's smallest ray id inserts
//       (ray id << 32 | id) into the owner's list of the entry's free-slot
//       count smallest such values (64-bit atomicMin cascade); one record per
//       id, so the list holds distinct ids in ray order.
//   U3 apply (winning records): rewrite the entry, release the claim, clear
//       the list and the pair set; an entry that was empty marks its group
//       for the reset.
//   U4 finish (records, with counters only): count drops, clear the record
//       slot, reset the queue count.
// ---------------------------------------------------------------------------
enum : uint32_t { kRecConflict = 1, kRecPresent = 2, kRecFresh = 3 };
constexpr uint32_t kRecOwner = 1u << 6;   // status flag: this record's ray holds the entry's claim
constexpr uint64_t kNone64 = 0xFFFFFFFFFFFFFFFFull;

__device__ __forceinline__ uint32_t pair_slot(uint64_t pair, uint32_t bits) {
    return (uint32_t)((pair * 0x9E3779B97F4A7C15ull) >> (64u - bits));
}

template <bool STATS>
__device__ __forceinline__ void body_update_classify(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    Counters c;
    c.zero();
    const uint32_t i = bx * blockDim.x + threadIdx.x;
    const uint32_t W = a.ways;
    // a fresh record's pair: the claiming ray and the id to insert
    uint32_t ins_owner = kNone, ins_leaf = kNone, free_slots = 0, status = 0, own = 0;
    if (i < count && a.rec_idx[i] != kNone) {
        const uint32_t idx = a.rec_idx[i];
        const uint32_t *e = entry_ptr(a, idx);
        const uint32_t owner = e[2 + W];                // smallest ray id (claim)
        if (owner == base + i) own = kRecOwner;         // the claim is final until the apply pass
        // with the resident policy an entry may have no claim: every record
        // of the epoch had another key than the resident tag
        const uint64_t kstar = owner == kNone ? ~a.rec_key[i] : a.rec_key[owner - base];
        const uint32_t leaf = a.rec_leaf[i];
        if (a.rec_key[i] != kstar) {
            status = kRecConflict;
            c.v[kConflicts]++;
        } else {
            bool present = false;
            if (*(const uint64_t *)e == kstar) {
                for (uint32_t s = 0; s < W; s++) {
                    const uint32_t l = e[2 + s];
                    if (l == kNone) break;
                    if (l == leaf) present = true;
                }
            }
            if (present) {
                status = kRecPresent;
            } else {
                status = kRecFresh;
                // room for new ids after this epoch's claim: the free slots,
                // or every slot with FIFO eviction
                free_slots = W;
                if (*(const uint64_t *)e == kstar && !(a.policy & 1u)) {
                    uint32_t used = 0;
                    while (used < W && e[2 + used] != kNone) used++;
                    free_slots = W - used;
                }
                ins_owner = owner;
                ins_leaf = leaf;
            }
        }
    }
    // Record slots are ray ids: a record whose left neighbour lane carries the
    // same (owner, id) pair has a larger ray id than that neighbour, so it is
    // not its pair's first record and takes no further part.
    const uint32_t lane = __lane_id();
    const uint32_t prev_owner = __shfl_up(ins_owner, 1), prev_leaf = __shfl_up(ins_leaf, 1);
    const bool dup = lane > 0 && prev_owner == ins_owner && prev_leaf == ins_leaf;
    uint32_t hslot1 = 0;
    if (ins_owner != kNone && !dup && free_slots > 0) {
        // enter the pair into the set (linear probing; the set is at most half
        // full, so a free or matching slot is always found) and lower its ray id
        const uint64_t pair = ((uint64_t)(ins_owner - base) << 32) | ins_leaf;
        const uint32_t mask = (1u << a.hash_bits) - 1u;
        uint32_t h = pair_slot(pair, a.hash_bits);
        for (;;) {
            uint64_t k = __hip_atomic_load(&a.pairs[h].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k == kNone64) k = atomicCAS(&a.pairs[h].key, kNone64, (unsigned long long)pair);
            if (k == kNone64 || k == pair) break;
            h = (h + 1u) & mask;
        }
        const uint32_t seen = __hip_atomic_load(&a.pairs[h].min, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (seen > base + i) atomicMin(&a.pairs[h].min, base + i);
        hslot1 = h + 1u;
    }
    if (i < count && status != 0)
        a.rec_status[i] = status | (free_slots << 2) | (hslot1 << 8) | own;
    flush_counters<STATS>(c, a.stats);
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_update_classify(TraceArgs a, uint32_t base, uint32_t count) {
    body_update_classify<STATS>(a, base, count, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void body_update_rank(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    const uint32_t i = bx * blockDim.x + threadIdx.x;
    if (i >= count || a.rec_idx[i] == kNone) return;
    const uint32_t st = a.rec_status[i];
    if ((st & 3u) != kRecFresh || (st >> 8) == 0) return;
    const uint32_t h = (st >> 8) - 1u;
    const uint32_t rid = base + i;
    if (a.pairs[h].min != rid) return;                 // a smaller ray id recorded the same pair
    const uint32_t free_slots = (st >> 2) & 15u;
    const uint32_t idx = a.rec_idx[i];
    const uint32_t owner = entry_ptr(a, idx)[2 + a.ways];
    // sorted insertion into the entry's list of the free_slots smallest
    // (ray id, id) values; list values only ever decrease, so a plain read that
    // is already below x lets us skip the atomic at that position
    uint64_t *list = a.topw + (size_t)(a.topw_by_entry ? idx : owner - base) * a.ways;
    uint64_t x = ((uint64_t)rid << 32) | a.rec_leaf[i];
    for (uint32_t s = 0; s < free_slots && x != kNone64; s++) {
        const uint64_t seen = __hip_atomic_load(&list[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (seen < x) continue;                      // x cannot go here
        const uint64_t old = atomicMin((unsigned long long *)&list[s], (unsigned long long)x);
        if (old > x) x = old;                        // x took this place; carry the old value on
    }
}

__global__ __launch_bounds__(256) void k_update_rank(TraceArgs a, uint32_t base, uint32_t count) {
    body_update_rank(a, base, count, blockIdx.x, gridDim.x);
}

template <bool STATS>
__device__ __forceinline__ void body_update_apply(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    Counters c;
    c.zero();
    const uint32_t i = bx * blockDim.x + threadIdx.x;
    if (i < count && a.rec_idx[i] != kNone) {
        const uint32_t idx = a.rec_idx[i];
        const uint32_t W = a.ways;
        const uint32_t st = a.rec_status[i];
        if (st & kRecOwner) {                          // this ray owns the entry
            uint32_t *e = (uint32_t *)entry_ptr(a, idx);
            const uint64_t kstar = a.rec_key[i];
            uint32_t used = 0;
            if (*(const uint64_t *)e != kstar) {
                // an entry that leaves the empty state marks its group for the
                // reset (a plain byte store: every writer stores the same 1)
                if (*(const uint64_t *)e == kEmptyTag) a.dirty[idx / kResetGroup] = 1;
                *(uint64_t *)e = kstar;
                for (uint32_t s = 0; s < W; s++) e[2 + s] = kNone;
                c.v[kTagClaims]++;
            } else {
                while (used < W && e[2 + used] != kNone) used++;
            }
            uint64_t *list = a.topw + (size_t)(a.topw_by_entry ? idx : i) * W;
            if (a.policy & 1u) {
                // FIFO: the oldest (front) slots make room for the new ids
                uint32_t nf = 0;
                while (nf < W && list[nf] != kNone64) nf++;
                const uint32_t evict = used + nf > W ? used + nf - W : 0;
                for (uint32_t s = 0; s + evict < used; s++) e[2 + s] = e[2 + s + evict];
                used -= evict;
                c.v[kEvictions] += evict;
            }
            for (uint32_t s = 0; s < W; s++) {
                const uint64_t l = list[s];
                if (l != kNone64 && used < W) {
                    e[2 + used++] = (uint32_t)l;           // ids in increasing ray id
                    c.v[kLeafInserts]++;
                }
                list[s] = kNone64;
            }
            e[2 + W] = kNone;                          // release the claim
        }
        // the pair set is read no more in this epoch: empty this record's slot
        // (every record of the pair writes the same values)
        if ((st >> 8) != 0) {
            a.pairs[(st >> 8) - 1u].key = kNone64;
            a.pairs[(st >> 8) - 1u].min = kNone;
        }
        if (!STATS) a.rec_idx[i] = kNone;            // no drop count to take: retire the record now
    }
    if (!STATS && i < kSubQueues) a.ctrl[i] = 0;   // queue counters of the next epoch
    flush_counters<STATS>(c, a.stats);
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_update_apply(TraceArgs a, uint32_t base, uint32_t count) {
    body_update_apply<STATS>(a, base, count, blockIdx.x, gridDim.x);
}

template <bool STATS>
__device__ __forceinline__ void body_update_finish(const TraceArgs &a, uint32_t base, uint32_t count, uint32_t bx, uint32_t gx) {
    Counters c;
    c.zero();
    const uint32_t i = bx * blockDim.x + threadIdx.x;
    if (i < kSubQueues) a.ctrl[i] = 0;   // queue counters of the next epoch
    if (i < count && a.rec_idx[i] != kNone) {
        // a record of the owner key counts a drop if its id is not in the
        // final entry (with FIFO eviction this includes ids present before)
        if ((a.rec_status[i] & 3u) != kRecConflict) {
            const uint32_t *e = entry_ptr(a, a.rec_idx[i]);
            const uint32_t leaf = a.rec_leaf[i];
            bool present = false;
            for (uint32_t s = 0; s < a.ways; s++)
                if (e[2 + s] == leaf) present = true;
            if (!present) c.v[kDropped]++;
        }
        a.rec_idx[i] = kNone;
    }
    flush_counters<STATS>(c, a.stats);
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_update_finish(TraceArgs a, uint32_t base, uint32_t count) {
    body_update_finish<STATS>(a, base, count, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// A whole call in one workgroup, for epochs of at most kBlockEpoch rays.  The
// workgroup runs each epoch's prediction (or first-epoch traversal), queue
// traversal and update passes in order, with a workgroup barrier where the
// multi-launch form has a kernel boundary; it calls the same bodies, the
// epoch split into chunks of blockDim lanes (chunk k playing block k), so
// every result, record, table entry and counter equals the multi-launch
// form's.  With small epochs a call is otherwise a chain of four or five
// launches per epoch whose cost is mostly launch and drain.  The waves of a
// workgroup run on one compute unit and share its L1 cache; the barrier
// (a workgroup-scope release and acquire) makes every phase's stores and
// atomics visible to the next phase's loads.
// ---------------------------------------------------------------------------
constexpr uint32_t kBlockEpoch = kBlockEpochRays;

template <bool ANY, bool EXACT, bool STATS, bool SUBTREE, bool INLINE>
__device__ __forceinline__ void body_epochs_block(const TraceArgs &a, uint32_t n, uint32_t first, uint32_t epoch,
                                                  bool empty_table) {
    for (uint32_t base = 0; base < n;) {
        const uint32_t cnt = min(base == 0 ? first : epoch, n - base);
        const uint32_t chunks = (cnt + blockDim.x - 1) / blockDim.x;
        if (base == 0 && empty_table) {
            body_epoch_empty<ANY, EXACT, STATS, kBlockEpoch>(a, base, cnt, 0, 1);
        } else {
            for (uint32_t k = 0; k < chunks; k++)
                body_predict<ANY, EXACT, STATS, SUBTREE, INLINE, kBlockEpoch>(a, base, cnt, k, chunks);
            if (a.inline_min > 1) {
                __syncthreads();
                body_traverse_queue<ANY, EXACT, STATS, kBlockEpoch>(a, base, cnt, 0, 1);
            }
        }
        __syncthreads();
        for (uint32_t k = 0; k < chunks; k++) body_update_classify<STATS>(a, base, cnt, k, chunks);
        __syncthreads();
        for (uint32_t k = 0; k < chunks; k++) body_update_rank(a, base, cnt, k, chunks);
        __syncthreads();
        for (uint32_t k = 0; k < chunks; k++) body_update_apply<STATS>(a, base, cnt, k, chunks);
        __syncthreads();
        if (STATS) {
            for (uint32_t k = 0; k < chunks; k++) body_update_finish<STATS>(a, base, cnt, k, chunks);
            __syncthreads();
        }
        base += cnt;
    }
}

template <bool ANY, bool EXACT, bool STATS, bool SUBTREE, bool INLINE>
__global__ __launch_bounds__(kBlockEpoch) void k_epochs_block(TraceArgs a, uint32_t n, uint32_t first,
                                                              uint32_t epoch, uint32_t empty_table) {
    body_epochs_block<ANY, EXACT, STATS, SUBTREE, INLINE>(a, n, first, epoch, empty_table != 0);
}

// ---------------------------------------------------------------------------
// Batched execution: many independent (BVH, predictor, rays) jobs.  Round r
// runs epoch r of every job of a group in one launch per kernel, over a flat
// grid in which each job owns as many blocks as its longest epoch needs; each
// job's epochs stay in order, and jobs share nothing, so every job computes
// exactly what its own call computes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool batch_epoch(const BatchJob &J, uint32_t round, uint32_t &base, uint32_t &count) {
    // round 0 is the first epoch (J.first rays), round r >= 1 the r-th of J.epoch
    const uint64_t b = round == 0 ? 0 : (uint64_t)J.first + (uint64_t)(round - 1) * J.epoch;
    if (b >= J.n) return false;
    base = (uint32_t)b;
    count = min(round == 0 ? J.first : J.epoch, J.n - base);
    return true;
}

// The job owning block bx of a flat grid: the k with off[k] <= bx < off[k + 1]
// (off increasing, off[0] = 0), counted 64 offsets at a time with one load
// and a ballot per wave.  Called by every lane of the wave.
__device__ __forceinline__ uint32_t batch_job_of(const uint32_t *__restrict__ off, uint32_t njobs, uint32_t bx) {
    uint32_t le = 0;
    for (uint32_t c = 0; c < njobs; c += 64u) {
        const uint32_t j = c + __lane_id();
        const uint32_t m = (uint32_t)__popcll(__ballot(j < njobs && off[j] <= bx));
        le += m;
        if (m < 64u) break;
    }
    return le - 1u;
}

// Resolve block blockIdx.x of a group's flat grid to its job, the job's epoch
// of this round, and the block's index among the job's blocks.
struct BatchBlock {
    const BatchJob *J;
    uint32_t base, count, bx, gx;
};
__device__ __forceinline__ bool batch_block(const BatchJob *__restrict__ jobs, const uint32_t *__restrict__ ids,
                                            const uint32_t *__restrict__ off, uint32_t njobs, uint32_t round,
                                            BatchBlock &b) {
    const uint32_t k = batch_job_of(off, njobs, blockIdx.x);
    const uint32_t first = off[k];
    b.J = &jobs[ids[k]];
    b.bx = blockIdx.x - first;
    b.gx = off[k + 1] - first;
    return batch_epoch(*b.J, round, b.base, b.count) && b.bx * blockDim.x < b.count;
}

template <bool ANY, bool EXACT, bool STATS, bool SUBTREE, bool INLINE>
__global__ __launch_bounds__(256) void kb_predict(const BatchJob *__restrict__ jobs, const uint32_t *__restrict__ ids,
                                                  const uint32_t *__restrict__ off, uint32_t njobs, uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_predict<ANY, EXACT, STATS, SUBTREE, INLINE>(b.J->a, b.base, b.count, b.bx, b.gx);
}

template <bool ANY, bool EXACT, bool STATS>
__global__ __launch_bounds__(128) void kb_traverse_queue(const BatchJob *__restrict__ jobs,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ off, uint32_t njobs,
                                                         uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_traverse_queue<ANY, EXACT, STATS>(b.J->a, b.base, b.count, b.bx, b.gx);
}

template <bool STATS>
__global__ __launch_bounds__(256) void kb_update_classify(const BatchJob *__restrict__ jobs,
                                                          const uint32_t *__restrict__ ids,
                                                          const uint32_t *__restrict__ off, uint32_t njobs,
                                                          uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_update_classify<STATS>(b.J->a, b.base, b.count, b.bx, b.gx);
}

__global__ __launch_bounds__(256) void kb_update_rank(const BatchJob *__restrict__ jobs,
                                                      const uint32_t *__restrict__ ids,
                                                      const uint32_t *__restrict__ off, uint32_t njobs,
                                                      uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_update_rank(b.J->a, b.base, b.count, b.bx, b.gx);
}

template <bool STATS>
__global__ __launch_bounds__(256) void kb_update_apply(const BatchJob *__restrict__ jobs,
                                                       const uint32_t *__restrict__ ids,
                                                       const uint32_t *__restrict__ off, uint32_t njobs,
                                                       uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_update_apply<STATS>(b.J->a, b.base, b.count, b.bx, b.gx);
}

template <bool STATS>
__global__ __launch_bounds__(256) void kb_update_finish(const BatchJob *__restrict__ jobs,
                                                        const uint32_t *__restrict__ ids,
                                                        const uint32_t *__restrict__ off, uint32_t njobs,
                                                        uint32_t round) {
    BatchBlock b;
    if (!batch_block(jobs, ids, off, njobs, round, b)) return;
    body_update_finish<STATS>(b.J->a, b.base, b.count, b.bx, b.gx);
}

// Jobs whose epochs all hold at most kBlockEpoch rays: one workgroup per job
// runs all of the job's epochs (as k_epochs_block does for one call; the
// batch's first epoch goes through the prediction kernel, as in its rounds).
template <bool ANY, bool EXACT, bool STATS, bool SUBTREE>
__global__ __launch_bounds__(kBlockEpoch) void kb_epochs_block(const BatchJob *__restrict__ jobs,
                                                               const uint32_t *__restrict__ ids) {
    const BatchJob &J = jobs[ids[blockIdx.x]];
    body_epochs_block<ANY, EXACT, STATS, SUBTREE, true>(J.a, J.n, J.first, J.epoch, false);
}

// Plain jobs: one flat grid, each job getting blocks in proportion to its rays.
template <bool ANY, bool STATS>
__global__ __launch_bounds__(128) void kb_traverse_plain(const BatchJob *__restrict__ jobs,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ block_off, uint32_t count) {
    const uint32_t k = batch_job_of(block_off, count, blockIdx.x);
    const BatchJob &J = jobs[ids[k]];
    body_traverse_plain<ANY, STATS>(J.a, J.n, blockIdx.x - block_off[k], block_off[k + 1] - block_off[k]);
}

// Fill a region with a 32-bit pattern (predictor reset; a kernel rather than
// a memset so that the call can sit inside a captured graph).
__global__ void k_fill32(uint32_t *p, size_t n, uint32_t value) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Reset of a predictor table.  The update marks the group of kResetGroup
// entries of every entry it tags while the entry is empty, so every entry that
// is not empty lies in a marked group.  One wave per 64 groups: each lane reads
// one mark, and the wave clears the marked groups with coalesced 16-byte
// stores of all-ones (every group with `full`), then clears the marks.
__global__ __launch_bounds__(256) void k_reset_table(uint4 *table, uint32_t entry_u4, uint32_t n_entries,
                                                     uint8_t *dirty, uint32_t full) {
    const uint32_t lane = __lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / 64u;
    const uint32_t n_groups = (n_entries + kResetGroup - 1u) / kResetGroup;
    const uint32_t g = wave * 64u + lane;
    bool marked = false;
    if (g < n_groups) {
        marked = full || dirty[g] != 0;
        if (marked) dirty[g] = 0;
    }
    uint64_t m = __ballot(marked);
    const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
    const size_t end_all = (size_t)n_entries * entry_u4;
    while (m) {
        const uint32_t b = (uint32_t)__builtin_ctzll(m);
        m &= m - 1ull;
        const size_t first = (size_t)(wave * 64u + b) * kResetGroup * entry_u4;
        const size_t end = min(end_all, first + (size_t)kResetGroup * entry_u4);
        for (size_t j = first + lane; j < end; j += 64) table[j] = ones;
    }
}

// ---------------------------------------------------------------------------
// Per-kernel timing (measurement only): when enabled, each launch is
// bracketed by two HIP events recorded on the launch stream.
// ---------------------------------------------------------------------------
namespace {
struct ProfRecord {
    int kind;
    hipEvent_t start, stop;
};
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    int kind;
    ProfScope(int k, hipStream_t st) : s(st), kind(k) {
        if (!g_prof_on) return;
        a = pooled_event();
        b = pooled_event();
        if (a) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!g_prof_on || !a || !b) return;
        (void)hipEventRecord(b, s);
        g_prof.push_back({kind, a, b});
    }
};
}  // namespace

const char *kernel_kind_name(int k) {
    static const char *names[kNumKernelKinds] = {"k_predict", "k_traverse_queue", "k_traverse_plain",
                                                 "k_update_classify", "k_update_apply", "k_update_finish",
                                                 "k_fill32", "k_traverse_wide", "k_epoch_empty", "k_reset_table",
                                                 "k_update_rank", "k_epochs_block"};
    return (k >= 0 && k < kNumKernelKinds) ? names[k] : "unknown";
}

void profile_start() {
    g_prof_on = true;
}

int profile_stop(double *ms, uint64_t *launches) {
    g_prof_on = false;
    for (int k = 0; k < kNumKernelKinds; k++) { ms[k] = 0.0; launches[k] = 0; }
    int err = 0;
    for (auto &r : g_prof) {
        float t = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess)
            err = 1;
        ms[r.kind] += t;
        launches[r.kind]++;
        g_event_pool.push_back(r.start);
        g_event_pool.push_back(r.stop);
    }
    g_prof.clear();
    return err;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static inline uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }


template <bool ANY, bool EXACT, bool STATS>
static void launch_epoch(const TraceArgs &a, uint32_t base, uint32_t count, bool empty_table, hipStream_t s) {
    const uint32_t g256 = ceil_div(count, 256);
    const size_t lds = 0;   // traversal stacks live in private memory
    const uint32_t persistent = std::min<uint32_t>(ceil_div(count, 128), a.max_blocks);
    if (empty_table) {
        // every valid ray traverses, one lane per ray (as plain traversal); no
        // queue is filled
        ProfScope p(kKindEpochEmpty, s);
        hipLaunchKernelGGL((k_epoch_empty<ANY, EXACT, STATS>), dim3(ceil_div(count, 128)), dim3(128), lds, s, a,
                           base, count);
    } else {
        {
            // with in-place traversal or predicted subtrees: blocks of 128 lanes
            // (like the traversal kernels); otherwise 256 lanes
            ProfScope p(kKindPredict, s);
            const bool inl = a.inline_min <= 64;
            const dim3 g128(ceil_div(count, 128)), b128(128);
            if (a.go_up != 0) {
                if (inl) hipLaunchKernelGGL((k_predict<ANY, EXACT, STATS, true, true>), g128, b128, lds, s, a, base, count);
                else     hipLaunchKernelGGL((k_predict<ANY, EXACT, STATS, true, false>), g128, b128, lds, s, a, base, count);
            } else if (inl) {
                hipLaunchKernelGGL((k_predict<ANY, EXACT, STATS, false, true>), g128, b128, lds, s, a, base, count);
            } else {
                hipLaunchKernelGGL((k_predict<ANY, EXACT, STATS, false, false>), dim3(g256), dim3(256), 0, s, a,
                                   base, count);
            }
        }
        if (a.inline_min > 1) {
            // (with inline_min 1 every wave that has a failing ray traverses
            // in place, so the queue stays empty and is not launched)
            ProfScope p(kKindTraverseQueue, s);
            hipLaunchKernelGGL((k_traverse_queue<ANY, EXACT, STATS>), dim3(persistent), dim3(128), lds, s, a, base,
                               count);
        }
    }
    {
        ProfScope p(kKindUpdateClassify, s);
        hipLaunchKernelGGL((k_update_classify<STATS>), dim3(g256), dim3(256), 0, s, a, base, count);
    }
    {
        ProfScope p(kKindUpdateRank, s);
        hipLaunchKernelGGL(k_update_rank, dim3(g256), dim3(256), 0, s, a, base, count);
    }
    {
        ProfScope p(kKindUpdateApply, s);
        hipLaunchKernelGGL((k_update_apply<STATS>), dim3(g256), dim3(256), 0, s, a, base, count);
    }
    if (STATS) {
        // counts records whose leaf did not fit, then retires the records
        ProfScope p(kKindUpdateFinish, s);
        hipLaunchKernelGGL((k_update_finish<STATS>), dim3(g256), dim3(256), 0, s, a, base, count);
    }
}

template <bool ANY, bool EXACT, bool STATS>
static void launch_epochs_block(const TraceArgs &a, uint32_t n, uint32_t first, uint32_t epoch, bool empty_table,
                                hipStream_t s) {
    ProfScope p(kKindEpochsBlock, s);
    const dim3 g(1), b(kBlockEpoch);
    const uint32_t e0 = empty_table ? 1u : 0u;
    const bool inl = a.inline_min <= 64;
    if (a.go_up != 0) {
        if (inl) hipLaunchKernelGGL((k_epochs_block<ANY, EXACT, STATS, true, true>), g, b, 0, s, a, n, first, epoch, e0);
        else     hipLaunchKernelGGL((k_epochs_block<ANY, EXACT, STATS, true, false>), g, b, 0, s, a, n, first, epoch, e0);
    } else {
        if (inl) hipLaunchKernelGGL((k_epochs_block<ANY, EXACT, STATS, false, true>), g, b, 0, s, a, n, first, epoch, e0);
        else     hipLaunchKernelGGL((k_epochs_block<ANY, EXACT, STATS, false, false>), g, b, 0, s, a, n, first, epoch, e0);
    }
}

template <bool ANY, bool STATS>
static void launch_plain(const TraceArgs &a, uint32_t n, hipStream_t s) {
    const size_t lds = 0;   // the traversal stack lives in private memory
    // one ray per lane: the hardware dispatcher balances blocks of uneven cost
    // better than a persistent grid-stride loop (4-7% faster on the at-scale
    // queries)
    const uint32_t blocks = ceil_div(n, 128);
    ProfScope p(kKindTraversePlain, s);
    hipLaunchKernelGGL((k_traverse_plain<ANY, STATS>), dim3(blocks), dim3(128), lds, s, a, n);
}

void launch_trace(const TraceArgs &args, uint32_t n, bool any, bool exact, bool hrpp, uint32_t epoch,
                  uint32_t first_epoch, bool empty_table, hipStream_t s) {
    const bool st = args.stats != nullptr;
    if (!hrpp) {
        if (any) { if (st) launch_plain<true, true>(args, n, s); else launch_plain<true, false>(args, n, s); }
        else     { if (st) launch_plain<false, true>(args, n, s); else launch_plain<false, false>(args, n, s); }
        return;
    }
    if (first_epoch <= kBlockEpoch && epoch <= kBlockEpoch) {
        // small epochs: the whole call in one workgroup, one launch
        if (any) {
            if (st) launch_epochs_block<true, false, true>(args, n, first_epoch, epoch, empty_table, s);
            else    launch_epochs_block<true, false, false>(args, n, first_epoch, epoch, empty_table, s);
        } else if (exact) {
            if (st) launch_epochs_block<false, true, true>(args, n, first_epoch, epoch, empty_table, s);
            else    launch_epochs_block<false, true, false>(args, n, first_epoch, epoch, empty_table, s);
        } else {
            if (st) launch_epochs_block<false, false, true>(args, n, first_epoch, epoch, empty_table, s);
            else    launch_epochs_block<false, false, false>(args, n, first_epoch, epoch, empty_table, s);
        }
        return;
    }
    for (uint32_t base = 0; base < n;) {
        const uint32_t cnt = std::min(base == 0 ? first_epoch : epoch, n - base);
        // an empty table predicts nothing: the first epoch after a reset
        // traverses every ray, with the dedicated kernel
        const bool e0 = (base == 0 && empty_table);
        if (any) {
            if (st) launch_epoch<true, false, true>(args, base, cnt, e0, s);
            else    launch_epoch<true, false, false>(args, base, cnt, e0, s);
        } else if (exact) {
            if (st) launch_epoch<false, true, true>(args, base, cnt, e0, s);
            else    launch_epoch<false, true, false>(args, base, cnt, e0, s);
        } else {
            if (st) launch_epoch<false, false, true>(args, base, cnt, e0, s);
            else    launch_epoch<false, false, false>(args, base, cnt, e0, s);
        }
        base += cnt;
    }
}

void launch_wide(const TraceArgs &a, uint32_t n, bool any, hipStream_t s) {
    const bool priv = a.stack_cap <= kWidePrivStack;
    const size_t lds = priv ? 0 : (size_t)(any ? 1 : 2) * a.stack_cap * 128 * sizeof(uint32_t);
    const uint32_t blocks = std::min<uint32_t>(ceil_div(n, 128), a.max_blocks);
    const bool st = a.stats != nullptr;
    const dim3 g(blocks), b(128);
    ProfScope p(kKindTraverseWide, s);
    if (priv) {
        if (any) {
            if (st) hipLaunchKernelGGL((k_traverse_wide<true, true, true>), g, b, 0, s, a, n);
            else    hipLaunchKernelGGL((k_traverse_wide<true, false, true>), g, b, 0, s, a, n);
        } else {
            if (st) hipLaunchKernelGGL((k_traverse_wide<false, true, true>), g, b, 0, s, a, n);
            else    hipLaunchKernelGGL((k_traverse_wide<false, false, true>), g, b, 0, s, a, n);
        }
    } else if (any) {
        if (st) hipLaunchKernelGGL((k_traverse_wide<true, true, false>), g, b, lds, s, a, n);
        else    hipLaunchKernelGGL((k_traverse_wide<true, false, false>), g, b, lds, s, a, n);
    } else {
        if (st) hipLaunchKernelGGL((k_traverse_wide<false, true, false>), g, b, lds, s, a, n);
        else    hipLaunchKernelGGL((k_traverse_wide<false, false, false>), g, b, lds, s, a, n);
    }
}

void launch_fill32(uint32_t *p, size_t n, uint32_t value, hipStream_t s) {
    if (n == 0) return;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + 255) / 256, 4096);
    ProfScope prof(kKindFill, s);
    hipLaunchKernelGGL(k_fill32, dim3(blocks), dim3(256), 0, s, p, n, value);
}

void launch_reset_table(void *table, uint32_t entry_bytes, uint32_t n_entries, uint8_t *dirty, bool full,
                        hipStream_t s) {
    const uint32_t n_groups = (n_entries + kResetGroup - 1u) / kResetGroup;
    const uint32_t waves = (n_groups + 63u) / 64u;
    const uint32_t blocks = (waves + 3u) / 4u;
    ProfScope prof(kKindResetTable, s);
    hipLaunchKernelGGL(k_reset_table, dim3(blocks), dim3(256), 0, s, (uint4 *)table, entry_bytes / 16u, n_entries,
                       dirty, full ? 1u : 0u);
}

}  // namespace hrpp

namespace hrpp {

template <bool ANY, bool EXACT, bool STATS>
static void launch_batch_round(const BatchJob *jobs, const uint32_t *ids, const BatchGroup &g, uint32_t r,
                               hipStream_t s) {
    const uint32_t *gid = ids + g.first_id;
    const uint32_t nj = g.count;
    const size_t lds = 0;   // traversal stacks live in private memory
    const dim3 g128(g.blocks128), g256(g.blocks256), gq(g.blocksq);
    if (g.subtree)
        hipLaunchKernelGGL((kb_predict<ANY, EXACT, STATS, true, true>), g128, dim3(128), lds, s, jobs, gid,
                           g.d_off128, nj, r);
    else if (g.inline_any)
        hipLaunchKernelGGL((kb_predict<ANY, EXACT, STATS, false, true>), g128, dim3(128), lds, s, jobs, gid,
                           g.d_off128, nj, r);
    else
        hipLaunchKernelGGL((kb_predict<ANY, EXACT, STATS, false, false>), g256, dim3(256), 0, s, jobs, gid,
                           g.d_off256, nj, r);
    hipLaunchKernelGGL((kb_traverse_queue<ANY, EXACT, STATS>), gq, dim3(128), lds, s, jobs, gid, g.d_offq, nj, r);
    hipLaunchKernelGGL((kb_update_classify<STATS>), g256, dim3(256), 0, s, jobs, gid, g.d_off256, nj, r);
    hipLaunchKernelGGL(kb_update_rank, g256, dim3(256), 0, s, jobs, gid, g.d_off256, nj, r);
    hipLaunchKernelGGL((kb_update_apply<STATS>), g256, dim3(256), 0, s, jobs, gid, g.d_off256, nj, r);
    if (STATS)
        hipLaunchKernelGGL((kb_update_finish<STATS>), g256, dim3(256), 0, s, jobs, gid, g.d_off256, nj, r);
}

template <bool ANY, bool EXACT, bool STATS>
static void launch_batch_block_epochs(const BatchJob *jobs, const uint32_t *ids, const BatchGroup &g,
                                      hipStream_t s) {
    const uint32_t *gid = ids + g.first_id;
    if (g.subtree)
        hipLaunchKernelGGL((kb_epochs_block<ANY, EXACT, STATS, true>), dim3(g.count), dim3(kBlockEpoch), 0, s, jobs,
                           gid);
    else
        hipLaunchKernelGGL((kb_epochs_block<ANY, EXACT, STATS, false>), dim3(g.count), dim3(kBlockEpoch), 0, s, jobs,
                           gid);
}

template <bool ANY, bool STATS>
static void launch_batch_plain(const BatchJob *jobs, const uint32_t *ids, const BatchGroup &g, hipStream_t s) {
    const size_t lds = 0;   // traversal stacks live in private memory
    hipLaunchKernelGGL((kb_traverse_plain<ANY, STATS>), dim3(g.total_blocks), dim3(128), lds, s, jobs,
                       ids + g.first_id, g.d_block_off, g.count);
}

void launch_batch(const BatchJob *jobs, const uint32_t *ids, const std::vector<BatchGroup> &groups,
                  uint32_t max_rounds, uint32_t max_blocks, hipStream_t s) {
    for (const BatchGroup &g : groups) {
        if (g.kind == kBatchAnyPlain) {
            if (g.stats) launch_batch_plain<true, true>(jobs, ids, g, s);
            else launch_batch_plain<true, false>(jobs, ids, g, s);
        } else if (g.kind == kBatchClosestPlain) {
            if (g.stats) launch_batch_plain<false, true>(jobs, ids, g, s);
            else launch_batch_plain<false, false>(jobs, ids, g, s);
        } else if (g.block_epochs) {
            // small epochs: every epoch of every job of the group in one launch
            if (g.kind == kBatchAnyHrpp) {
                if (g.stats) launch_batch_block_epochs<true, false, true>(jobs, ids, g, s);
                else launch_batch_block_epochs<true, false, false>(jobs, ids, g, s);
            } else if (g.kind == kBatchExactHrpp) {
                if (g.stats) launch_batch_block_epochs<false, true, true>(jobs, ids, g, s);
                else launch_batch_block_epochs<false, true, false>(jobs, ids, g, s);
            } else {
                if (g.stats) launch_batch_block_epochs<false, false, true>(jobs, ids, g, s);
                else launch_batch_block_epochs<false, false, false>(jobs, ids, g, s);
            }
        }
    }
    for (uint32_t r = 0; r < max_rounds; r++) {
        for (const BatchGroup &g : groups) {
            if (r >= g.rounds) continue;
            switch (g.kind) {
                case kBatchAnyHrpp:
                    if (g.stats) launch_batch_round<true, false, true>(jobs, ids, g, r, s);
                    else launch_batch_round<true, false, false>(jobs, ids, g, r, s);
                    break;
                case kBatchPaperHrpp:
                    if (g.stats) launch_batch_round<false, false, true>(jobs, ids, g, r, s);
                    else launch_batch_round<false, false, false>(jobs, ids, g, r, s);
                    break;
                case kBatchExactHrpp:
                    if (g.stats) launch_batch_round<false, true, true>(jobs, ids, g, r, s);
                    else launch_batch_round<false, true, false>(jobs, ids, g, r, s);
                    break;
                default:
                    break;
            }
        }
    }
}

}  // namespace hrpp
