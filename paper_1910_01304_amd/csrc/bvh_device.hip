// Device BVH build of the HRPP library: a linear BVH over Morton codes.
//
// The paper takes the BVH as given ("Overview", "Limit Study").  The host
// builder (bvh_build.cpp) makes a binned-SAH tree; this file builds, entirely
// on the GPU, the binary radix tree over the triangles' Morton codes
// (Lauterbach et al. 2009; Karras, HPG 2012), for callers that must build
// scenes quickly (the serving loop takes new scenes while it runs).  The tree:
//   * centre of a triangle on axis a: (lo + hi) * 0.5 with lo / hi the min /
//     max of its vertices (the SAH builder's centre);
//   * cubic cells over the centres' bounds: one scale = 2^21 / (the largest
//     extent cmax - cmin), 0 when that extent is 0 or the quotient is not
//     finite; cell = min(floor((c - cmin) * scale), 2^21 - 1) per axis; code
//     bit 3k+2 / 3k+1 / 3k = bit k of the x / y / z cell (63 bits);
//   * triangles sorted by (code, primitive id) -- a stable radix sort;
//   * the radix tree over the keys (code, sorted position): each node splits
//     its range at the highest bit in which its first and last keys differ;
//   * a node over at most leaf_max triangles is a leaf (its subtree is
//     dropped); boxes are exact bounds; nodes numbered in DFS pre-order.
// The output is the same GPU layout hrpp_bvh_upload writes for a host tree:
// interior nodes (64 B), triangles (48 B), leaf boxes (32 B), canonical node
// records (48 B); there is no 4-wide tree.
//
// No kernel hands data to another workgroup of the same launch: every
// dependency is a kernel boundary.  In launch order:
//   k_lbvh_bounds / k_lbvh_bounds_final  centre bounds (per-block partials)
//   k_lbvh_codes, radix sort             Morton codes in (code, id) order
//                                        (device_sort.hip)
//   k_lbvh_karras                        each internal node's range and split
//   k_lbvh_mark, exclusive scan          output leaves starting before each
//                                        sorted position (device_sort.hip)
//   k_lbvh_number                        depth and DFS pre-order index
//   k_lbvh_leaf_boxes, k_lbvh_level      leaf boxes, then interior boxes one
//                                        depth at a time, deepest first
//   k_lbvh_emit                          the GPU layout
// The pre-order index of a node is closed-form: the subtrees left of it along
// its root path tile the sorted positions before its range, and a subtree of
// k leaves has 2k - 1 nodes, so index = 2 * (output leaves before its first
// position) + (ancestors it descends from on the left).
//
// Optional treelet passes (Karras and Aila, "Fast Parallel Construction of
// High-Quality Bounding Volume Hierarchies", HPG 2013) then rearrange the
// interior nodes; the output leaves stay.  Each pass runs the interior nodes
// level by level, deepest first (k_tl_depth / k_tl_bucket list the levels,
// k_tl_treelet restructures one level, a wave per node), so every node comes
// after every node below it and the nodes of one launch have disjoint
// subtrees.  A restructured tree is no longer in sorted-position order, so
// it is numbered and laid out from explicit subtree counts instead
// (k_tl_number, k_tl_emit): triangles in leaf order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "device_sort.h"
#include "hrpp_internal.h"
#include "hrpp_kernels.h"

namespace hrpp {

namespace {

constexpr uint32_t kCellMax = (1u << 21) - 1u;
constexpr uint32_t kWalkLimit = 128;   // deeper than any radix tree over 63-bit codes + 28-bit positions

// Header of the build scratch (also read back by the host).
struct LbvhHeader {
    uint32_t bad;          // bit 0: a non-finite vertex; bit 1: inconsistent numbering; bit 2: too deep
    uint32_t cmin[3];      // order-preserving images of the centre bounds
    uint32_t cmax[3];
    uint32_t max_depth;    // deepest leaf
    uint32_t num_nodes;    // nodes of the output tree
    float root_box[6];
    uint32_t pad[49];
};
static_assert(sizeof(LbvhHeader) == 256, "one 256-byte header");

// Total order of binary32 values as unsigned integers (for integer min / max
// reductions; NaN images lie outside the finite ones and are rejected).
__device__ inline uint32_t ord_of(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float float_of(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Vertex min / max of one triangle on each axis (strict comparisons, first
// vertex wins ties); the centre is (lo + hi) * 0.5.
__device__ inline void tri_bounds(const float *__restrict__ v, float lo[3], float hi[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float l = v[a], h = v[a];
        if (v[3 + a] < l) l = v[3 + a];
        if (v[6 + a] < l) l = v[6 + a];
        if (v[3 + a] > h) h = v[3 + a];
        if (v[6 + a] > h) h = v[6 + a];
        lo[a] = l;
        hi[a] = h;
    }
}

// Spread the low 21 bits of x so that bit k lands on bit 3k.
__device__ inline uint64_t spread3(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

constexpr uint32_t kBoundBlocks = 512;   // blocks of the bounds pass (partials reduced by one block)
constexpr uint32_t kRightChild = 0x80000000u;   // parent word: the node is its parent's right child

__device__ inline uint32_t wave_min(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, off, 64));
    return x;
}
__device__ inline uint32_t wave_max(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off, 64));
    return x;
}

// Block reduction of 7 words (min of words 0..2, max of words 3..6) over 256
// threads; thread 0 ends with the block's values.
__device__ inline void block_reduce7(uint32_t v[7], uint32_t (*lds)[7]) {
    for (int k = 0; k < 7; k++) v[k] = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0)
        for (int k = 0; k < 7; k++) lds[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (uint32_t q = 1; q < (blockDim.x >> 6); q++)
            for (int k = 0; k < 7; k++) v[k] = k < 3 ? min(v[k], lds[q][k]) : max(v[k], lds[q][k]);
}

// Centre bounds and the non-finite check: each block reduces a strided share
// of the triangles into partial[block] (cmin xyz, cmax xyz, bad).
__global__ __launch_bounds__(256) void k_lbvh_bounds(const float *__restrict__ verts, uint32_t n,
                                                     uint32_t *__restrict__ partial) {
    __shared__ uint32_t lds[4][7];
    uint32_t v[7] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u};
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const float *p = verts + 9 * (size_t)t;
        bool finite = true;
        for (int k = 0; k < 9; k++) finite = finite && isfinite(p[k]);
        if (!finite) v[6] = 1u;
        float lo[3], hi[3];
        tri_bounds(p, lo, hi);
        for (int a = 0; a < 3; a++) {
            const uint32_t c = ord_of((lo[a] + hi[a]) * 0.5f);
            v[a] = min(v[a], c);
            v[3 + a] = max(v[3 + a], c);
        }
    }
    block_reduce7(v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 7; k++) partial[7 * blockIdx.x + k] = v[k];
}

// One block: the partials into the header; the header's other fields start.
__global__ __launch_bounds__(256) void k_lbvh_bounds_final(const uint32_t *__restrict__ partial, uint32_t nblocks,
                                                           LbvhHeader *h, uint32_t *parent) {
    __shared__ uint32_t lds[4][7];
    uint32_t v[7] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u};
    for (uint32_t b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < 7; k++) v[k] = k < 3 ? min(v[k], partial[7 * b + k]) : max(v[k], partial[7 * b + k]);
    block_reduce7(v, lds);
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; a++) { h->cmin[a] = v[a]; h->cmax[a] = v[3 + a]; }
        h->bad = v[6];
        h->max_depth = 0;
        h->num_nodes = 0;
        parent[0] = kNone;   // node 0 is the root (internal node 0, or the only leaf)
    }
}

__global__ __launch_bounds__(256) void k_lbvh_codes(const float *__restrict__ verts, uint32_t n,
                                                    const LbvhHeader *__restrict__ h, uint64_t *__restrict__ code,
                                                    uint32_t *__restrict__ id) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float lo[3], hi[3];
    tri_bounds(verts + 9 * (size_t)t, lo, hi);
    // cubic cells: one scale, from the largest extent
    float emax = 0.0f;
    for (int a = 0; a < 3; a++) {
        const float ext = float_of(h->cmax[a]) - float_of(h->cmin[a]);
        if (ext > emax) emax = ext;
    }
    float s = emax > 0.0f ? 2097152.0f / emax : 0.0f;
    if (!isfinite(s)) s = 0.0f;
    uint64_t q[3];
    for (int a = 0; a < 3; a++) {
        const float f = floorf(((lo[a] + hi[a]) * 0.5f - float_of(h->cmin[a])) * s);
        q[a] = f >= (float)kCellMax ? kCellMax : (uint32_t)f;
    }
    code[t] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    id[t] = t;
}

// Length of the common prefix of the keys (code, position) at sorted
// positions i and j; -1 outside [0, n).
__device__ inline int prefix_len(const uint64_t *__restrict__ code, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = code[i], b = code[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// Node ids: internal node i in [0, n-1), leaf k at n - 1 + k.  Internal node
// i covers sorted positions [lo[i], hi[i]] and splits after position gamma.
__global__ __launch_bounds__(256) void k_lbvh_karras(const uint64_t *__restrict__ code, uint32_t n,
                                                     uint32_t *__restrict__ parent, uint32_t *__restrict__ left,
                                                     uint32_t *__restrict__ right, uint32_t *__restrict__ lo,
                                                     uint32_t *__restrict__ hi) {
    const uint32_t iu = blockIdx.x * blockDim.x + threadIdx.x;
    if (iu + 1 >= n) return;
    const int64_t i = iu, nn = n;
    const int d = prefix_len(code, nn, i, i + 1) > prefix_len(code, nn, i, i - 1) ? 1 : -1;
    const int dmin = prefix_len(code, nn, i, i - d);
    int64_t lmax = 2;
    while (prefix_len(code, nn, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(code, nn, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = prefix_len(code, nn, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(code, nn, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const uint32_t first = (uint32_t)(i < j ? i : j), last = (uint32_t)(i < j ? j : i);
    const uint32_t g = (uint32_t)gamma;
    const uint32_t lc = (first == g) ? (n - 1u + g) : g;
    const uint32_t rc = (last == g + 1u) ? (n - 1u + g + 1u) : g + 1u;
    left[iu] = lc;
    right[iu] = rc;
    lo[iu] = first;
    hi[iu] = last;
    parent[lc] = iu;
    parent[rc] = iu | kRightChild;
}

struct Tree {
    uint32_t n, leaf_max;
    const uint32_t *parent, *left, *right, *lo, *hi;
    __device__ uint32_t up(uint32_t v) const { return parent[v] & ~kRightChild; }
    __device__ uint32_t first(uint32_t v) const { return v + 1u < n ? lo[v] : v - (n - 1u); }
    __device__ uint32_t size(uint32_t v) const { return v + 1u < n ? hi[v] - lo[v] + 1u : 1u; }
    __device__ bool out_interior(uint32_t v) const { return v + 1u < n && size(v) > leaf_max; }
    __device__ bool out_leaf(uint32_t v) const { return size(v) <= leaf_max && (v == 0 || size(up(v)) > leaf_max); }
};

// mark[k] = 1 when sorted position k is the first of an output leaf (the
// leaf holding k is found by climbing while the parent is small enough to be
// a leaf itself: at most leaf_max - 1 <= 7 steps, since a subtree of at most
// leaf_max leaves is at most that tall); mark[n] = 0.
__global__ __launch_bounds__(256) void k_lbvh_mark(Tree tr, uint32_t *__restrict__ mark) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > tr.n) return;
    if (k == tr.n) { mark[k] = 0u; return; }
    uint32_t v = tr.n - 1u + k;
    for (uint32_t step = 0; v != 0 && step < 8 && tr.size(tr.up(v)) <= tr.leaf_max; step++) v = tr.up(v);
    mark[k] = tr.first(v) == k ? 1u : 0u;
}

// Depth and pre-order index of every output node (dep = kNone for dropped
// nodes; bit 31 of dep set for leaves).  lb[k] = output leaves starting
// before position k.
__global__ __launch_bounds__(256) void k_lbvh_number(Tree tr, const uint32_t *__restrict__ lb,
                                                     uint32_t *__restrict__ pre, uint32_t *__restrict__ dep,
                                                     LbvhHeader *h) {
    __shared__ uint32_t lds[4][7];
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t deepest[7] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u};
    if (v < 2u * tr.n - 1u) {
        const bool leaf = tr.out_leaf(v);
        if (leaf || tr.out_interior(v)) {
            uint32_t depth = 0, lefts = 0, cur = v;
            while (cur != 0 && depth < kWalkLimit) {
                const uint32_t w = tr.parent[cur];
                lefts += (w & kRightChild) ? 0u : 1u;
                depth += 1u;
                cur = w & ~kRightChild;
            }
            if (cur != 0) atomicOr(&h->bad, 4u);
            pre[v] = 2u * lb[tr.first(v)] + lefts;
            dep[v] = depth | (leaf ? 0x80000000u : 0u);
            if (leaf) deepest[6] = depth;
        } else {
            dep[v] = kNone;
        }
    }
    if (v == 0) h->num_nodes = 2u * lb[tr.n] - 1u;
    block_reduce7(deepest, lds);
    if (threadIdx.x == 0 && deepest[6]) atomicMax(&h->max_depth, deepest[6]);
}

// Boxes keep the first minimum / maximum in triangle order, as a sequential
// scan would (a union keeps the left child's value on ties).
__global__ __launch_bounds__(256) void k_lbvh_leaf_boxes(Tree tr, const float *__restrict__ verts,
                                                         const uint32_t *__restrict__ perm,
                                                         const uint32_t *__restrict__ dep, float *__restrict__ box) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 2u * tr.n - 1u) return;
    const uint32_t d = dep[v];
    if (d == kNone || !(d & 0x80000000u)) return;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const uint32_t f = tr.first(v), c = tr.size(v);
    for (uint32_t k = f; k < f + c; k++) {
        const float *p = verts + 9 * (size_t)perm[k];
        for (int q = 0; q < 3; q++)
            for (int a = 0; a < 3; a++) {
                const float x = p[3 * q + a];
                if (x < mn[a]) mn[a] = x;
                if (x > mx[a]) mx[a] = x;
            }
    }
    for (int a = 0; a < 3; a++) { box[6 * (size_t)v + a] = mn[a]; box[6 * (size_t)v + 3 + a] = mx[a]; }
}

// Interior nodes at one depth: the union of their children's boxes (written
// by an earlier launch).
__global__ __launch_bounds__(256) void k_lbvh_level(Tree tr, const uint32_t *__restrict__ dep, uint32_t level,
                                                    float *__restrict__ box) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v + 1u >= tr.n || dep[v] != level) return;
    const float *bl = box + 6 * (size_t)tr.left[v], *br = box + 6 * (size_t)tr.right[v];
    float out[6];
    for (int a = 0; a < 3; a++) {
        out[a] = br[a] < bl[a] ? br[a] : bl[a];
        out[3 + a] = br[3 + a] > bl[3 + a] ? br[3 + a] : bl[3 + a];
    }
    for (int a = 0; a < 6; a++) box[6 * (size_t)v + a] = out[a];
}

struct EmitOut {
    float *nodes;       // 16 words per interior node
    float *tris;        // 12 words per triangle
    float *leafbox;     // 8 words per triangle position
    uint32_t *cnode;    // 12 words per node
    uint32_t node_cap;  // 2n - 1
    uint32_t interior_cap;
};

// Reference of an output node: a leaf id, or the interior node's index among
// interior nodes in pre-order (its pre-order index minus the leaves before it).
__device__ inline uint32_t ref_of(const Tree &tr, const uint32_t *pre, const uint32_t *lb, uint32_t v) {
    if (tr.out_leaf(v)) return kLeafFlag | (tr.first(v) << 3) | (tr.size(v) - 1u);
    return pre[v] - lb[tr.first(v)];
}

__global__ __launch_bounds__(256) void k_lbvh_emit(Tree tr, const float *__restrict__ verts,
                                                   const uint32_t *__restrict__ perm, const float *__restrict__ box,
                                                   const uint32_t *__restrict__ pre, const uint32_t *__restrict__ lb,
                                                   const uint32_t *__restrict__ dep, EmitOut o, LbvhHeader *h) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 2u * tr.n - 1u) return;
    const uint32_t dw = dep[v];
    if (dw == kNone) return;
    const bool leaf = (dw & 0x80000000u) != 0;
    const uint32_t depth = dw & 0x7FFFFFFFu;
    const uint32_t i = pre[v];
    const uint32_t f = tr.first(v), c = tr.size(v);
    if (i >= o.node_cap || f + c > tr.n) { atomicOr(&h->bad, 2u); return; }
    const float *b = box + 6 * (size_t)v;
    uint32_t *cn = o.cnode + 12 * (size_t)i;
    for (int a = 0; a < 6; a++) cn[a] = __float_as_uint(b[a]);
    cn[6] = ref_of(tr, pre, lb, v);
    cn[7] = depth;
    cn[8] = v == 0 ? kNone : pre[tr.up(v)];
    cn[9] = f;
    cn[10] = f + c;
    cn[11] = 0u;
    if (v == 0)
        for (int a = 0; a < 6; a++) h->root_box[a] = b[a];
    if (!leaf) {
        const uint32_t iid = pre[v] - lb[f];
        if (iid >= o.interior_cap) { atomicOr(&h->bad, 2u); return; }
        const uint32_t l = tr.left[v], r = tr.right[v];
        float *nd = o.nodes + 16 * (size_t)iid;
        for (int a = 0; a < 6; a++) { nd[a] = box[6 * (size_t)l + a]; nd[6 + a] = box[6 * (size_t)r + a]; }
        nd[12] = __uint_as_float(ref_of(tr, pre, lb, l));
        nd[13] = __uint_as_float(ref_of(tr, pre, lb, r));
        nd[14] = 0.0f;
        nd[15] = 0.0f;
        return;
    }
    float *lbx = o.leafbox + 8 * (size_t)f;
    for (int a = 0; a < 6; a++) lbx[a] = b[a];
    lbx[6] = __uint_as_float(depth);
    lbx[7] = __uint_as_float(i);
    for (uint32_t k = f; k < f + c; k++) {
        const uint32_t prim = perm[k];
        const float *p = verts + 9 * (size_t)prim;
        float *t = o.tris + 12 * (size_t)k;
        t[0] = p[0]; t[1] = p[1]; t[2] = p[2];
        t[3] = __uint_as_float(prim);
        t[4] = p[3] - p[0]; t[5] = p[4] - p[1]; t[6] = p[5] - p[2];
        t[7] = __uint_as_float(depth);
        t[8] = p[6] - p[0]; t[9] = p[7] - p[1]; t[10] = p[8] - p[2];
        t[11] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Treelet restructuring.  Node identities stay those of the radix tree
// (interior nodes in [0, n-1), output leaves wherever the radix tree had
// them); a restructured interior node's lo / hi no longer describe its
// subtree, so its triangle count (cnt) and output-leaf count (atoms) are kept
// explicitly.  The rules -- treelet growth, cost, tie-breaking, which
// identity each new interior node takes -- are those the plain C reading of
// the method states; only the schedule (levels, a wave per treelet) is this
// file's.
// ---------------------------------------------------------------------------
constexpr uint32_t kTlLeaves = 7;            // leaves of a treelet
constexpr uint32_t kTlLevels = kWalkLimit;   // node depths are below the walk limit
constexpr uint32_t kTlThreads = 64;          // one wave per treelet

struct TlTree {
    uint32_t *parent, *left, *right, *dep, *cnt, *atoms;
    float *box;
    uint32_t *bad;                           // header word: bit 1 on an inconsistent treelet
};

__device__ inline bool tl_is_leaf(const uint32_t *dep, uint32_t v) { return (dep[v] & 0x80000000u) != 0; }

// Half surface area in binary32, summed left to right.
__device__ inline float tl_half_area(const float *b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

// Subtree counts of the linear BVH's output nodes.
__global__ __launch_bounds__(256) void k_tl_init(Tree tr, const uint32_t *__restrict__ lb,
                                                 const uint32_t *__restrict__ dep, uint32_t *__restrict__ cnt,
                                                 uint32_t *__restrict__ atoms) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 2u * tr.n - 1u) return;
    const uint32_t d = dep[v];
    if (d == kNone) return;
    const uint32_t f = tr.first(v), c = tr.size(v);
    cnt[v] = c;
    atoms[v] = (d & 0x80000000u) ? 1u : lb[f + c] - lb[f];
}

// Level counts and the deepest leaf start from zero.
__global__ __launch_bounds__(kTlLevels) void k_tl_zero(uint32_t *__restrict__ levels, LbvhHeader *h) {
    levels[threadIdx.x] = 0u;
    if (threadIdx.x == 0) h->max_depth = 0u;
}

// Depth of every output node (leaf flag kept), the deepest leaf, and the
// number of interior nodes at each depth.
__global__ __launch_bounds__(256) void k_tl_depth(const uint32_t *__restrict__ parent, uint32_t *__restrict__ dep,
                                                  uint32_t m, uint32_t *__restrict__ hist, LbvhHeader *h) {
    __shared__ uint32_t lh[kTlLevels];
    for (uint32_t k = threadIdx.x; k < kTlLevels; k += blockDim.x) lh[k] = 0u;
    __syncthreads();
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t leaf_depth = 0;
    if (v < m && dep[v] != kNone) {
        const uint32_t flag = dep[v] & 0x80000000u;
        uint32_t depth = 0, cur = v;
        while (cur != 0 && depth < kWalkLimit) {
            cur = parent[cur] & ~kRightChild;
            depth++;
        }
        if (cur != 0) {
            atomicOr(&h->bad, 4u);
        } else {
            dep[v] = depth | flag;
            if (flag) leaf_depth = depth;
            else atomicAdd(&lh[depth], 1u);
        }
    }
    leaf_depth = wave_max(leaf_depth);
    if ((threadIdx.x & 63u) == 0 && leaf_depth) atomicMax(&h->max_depth, leaf_depth);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kTlLevels; k += blockDim.x)
        if (lh[k]) atomicAdd(&hist[k], lh[k]);
}

// Start of each level's list (exclusive prefix of the counts); fill counters
// start from zero.
__global__ __launch_bounds__(64) void k_tl_start(const uint32_t *__restrict__ hist, uint32_t *__restrict__ start,
                                                 uint32_t *__restrict__ fill) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (uint32_t k = 0; k < kTlLevels; k++) {
        start[k] = run;
        fill[k] = 0u;
        run += hist[k];
    }
}

// Interior nodes listed by level (in any order within a level): a block
// counts its nodes per level in LDS and reserves each level's range once.
__global__ __launch_bounds__(256) void k_tl_bucket(const uint32_t *__restrict__ dep, uint32_t n_internal,
                                                   const uint32_t *__restrict__ start, uint32_t *__restrict__ fill,
                                                   uint32_t *__restrict__ list) {
    __shared__ uint32_t lc[kTlLevels], lbase[kTlLevels];
    for (uint32_t k = threadIdx.x; k < kTlLevels; k += blockDim.x) lc[k] = 0u;
    __syncthreads();
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t d = kNone, loc = 0;
    if (v < n_internal && dep[v] != kNone && !(dep[v] & 0x80000000u)) {
        d = dep[v];
        loc = atomicAdd(&lc[d], 1u);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kTlLevels; k += blockDim.x)
        if (lc[k]) lbase[k] = atomicAdd(&fill[k], lc[k]);
    __syncthreads();
    if (d != kNone) list[start[d] + lbase[d] + loc] = v;
}

// One treelet per wave: grow it, find the best topology over its leaves by
// dynamic programming over subsets (lanes take the subsets of one size at a
// time), and rebuild it when that beats the current topology.
__global__ __launch_bounds__(kTlThreads) void k_tl_treelet(TlTree t, const uint32_t *__restrict__ list) {
    constexpr uint32_t kSub = 1u << kTlLeaves;
    __shared__ float s_area[kSub], s_cost[kSub];
    __shared__ uint32_t s_bestp[kSub], s_id[kSub];
    __shared__ float s_box[kTlLeaves][6];
    __shared__ uint32_t s_L[kTlLeaves], s_I[kTlLeaves - 1], s_nl, s_ni;
    const uint32_t lane = threadIdx.x;
    const uint32_t r = list[blockIdx.x];
    if (lane == 0) {
        // grow: open the treelet leaf of largest area among the interior ones
        // (the first on ties); its left child takes its place, its right
        // child goes to the end
        uint32_t nl = 2, ni = 1;
        s_L[0] = t.left[r];
        s_L[1] = t.right[r];
        s_I[0] = r;
        while (nl < kTlLeaves) {
            int best = -1;
            float ba = 0.0f;
            for (uint32_t i = 0; i < nl; i++) {
                const uint32_t x = s_L[i];
                if (tl_is_leaf(t.dep, x)) continue;
                const float a = tl_half_area(t.box + 6 * (size_t)x);
                if (best < 0 || a > ba) { best = (int)i; ba = a; }
            }
            if (best < 0) break;
            const uint32_t x = s_L[best];
            s_I[ni++] = x;
            s_L[best] = t.left[x];
            s_L[nl++] = t.right[x];
        }
        for (uint32_t i = 0; i < nl; i++)
            for (int a = 0; a < 6; a++) s_box[i][a] = t.box[6 * (size_t)s_L[i] + a];
        s_nl = nl;
        s_ni = ni;
    }
    __syncthreads();
    const uint32_t nl = s_nl, ni = s_ni;
    if (nl < 3) return;                        // two leaves: one topology (uniform)
    const uint32_t full = (1u << nl) - 1u;
    // the union box of every subset, members in increasing order (a union
    // keeps the earlier value on ties), and its half area
    for (uint32_t S = lane + 1u; S <= full; S += kTlThreads) {
        float u[6];
        bool have = false;
        for (uint32_t i = 0; i < nl; i++) {
            if (!((S >> i) & 1u)) continue;
            if (!have) {
                for (int a = 0; a < 6; a++) u[a] = s_box[i][a];
                have = true;
            } else {
                for (int a = 0; a < 3; a++) {
                    u[a] = s_box[i][a] < u[a] ? s_box[i][a] : u[a];
                    u[3 + a] = s_box[i][3 + a] > u[3 + a] ? s_box[i][3 + a] : u[3 + a];
                }
            }
        }
        s_area[S] = tl_half_area(u);
        s_cost[S] = 0.0f;
        s_bestp[S] = 0u;
    }
    __syncthreads();
    // c(S) = A(S) + min over P (c(P) + c(S \ P)), P over the proper subsets
    // of S holding its lowest member in increasing order, the first minimum
    // kept; subsets of one size depend only on smaller ones
    for (uint32_t sz = 2; sz <= nl; sz++) {
        for (uint32_t S = lane + 1u; S <= full; S += kTlThreads) {
            if ((uint32_t)__popc(S) != sz) continue;
            const uint32_t low = S & (0u - S);
            float best = 0.0f;
            uint32_t bp = 0;
            for (uint32_t P = low; P != S; P = (P - S) & S) {   // the subsets of S, increasing
                if (!(P & low)) continue;
                const float c = s_cost[P] + s_cost[S ^ P];
                if (bp == 0 || c < best) { best = c; bp = P; }
            }
            s_cost[S] = s_area[S] + best;
            s_bestp[S] = bp;
        }
        __syncthreads();
    }
    if (lane != 0) return;
    // the current topology's cost by the same recurrence: an opened node's
    // children were opened later, so a reverse sweep meets children first
    uint32_t mask[kTlLeaves - 1];
    float cur[kTlLeaves - 1];
    for (int j = (int)ni - 1; j >= 0; j--) {
        const uint32_t x = s_I[j];
        const uint32_t ch[2] = {t.left[x], t.right[x]};
        uint32_t m2[2];
        float c2[2];
        for (int k = 0; k < 2; k++) {
            m2[k] = 0u;
            c2[k] = 0.0f;
            for (uint32_t i = 0; i < nl; i++)
                if (s_L[i] == ch[k]) m2[k] = 1u << i;
            for (uint32_t q = (uint32_t)j + 1u; q < ni; q++)
                if (s_I[q] == ch[k]) { m2[k] = mask[q]; c2[k] = cur[q]; }
        }
        mask[j] = m2[0] | m2[1];
        if (mask[j] == 0u || mask[j] > full) { atomicOr(t.bad, 2u); return; }
        cur[j] = s_area[mask[j]] + (c2[0] + c2[1]);
    }
    if (!(s_cost[full] < cur[0])) return;
    // rebuild: identities in depth-first pre-order (r, then the opened nodes
    // in opening order), the part with the lowest member on the left
    uint32_t order[kTlLeaves - 1], stack[kTlLeaves];
    uint32_t sp = 0, no = 0, next = 1;
    stack[sp++] = full;
    while (sp) {
        const uint32_t S = stack[--sp];
        const uint32_t P = s_bestp[S], Q = S ^ P;
        if (P == 0u || (P & ~S) != 0u || P == S || no >= nl - 1u || (S != full && next >= ni)) {
            atomicOr(t.bad, 2u);
            return;
        }
        s_id[S] = S == full ? r : s_I[next++];
        order[no++] = S;
        if (__popc(Q) > 1) stack[sp++] = Q;
        if (__popc(P) > 1) stack[sp++] = P;
    }
    // children before parents: links, boxes (union, the left child's value
    // kept on ties) and counts
    for (int k = (int)no - 1; k >= 0; k--) {
        const uint32_t S = order[k], P = s_bestp[S], Q = S ^ P;
        const uint32_t id = s_id[S];
        const uint32_t l = __popc(P) == 1 ? s_L[__ffs(P) - 1] : s_id[P];
        const uint32_t rr = __popc(Q) == 1 ? s_L[__ffs(Q) - 1] : s_id[Q];
        t.left[id] = l;
        t.right[id] = rr;
        t.parent[l] = id;
        t.parent[rr] = id | kRightChild;
        const float *bl = t.box + 6 * (size_t)l, *br = t.box + 6 * (size_t)rr;
        float out[6];
        for (int a = 0; a < 3; a++) {
            out[a] = br[a] < bl[a] ? br[a] : bl[a];
            out[3 + a] = br[3 + a] > bl[3 + a] ? br[3 + a] : bl[3 + a];
        }
        for (int a = 0; a < 6; a++) t.box[6 * (size_t)id + a] = out[a];
        t.cnt[id] = t.cnt[l] + t.cnt[rr];
        t.atoms[id] = t.atoms[l] + t.atoms[rr];
    }
}

// Pre-order index, first triangle position and interior index of every
// output node of the restructured tree, from its root path: a step up from a
// right child passes the left sibling's subtree (2a - 1 nodes of which a - 1
// interior, and its triangles), and every step passes the parent.
__global__ __launch_bounds__(256) void k_tl_number(TlTree t, uint32_t m, uint32_t *__restrict__ pre,
                                                   uint32_t *__restrict__ off, uint32_t *__restrict__ iref,
                                                   LbvhHeader *h) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m || t.dep[v] == kNone) return;
    uint32_t p = 0, o = 0, ir = 0, cur = v, steps = 0;
    while (cur != 0 && steps < kWalkLimit) {
        const uint32_t w = t.parent[cur], u = w & ~kRightChild;
        if (w & kRightChild) {
            const uint32_t l = t.left[u];
            p += 2u * t.atoms[l];
            ir += t.atoms[l];
            o += t.cnt[l];
        } else {
            p += 1u;
            ir += 1u;
        }
        cur = u;
        steps++;
    }
    if (cur != 0) { atomicOr(&h->bad, 4u); return; }
    pre[v] = p;
    off[v] = o;
    iref[v] = ir;
    if (v == 0) h->num_nodes = 2u * t.atoms[0] - 1u;
}

__device__ inline uint32_t tl_ref_of(const TlTree &t, const uint32_t *off, const uint32_t *iref, uint32_t v) {
    if (tl_is_leaf(t.dep, v)) return kLeafFlag | (off[v] << 3) | (t.cnt[v] - 1u);
    return iref[v];
}

// The GPU layout of the restructured tree (the same records as k_lbvh_emit).
__global__ __launch_bounds__(256) void k_tl_emit(Tree tr, TlTree t, const float *__restrict__ verts,
                                                 const uint32_t *__restrict__ perm, const uint32_t *__restrict__ pre,
                                                 const uint32_t *__restrict__ off, const uint32_t *__restrict__ iref,
                                                 EmitOut o, LbvhHeader *h) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 2u * tr.n - 1u) return;
    const uint32_t dw = t.dep[v];
    if (dw == kNone) return;
    const bool leaf = (dw & 0x80000000u) != 0;
    const uint32_t depth = dw & 0x7FFFFFFFu;
    const uint32_t i = pre[v], fo = off[v], c = t.cnt[v];
    if (i >= o.node_cap || c == 0u || fo + c > tr.n || (leaf && c > 8u)) { atomicOr(&h->bad, 2u); return; }
    const float *b = t.box + 6 * (size_t)v;
    uint32_t *cn = o.cnode + 12 * (size_t)i;
    for (int a = 0; a < 6; a++) cn[a] = __float_as_uint(b[a]);
    cn[6] = tl_ref_of(t, off, iref, v);
    cn[7] = depth;
    cn[8] = v == 0 ? kNone : pre[t.parent[v] & ~kRightChild];
    cn[9] = fo;
    cn[10] = fo + c;
    cn[11] = 0u;
    if (v == 0)
        for (int a = 0; a < 6; a++) h->root_box[a] = b[a];
    if (!leaf) {
        const uint32_t iid = iref[v];
        if (iid >= o.interior_cap) { atomicOr(&h->bad, 2u); return; }
        const uint32_t l = t.left[v], r = t.right[v];
        float *nd = o.nodes + 16 * (size_t)iid;
        for (int a = 0; a < 6; a++) { nd[a] = t.box[6 * (size_t)l + a]; nd[6 + a] = t.box[6 * (size_t)r + a]; }
        nd[12] = __uint_as_float(tl_ref_of(t, off, iref, l));
        nd[13] = __uint_as_float(tl_ref_of(t, off, iref, r));
        nd[14] = 0.0f;
        nd[15] = 0.0f;
        return;
    }
    // a leaf keeps the linear BVH's triangles, now at its own position
    float *lbx = o.leafbox + 8 * (size_t)fo;
    for (int a = 0; a < 6; a++) lbx[a] = b[a];
    lbx[6] = __uint_as_float(depth);
    lbx[7] = __uint_as_float(i);
    const uint32_t f = tr.first(v);
    for (uint32_t k = 0; k < c; k++) {
        const uint32_t prim = perm[f + k];
        const float *p = verts + 9 * (size_t)prim;
        float *tt = o.tris + 12 * (size_t)(fo + k);
        tt[0] = p[0]; tt[1] = p[1]; tt[2] = p[2];
        tt[3] = __uint_as_float(prim);
        tt[4] = p[3] - p[0]; tt[5] = p[4] - p[1]; tt[6] = p[5] - p[2];
        tt[7] = __uint_as_float(depth);
        tt[8] = p[6] - p[0]; tt[9] = p[7] - p[1]; tt[10] = p[8] - p[2];
        tt[11] = 0.0f;
    }
}

struct ScratchLayout {
    size_t hdr, partial, code_a, code_b, id_a, id_b, sort_tmp, scan_tmp, parent, left, right, lo, hi, mark, lb, pre,
        dep, box, cnt, atoms, off, iref, tl_list, tl_levels, total;
};

ScratchLayout scratch_layout(uint32_t n) {
    ScratchLayout L{};
    const size_t N = n, M = 2 * (size_t)n - 1, I = n > 1 ? (size_t)n - 1 : 1;
    size_t off = 0;
    L.hdr = off; off += 256;
    L.partial = off; off += align256((size_t)kBoundBlocks * 7 * 4);
    L.code_a = off; off += align256(N * 8);      // codes and ids, then the sort's two buffers
    L.code_b = off; off += align256(N * 8);
    L.id_a = off; off += align256(N * 4);
    L.id_b = off; off += align256(N * 4);
    L.sort_tmp = off; off += align256(radix_sort_scratch_bytes(n));
    L.scan_tmp = off; off += align256(exclusive_scan_scratch_bytes(n + 1));
    L.parent = off; off += align256(M * 4);
    L.left = off; off += align256(I * 4);
    L.right = off; off += align256(I * 4);
    L.lo = off; off += align256(I * 4);
    L.hi = off; off += align256(I * 4);
    L.mark = off; off += align256((N + 1) * 4);
    L.lb = off; off += align256((N + 1) * 4);
    L.pre = off; off += align256(M * 4);
    L.dep = off; off += align256(M * 4);
    L.box = off; off += align256(M * 24);
    L.cnt = off; off += align256(M * 4);         // treelet passes: triangles and output leaves per subtree,
    L.atoms = off; off += align256(M * 4);       // and the restructured tree's numbering
    L.off = off; off += align256(M * 4);
    L.iref = off; off += align256(M * 4);
    L.tl_list = off; off += align256(I * 4);     // interior nodes grouped by level
    L.tl_levels = off; off += align256(3 * kTlLevels * 4);   // per level: count, start, fill
    L.total = off;
    return L;
}

inline dim3 grid_for(size_t n, uint32_t block) { return dim3((uint32_t)((n + block - 1) / block)); }

}  // namespace

size_t lbvh_scratch_bytes(uint32_t n) { return n ? scratch_layout(n).total : 0; }

// Build scratch of the entry point that allocates nothing: a file-scope
// device array, one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kStaticBuildScratchBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxStaticDevices] = {};
}  // namespace

hipError_t lbvh_static_scratch(void **ptr) {
    *ptr = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return hipErrorInvalidSymbol;
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    return hipSuccess;
}

hipError_t lbvh_build(const float *d_verts, uint32_t n, uint32_t leaf_max, uint32_t max_depth, uint32_t passes,
                      void *d_scratch, const LbvhOut &out, hipStream_t s, LbvhResult *res) {
    const ScratchLayout L = scratch_layout(n);
    if (L.total == 0) return hipErrorInvalidValue;
    char *base = static_cast<char *>(d_scratch);
    auto *h = reinterpret_cast<LbvhHeader *>(base + L.hdr);
    auto *partial = reinterpret_cast<uint32_t *>(base + L.partial);
    auto *code_a = reinterpret_cast<uint64_t *>(base + L.code_a);
    auto *code_b = reinterpret_cast<uint64_t *>(base + L.code_b);
    auto *id_a = reinterpret_cast<uint32_t *>(base + L.id_a);
    auto *id_b = reinterpret_cast<uint32_t *>(base + L.id_b);
    auto *parent = reinterpret_cast<uint32_t *>(base + L.parent);
    auto *left = reinterpret_cast<uint32_t *>(base + L.left);
    auto *right = reinterpret_cast<uint32_t *>(base + L.right);
    auto *lo = reinterpret_cast<uint32_t *>(base + L.lo);
    auto *hi = reinterpret_cast<uint32_t *>(base + L.hi);
    auto *mark = reinterpret_cast<uint32_t *>(base + L.mark);
    auto *lb = reinterpret_cast<uint32_t *>(base + L.lb);
    auto *pre = reinterpret_cast<uint32_t *>(base + L.pre);
    auto *dep = reinterpret_cast<uint32_t *>(base + L.dep);
    auto *box = reinterpret_cast<float *>(base + L.box);
    auto *cnt = reinterpret_cast<uint32_t *>(base + L.cnt);
    auto *atoms = reinterpret_cast<uint32_t *>(base + L.atoms);
    auto *offs = reinterpret_cast<uint32_t *>(base + L.off);
    auto *iref = reinterpret_cast<uint32_t *>(base + L.iref);
    auto *tl_list = reinterpret_cast<uint32_t *>(base + L.tl_list);
    auto *tl_hist = reinterpret_cast<uint32_t *>(base + L.tl_levels);
    uint32_t *tl_start = tl_hist + kTlLevels, *tl_fill = tl_hist + 2 * kTlLevels;
    const uint32_t n_internal = n - 1u;
    const size_t m = 2 * (size_t)n - 1;
    const uint32_t bound_blocks = (uint32_t)std::min<size_t>(kBoundBlocks, (n + 255) / 256);

    hipError_t e = hipMemsetAsync(out.leafbox, 0, (size_t)n * kLeafBoxBytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lbvh_bounds, dim3(bound_blocks), dim3(256), 0, s, d_verts, n, partial);
    hipLaunchKernelGGL(k_lbvh_bounds_final, dim3(1), dim3(256), 0, s, partial, bound_blocks, h, parent);
    hipLaunchKernelGGL(k_lbvh_codes, grid_for(n, 256), dim3(256), 0, s, d_verts, n, h, code_a, id_a);
    uint32_t sorted_in = 0;
    e = radix_sort_pairs(code_a, id_a, code_b, id_b, n, 63, base + L.sort_tmp, s, &sorted_in);
    if (e != hipSuccess) return e;
    const uint64_t *code_out = sorted_in ? code_b : code_a;   // codes in (code, id) order
    const uint32_t *perm = sorted_in ? id_b : id_a;            // their primitive ids
    if (n_internal)
        hipLaunchKernelGGL(k_lbvh_karras, grid_for(n_internal, 256), dim3(256), 0, s, code_out, n, parent, left,
                           right, lo, hi);
    Tree tr{n, leaf_max, parent, left, right, lo, hi};
    hipLaunchKernelGGL(k_lbvh_mark, grid_for((size_t)n + 1, 256), dim3(256), 0, s, tr, mark);
    e = exclusive_scan_u32(mark, lb, n + 1, base + L.scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lbvh_number, grid_for(m, 256), dim3(256), 0, s, tr, lb, pre, dep, h);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the depth decides how many interior levels follow
    LbvhHeader hh;
    e = hipMemcpyAsync(&hh, h, sizeof hh, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    res->bad = hh.bad;
    res->max_depth = hh.max_depth;
    res->num_nodes = hh.num_nodes;
    // with treelet passes the depth that counts is the restructured tree's
    if (hh.bad || (!passes && hh.max_depth > max_depth) || hh.num_nodes == 0 || hh.num_nodes > m) return hipSuccess;
    hipLaunchKernelGGL(k_lbvh_leaf_boxes, grid_for(m, 256), dim3(256), 0, s, tr, d_verts, perm, dep, box);
    for (uint32_t level = hh.max_depth; level-- > 0;)
        hipLaunchKernelGGL(k_lbvh_level, grid_for(n_internal ? n_internal : 1, 256), dim3(256), 0, s, tr, dep,
                           level, box);
    EmitOut o{static_cast<float *>(out.nodes), static_cast<float *>(out.tris), static_cast<float *>(out.leafbox),
              static_cast<uint32_t *>(out.cnode), (uint32_t)m, n_internal ? n_internal : 1u};
    if (passes == 0) {
        hipLaunchKernelGGL(k_lbvh_emit, grid_for(m, 256), dim3(256), 0, s, tr, d_verts, perm, box, pre, lb, dep, o, h);
    } else {
        TlTree t{parent, left, right, dep, cnt, atoms, box, &h->bad};
        hipLaunchKernelGGL(k_tl_init, grid_for(m, 256), dim3(256), 0, s, tr, lb, dep, cnt, atoms);
        uint32_t hist[kTlLevels];
        // depths and level sizes of the current tree (one synchronisation)
        auto levels = [&]() -> hipError_t {
            hipLaunchKernelGGL(k_tl_zero, dim3(1), dim3(kTlLevels), 0, s, tl_hist, h);
            hipLaunchKernelGGL(k_tl_depth, grid_for(m, 256), dim3(256), 0, s, parent, dep, (uint32_t)m, tl_hist, h);
            hipError_t e2 = hipMemcpyAsync(hist, tl_hist, sizeof hist, hipMemcpyDeviceToHost, s);
            if (e2 == hipSuccess) e2 = hipMemcpyAsync(&hh, h, sizeof hh, hipMemcpyDeviceToHost, s);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
            return e2;
        };
        for (uint32_t p = 0; p < passes && n_internal > 1; p++) {
            e = levels();
            if (e != hipSuccess) return e;
            if (hh.bad) { res->bad = hh.bad; return hipSuccess; }
            uint32_t start[kTlLevels], run = 0;
            for (uint32_t k = 0; k < kTlLevels; k++) { start[k] = run; run += hist[k]; }
            if (run != (hh.num_nodes - 1u) / 2u) { res->bad = 2u; return hipSuccess; }
            hipLaunchKernelGGL(k_tl_start, dim3(1), dim3(64), 0, s, tl_hist, tl_start, tl_fill);
            hipLaunchKernelGGL(k_tl_bucket, grid_for(n_internal, 256), dim3(256), 0, s, dep, n_internal, tl_start,
                               tl_fill, tl_list);
            for (uint32_t level = kTlLevels; level-- > 0;)
                if (hist[level])
                    hipLaunchKernelGGL(k_tl_treelet, dim3(hist[level]), dim3(kTlThreads), 0, s, t,
                                       tl_list + start[level]);
        }
        e = levels();
        if (e != hipSuccess) return e;
        res->bad = hh.bad;
        res->max_depth = hh.max_depth;
        if (hh.bad || hh.max_depth > max_depth) return hipSuccess;
        hipLaunchKernelGGL(k_tl_number, grid_for(m, 256), dim3(256), 0, s, t, (uint32_t)m, pre, offs, iref, h);
        hipLaunchKernelGGL(k_tl_emit, grid_for(m, 256), dim3(256), 0, s, tr, t, d_verts, perm, pre, offs, iref, o, h);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&hh, h, sizeof hh, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    res->bad = hh.bad;
    for (int a = 0; a < 6; a++) res->root_box[a] = hh.root_box[a];
    return hipSuccess;
}

}  // namespace hrpp
