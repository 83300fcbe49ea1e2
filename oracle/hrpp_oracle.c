/*
 * hrpp_oracle.c -- TEST INFRASTRUCTURE ONLY (not part of the product).
 *
 * A plain, slow, sequential-per-ray CPU model of Hash-Based Ray Path
 * Prediction (HRPP; Demoullin, Gubran and Aamodt, "Hash-Based Ray Path
 * Prediction: Skipping BVH Traversal Computation by Exploiting Ray
 * Locality").  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file.  It shares no code, header or
 * constant table with the GPU library; the two meet only through the
 * seeded inputs and the canonical BVH export.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * Every floating-point operation below is a single IEEE-754 binary32
 * operation, rounded to nearest-even, with no contraction and no
 * flush-to-zero, in the order written.
 *
 * What the paper fixes and what is our reading is stated at each function.
 * Sections cited: "Overview" (HRPP direct flow), "Precision and Recall"
 * (true/false positives, re-adding failed rays to the ray pool),
 * "HRPP Hash Function" (conflict insertion without duplicates), "Limit
 * Study" (separate hit-any / hit-all predictors, no replacement policy).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define NONE32 0xFFFFFFFFu
#define EMPTY_TAG 0xFFFFFFFFFFFFFFFFull

/* Counter slots (all uint64).  The order is part of the oracle's interface. */
enum {
    S_RAYS, S_INVALID, S_HITS, S_LOOKUPS, S_POSITIVES, S_PRED_HITS, S_FALSE_POS,
    S_TRAVERSALS, S_NODES_VISITED, S_INTERIOR_VISITED, S_LEAF_VISITED, S_BOX_TESTS,
    S_TRI_TESTS, S_NODES_SKIPPED, S_RECORDS, S_TAG_CLAIMS, S_LEAF_INSERTS, S_DROPPED,
    S_CONFLICTS, S_PRED_LEAF_VISITED, S_PRED_TRI_TESTS, S_PRED_BOX_TESTS, S_EVICTIONS, S_COUNT
};
#define STATS_SLOTS 24

/* ------------------------------------------------------------------------ */
/* Scalar helpers: IEEE minNum / maxNum (a NaN operand is ignored).          */
/* ------------------------------------------------------------------------ */
static float min_num(float a, float b)
{
    if (a != a) return b;
    if (b != b) return a;
    return (b < a) ? b : a;
}
static float max_num(float a, float b)
{
    if (a != a) return b;
    if (b != b) return a;
    return (b > a) ? b : a;
}
static float bits_to_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t float_to_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* ------------------------------------------------------------------------ */
/* Canonical BVH (the layout both builders export).                          */
/* Nodes in depth-first pre-order; an interior node's left child is the     */
/* next node, its right child is right[i]; a leaf has right[i] = NONE32 and  */
/* owns triangles [first[i], first[i]+count[i]) of the BVH-ordered array.    */
/* depth[i] = number of interior ancestors.  perm[k] = original primitive id */
/* of BVH-ordered triangle k.                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t num_nodes;
    uint32_t num_tris;
    float *box;        /* 6 per node: min xyz, max xyz */
    uint32_t *right;
    uint32_t *first;
    uint32_t *count;
    uint32_t *depth;
    uint32_t *perm;
} orc_bvh;

/* ======================================================================== */
/* BVH construction (the paper treats the BVH as given; this is our         */
/* deterministic binned-SAH reading, specified so that an independent       */
/* implementation reproduces it bit for bit).                               */
/* ======================================================================== */
typedef struct {
    const float *tris;   /* 9 floats per original triangle */
    float *tb;           /* per original triangle: bounds min xyz, max xyz */
    float *tc;           /* per original triangle: centroid xyz */
    uint32_t *idx;       /* working permutation */
    uint32_t *tmp;
    orc_bvh *out;
    uint32_t leaf_max, bins, max_depth;
    int error;
} build_ctx;

/* half surface area of a box, in double */
static double half_area(const float *mn, const float *mx)
{
    double dx = (double)mx[0] - (double)mn[0];
    double dy = (double)mx[1] - (double)mn[1];
    double dz = (double)mx[2] - (double)mn[2];
    return dx * dy + dy * dz + dz * dx;
}

static uint32_t bin_of(float c, float cmin, float k, uint32_t bins)
{
    float f = (c - cmin) * k;
    uint32_t b = (uint32_t)f;             /* f >= 0 and finite here */
    if (b > bins - 1) b = bins - 1;
    return b;
}

static uint32_t build_node(build_ctx *ctx, uint32_t begin, uint32_t end, uint32_t depth)
{
    orc_bvh *o = ctx->out;
    uint32_t node = o->num_nodes++;
    uint32_t n = end - begin;
    float mn[3] = { INFINITY, INFINITY, INFINITY }, mx[3] = { -INFINITY, -INFINITY, -INFINITY };
    float cmn[3] = { INFINITY, INFINITY, INFINITY }, cmx[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (uint32_t i = begin; i < end; i++) {
        const float *b = ctx->tb + 6 * (size_t)ctx->idx[i];
        const float *c = ctx->tc + 3 * (size_t)ctx->idx[i];
        for (int a = 0; a < 3; a++) {
            if (b[a] < mn[a]) mn[a] = b[a];
            if (b[a + 3] > mx[a]) mx[a] = b[a + 3];
            if (c[a] < cmn[a]) cmn[a] = c[a];
            if (c[a] > cmx[a]) cmx[a] = c[a];
        }
    }
    for (int a = 0; a < 3; a++) { o->box[6 * node + a] = mn[a]; o->box[6 * node + 3 + a] = mx[a]; }
    o->depth[node] = depth;
    if (n <= ctx->leaf_max) {
        o->right[node] = NONE32;
        o->first[node] = begin;
        o->count[node] = n;
        return node;
    }
    if (depth + 1 > ctx->max_depth) { ctx->error = 1; o->right[node] = NONE32; o->first[node] = begin; o->count[node] = n; return node; }

    /* binned SAH: cost(split) = A(L)*|L| + A(R)*|R|; minimal cost wins,
       ties go to the smaller axis, then the smaller split position */
    uint32_t B = ctx->bins;
    double best = INFINITY;
    int best_axis = -1;
    uint32_t best_split = 0;
    float best_k = 0.0f;
    uint32_t *cnt = (uint32_t *)malloc(sizeof(uint32_t) * B);
    float *bmn = (float *)malloc(sizeof(float) * 3 * B), *bmx = (float *)malloc(sizeof(float) * 3 * B);
    for (int a = 0; a < 3; a++) {
        float extent = cmx[a] - cmn[a];
        if (!(extent > 0.0f)) continue;
        float k = (float)B / extent;
        if (!isfinite(k)) continue;
        for (uint32_t j = 0; j < B; j++) {
            cnt[j] = 0;
            for (int q = 0; q < 3; q++) { bmn[3 * j + q] = INFINITY; bmx[3 * j + q] = -INFINITY; }
        }
        for (uint32_t i = begin; i < end; i++) {
            uint32_t t = ctx->idx[i];
            uint32_t j = bin_of(ctx->tc[3 * (size_t)t + a], cmn[a], k, B);
            const float *b = ctx->tb + 6 * (size_t)t;
            cnt[j]++;
            for (int q = 0; q < 3; q++) {
                if (b[q] < bmn[3 * j + q]) bmn[3 * j + q] = b[q];
                if (b[q + 3] > bmx[3 * j + q]) bmx[3 * j + q] = b[q + 3];
            }
        }
        for (uint32_t s = 1; s < B; s++) {
            float lmn[3] = { INFINITY, INFINITY, INFINITY }, lmx[3] = { -INFINITY, -INFINITY, -INFINITY };
            float rmn[3] = { INFINITY, INFINITY, INFINITY }, rmx[3] = { -INFINITY, -INFINITY, -INFINITY };
            uint32_t nl = 0, nr = 0;
            for (uint32_t j = 0; j < B; j++) {
                float *xmn = j < s ? lmn : rmn, *xmx = j < s ? lmx : rmx;
                if (j < s) nl += cnt[j]; else nr += cnt[j];
                if (cnt[j] == 0) continue;
                for (int q = 0; q < 3; q++) {
                    if (bmn[3 * j + q] < xmn[q]) xmn[q] = bmn[3 * j + q];
                    if (bmx[3 * j + q] > xmx[q]) xmx[q] = bmx[3 * j + q];
                }
            }
            if (nl == 0 || nr == 0) continue;
            double cost = half_area(lmn, lmx) * (double)nl + half_area(rmn, rmx) * (double)nr;
            if (cost < best) { best = cost; best_axis = a; best_split = s; best_k = k; }
        }
    }
    free(cnt); free(bmn); free(bmx);

    uint32_t mid;
    if (best_axis < 0) {
        mid = begin + n / 2;          /* all centroids coincide: split the list in half */
    } else {
        /* stable partition: bin < split goes left, original relative order kept */
        uint32_t w = begin;
        uint32_t r = 0;
        for (uint32_t i = begin; i < end; i++) {
            uint32_t t = ctx->idx[i];
            if (bin_of(ctx->tc[3 * (size_t)t + best_axis], cmn[best_axis], best_k, B) < best_split) ctx->idx[w++] = t;
            else ctx->tmp[r++] = t;
        }
        memcpy(ctx->idx + w, ctx->tmp, sizeof(uint32_t) * r);
        mid = w;
    }
    o->first[node] = 0;
    o->count[node] = 0;
    build_node(ctx, begin, mid, depth + 1);
    o->right[node] = build_node(ctx, mid, end, depth + 1);
    return node;
}

/* Build the binned-SAH BVH.  Arrays of out must hold 2n-1 nodes and n
   permutation entries.  Returns 0 on success, -1 on bad input, -2 when a
   leaf would exceed max_depth. */
int orc_build_sah(const float *tris, uint32_t n, uint32_t leaf_max, uint32_t bins,
                  uint32_t max_depth, orc_bvh *out)
{
    if (n == 0 || leaf_max < 1 || leaf_max > 8 || bins < 2 || n >= (1u << 28) || max_depth > 120) return -1;
    for (size_t i = 0; i < 9 * (size_t)n; i++) if (!isfinite(tris[i])) return -1;
    build_ctx ctx;
    memset(&ctx, 0, sizeof ctx);
    ctx.tris = tris;
    ctx.tb = (float *)malloc(sizeof(float) * 6 * (size_t)n);
    ctx.tc = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    ctx.idx = out->perm;
    ctx.tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    ctx.out = out;
    ctx.leaf_max = leaf_max; ctx.bins = bins; ctx.max_depth = max_depth;
    for (uint32_t t = 0; t < n; t++) {
        const float *v = tris + 9 * (size_t)t;
        for (int a = 0; a < 3; a++) {
            float lo = v[a], hi = v[a];
            if (v[3 + a] < lo) lo = v[3 + a];
            if (v[6 + a] < lo) lo = v[6 + a];
            if (v[3 + a] > hi) hi = v[3 + a];
            if (v[6 + a] > hi) hi = v[6 + a];
            ctx.tb[6 * (size_t)t + a] = lo;
            ctx.tb[6 * (size_t)t + 3 + a] = hi;
            ctx.tc[3 * (size_t)t + a] = (lo + hi) * 0.5f;
        }
        ctx.idx[t] = t;
    }
    out->num_nodes = 0;
    out->num_tris = n;
    build_node(&ctx, 0, n, 0);
    free(ctx.tb); free(ctx.tc); free(ctx.tmp);
    return ctx.error ? -2 : 0;
}

/* A second, deliberately different builder used to show that query results
   do not depend on the tree's shape: split at the median centroid along the
   axis of largest centroid extent (ties by original id). */
static const float *g_med_c;
static int g_med_axis;
static int med_cmp(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    float ca = g_med_c[3 * (size_t)a + g_med_axis], cb = g_med_c[3 * (size_t)b + g_med_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return a < b ? -1 : (a > b);
}

static uint32_t build_median_node(build_ctx *ctx, uint32_t begin, uint32_t end, uint32_t depth)
{
    orc_bvh *o = ctx->out;
    uint32_t node = o->num_nodes++;
    uint32_t n = end - begin;
    float mn[3] = { INFINITY, INFINITY, INFINITY }, mx[3] = { -INFINITY, -INFINITY, -INFINITY };
    float cmn[3] = { INFINITY, INFINITY, INFINITY }, cmx[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (uint32_t i = begin; i < end; i++) {
        const float *b = ctx->tb + 6 * (size_t)ctx->idx[i];
        const float *c = ctx->tc + 3 * (size_t)ctx->idx[i];
        for (int a = 0; a < 3; a++) {
            if (b[a] < mn[a]) mn[a] = b[a];
            if (b[a + 3] > mx[a]) mx[a] = b[a + 3];
            if (c[a] < cmn[a]) cmn[a] = c[a];
            if (c[a] > cmx[a]) cmx[a] = c[a];
        }
    }
    for (int a = 0; a < 3; a++) { o->box[6 * node + a] = mn[a]; o->box[6 * node + 3 + a] = mx[a]; }
    o->depth[node] = depth;
    if (n <= ctx->leaf_max || depth + 1 > ctx->max_depth) {
        if (n > ctx->leaf_max) ctx->error = 1;
        o->right[node] = NONE32; o->first[node] = begin; o->count[node] = n;
        return node;
    }
    int axis = 0;
    for (int a = 1; a < 3; a++) if (cmx[a] - cmn[a] > cmx[axis] - cmn[axis]) axis = a;
    g_med_c = ctx->tc; g_med_axis = axis;
    qsort(ctx->idx + begin, n, sizeof(uint32_t), med_cmp);
    uint32_t mid = begin + n / 2;
    o->first[node] = 0; o->count[node] = 0;
    build_median_node(ctx, begin, mid, depth + 1);
    o->right[node] = build_median_node(ctx, mid, end, depth + 1);
    return node;
}

int orc_build_median(const float *tris, uint32_t n, uint32_t leaf_max, uint32_t max_depth, orc_bvh *out)
{
    if (n == 0 || leaf_max < 1 || leaf_max > 8 || n >= (1u << 28) || max_depth > 120) return -1;
    build_ctx ctx;
    memset(&ctx, 0, sizeof ctx);
    ctx.tris = tris;
    ctx.tb = (float *)malloc(sizeof(float) * 6 * (size_t)n);
    ctx.tc = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    ctx.idx = out->perm;
    ctx.out = out;
    ctx.leaf_max = leaf_max; ctx.max_depth = max_depth;
    for (uint32_t t = 0; t < n; t++) {
        const float *v = tris + 9 * (size_t)t;
        for (int a = 0; a < 3; a++) {
            float lo = fminf(fminf(v[a], v[3 + a]), v[6 + a]);
            float hi = fmaxf(fmaxf(v[a], v[3 + a]), v[6 + a]);
            ctx.tb[6 * (size_t)t + a] = lo;
            ctx.tb[6 * (size_t)t + 3 + a] = hi;
            ctx.tc[3 * (size_t)t + a] = (lo + hi) * 0.5f;
        }
        ctx.idx[t] = t;
    }
    out->num_nodes = 0;
    out->num_tris = n;
    build_median_node(&ctx, 0, n, 0);
    free(ctx.tb); free(ctx.tc);
    return ctx.error ? -2 : 0;
}

/* A third builder, the linear BVH of the device build (Lauterbach et al.,
   "Fast BVH Construction on GPUs", 2009; the binary radix tree of Karras,
   "Maximizing Parallelism in the Construction of BVHs, Octrees, and k-d
   Trees", HPG 2012), written top-down from its definition:
   * centre of triangle t on axis a: c = (lo + hi) * 0.5 with lo / hi the
     vertices' min / max (the same centre as the SAH builder);
   * cmin / cmax = min / max centre over all triangles; cubic cells: one
     scale = 2^21 / (the largest of the three extents cmax - cmin), or 0 when
     that extent is 0 or the quotient is not finite;
     cell q = min(floor((c - cmin) * scale), 2^21 - 1) on each axis;
   * Morton code: bit k of the x / y / z cell goes to bit 3k+2 / 3k+1 / 3k;
   * triangles sorted by (code, primitive id);
   * the node over sorted positions [b, e) is a leaf when e - b <= leaf_max;
     otherwise it splits where the key (code, position) first changes at the
     highest bit in which its first and last keys differ: the code's bit when
     the codes differ, else the position's bit;
   * boxes are the exact bounds of the node's triangles; DFS pre-order. */
typedef struct {
    uint64_t *code;      /* by sorted position */
    uint32_t *perm;      /* sorted position -> primitive id */
    const float *tris;
    orc_bvh *out;
    uint32_t leaf_max, max_depth;
    int error;
} lbvh_ctx;

static const uint64_t *g_lb_codes;
static int lb_cmp(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (g_lb_codes[a] != g_lb_codes[b]) return g_lb_codes[a] < g_lb_codes[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int top_bit64(uint64_t x) { int h = 63; while (!((x >> h) & 1u)) h--; return h; }

static uint32_t lbvh_node(lbvh_ctx *ctx, uint32_t b, uint32_t e, uint32_t depth)
{
    orc_bvh *o = ctx->out;
    uint32_t node = o->num_nodes++;
    float mn[3] = { INFINITY, INFINITY, INFINITY }, mx[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (uint32_t i = b; i < e; i++) {
        const float *v = ctx->tris + 9 * (size_t)ctx->perm[i];
        for (int k = 0; k < 3; k++)
            for (int a = 0; a < 3; a++) {
                if (v[3 * k + a] < mn[a]) mn[a] = v[3 * k + a];
                if (v[3 * k + a] > mx[a]) mx[a] = v[3 * k + a];
            }
    }
    for (int a = 0; a < 3; a++) { o->box[6 * node + a] = mn[a]; o->box[6 * node + 3 + a] = mx[a]; }
    o->depth[node] = depth;
    if (e - b <= ctx->leaf_max) {
        if (depth > ctx->max_depth) ctx->error = 1;
        o->right[node] = NONE32; o->first[node] = b; o->count[node] = e - b;
        return node;
    }
    uint32_t split = e;
    uint64_t cb = ctx->code[b], ce = ctx->code[e - 1];
    if (cb != ce) {
        int h = top_bit64(cb ^ ce);
        for (uint32_t i = b + 1; i < e; i++)
            if ((ctx->code[i] >> h) != (cb >> h)) { split = i; break; }
    } else {
        int h = top_bit64((uint64_t)(b ^ (e - 1)));
        for (uint32_t i = b + 1; i < e; i++)
            if ((i >> h) != (b >> h)) { split = i; break; }
    }
    o->first[node] = 0; o->count[node] = 0;
    lbvh_node(ctx, b, split, depth + 1);
    o->right[node] = lbvh_node(ctx, split, e, depth + 1);
    return node;
}

/* Morton code of every triangle (original order), as defined above. */
void orc_lbvh_codes(const float *tris, uint32_t n, uint64_t *code)
{
    float *c = (float *)malloc(sizeof(float) * 3 * (size_t)n);
    float cmin[3] = { INFINITY, INFINITY, INFINITY }, cmax[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (uint32_t t = 0; t < n; t++) {
        const float *v = tris + 9 * (size_t)t;
        for (int a = 0; a < 3; a++) {
            float lo = v[a], hi = v[a];
            if (v[3 + a] < lo) lo = v[3 + a];
            if (v[6 + a] < lo) lo = v[6 + a];
            if (v[3 + a] > hi) hi = v[3 + a];
            if (v[6 + a] > hi) hi = v[6 + a];
            float ce = (lo + hi) * 0.5f;
            c[3 * (size_t)t + a] = ce;
            if (ce < cmin[a]) cmin[a] = ce;
            if (ce > cmax[a]) cmax[a] = ce;
        }
    }
    /* cubic cells: one scale, from the largest extent */
    float emax = 0.0f;
    for (int a = 0; a < 3; a++) {
        float ext = cmax[a] - cmin[a];
        if (ext > emax) emax = ext;
    }
    float scale = emax > 0.0f ? 2097152.0f / emax : 0.0f;
    if (!isfinite(scale)) scale = 0.0f;
    for (uint32_t t = 0; t < n; t++) {
        uint32_t q[3];
        for (int a = 0; a < 3; a++) {
            float f = floorf((c[3 * (size_t)t + a] - cmin[a]) * scale);
            q[a] = f >= 2097151.0f ? 2097151u : (uint32_t)f;
        }
        uint64_t m = 0;
        for (int k = 0; k < 21; k++) {
            m |= (uint64_t)((q[0] >> k) & 1u) << (3 * k + 2);
            m |= (uint64_t)((q[1] >> k) & 1u) << (3 * k + 1);
            m |= (uint64_t)((q[2] >> k) & 1u) << (3 * k);
        }
        code[t] = m;
    }
    free(c);
}

int orc_build_lbvh(const float *tris, uint32_t n, uint32_t leaf_max, uint32_t max_depth, orc_bvh *out)
{
    if (n == 0 || leaf_max < 1 || leaf_max > 8 || n >= (1u << 28) || max_depth > 120) return -1;
    for (size_t i = 0; i < 9 * (size_t)n; i++) if (!isfinite(tris[i])) return -1;
    uint64_t *code = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t *sorted = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    orc_lbvh_codes(tris, n, code);
    for (uint32_t t = 0; t < n; t++) out->perm[t] = t;
    g_lb_codes = code;
    qsort(out->perm, n, sizeof(uint32_t), lb_cmp);
    for (uint32_t i = 0; i < n; i++) sorted[i] = code[out->perm[i]];
    lbvh_ctx ctx = { sorted, out->perm, tris, out, leaf_max, max_depth, 0 };
    out->num_nodes = 0;
    out->num_tris = n;
    lbvh_node(&ctx, 0, n, 0);
    free(code); free(sorted);
    return ctx.error ? -2 : 0;
}

/* Treelet restructuring of the linear BVH (Karras and Aila, "Fast Parallel
   Construction of High-Quality Bounding Volume Hierarchies", HPG 2013),
   written from its description, with this library's choices:
   * the linear BVH's leaves (at most leaf_max triangles) stay as they are;
     only interior nodes are rearranged;
   * a pass visits every interior node after every interior node below it
     (post-order).  At node r the treelet's leaves start as r's two
     children; while there are fewer than 7, the one with the largest half
     surface area among those that are interior nodes (the first in list
     order on ties) is expanded: its left child takes its place in the list
     and its right child goes to the end;
   * the cost of a treelet topology is the sum of the half surface areas of
     its interior nodes (what lies below the treelet's leaves is fixed).
     The optimum over every binary tree on the leaves, by dynamic
     programming over subsets S of the leaves: c({i}) = 0,
     c(S) = A(S) + min over P of (c(P) + c(S \ P)), P ranging in increasing
     bitmask order over the proper subsets of S that hold S's lowest member,
     the first minimum kept; A(S) = half area of the union of S's boxes;
   * the treelet is rebuilt only when the optimum is below the current
     topology's cost (the same recurrence along the current topology).  r
     stays the root; the other new interior nodes, in depth-first pre-order,
     take the identities of the expanded nodes in expansion order; P (the
     part with the lowest member) is the left child;
   * an interior node's box is the union of its children's boxes, the left
     child's value kept on ties, as everywhere in this library;
   * half area of a box: dx*dy + dy*dz + dz*dx in binary32, summed left to
     right.
   The result is written in depth-first pre-order with the triangles in leaf
   order. */
#define TL_LEAVES 7

typedef struct {
    uint32_t *left, *right;    /* interior: children; leaf: right = NONE32 */
    uint32_t *first, *count;   /* leaf: range of the linear BVH's triangle order */
    float *box;
} tl_tree;

static float tl_half_area(const float *b)
{
    float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

static void tl_union(const float *l, const float *r, float *out)
{
    for (int a = 0; a < 3; a++) {
        out[a] = r[a] < l[a] ? r[a] : l[a];
        out[3 + a] = r[3 + a] > l[3 + a] ? r[3 + a] : l[3 + a];
    }
}

static int tl_popc(uint32_t x) { int c = 0; while (x) { c += x & 1u; x >>= 1; } return c; }
static int tl_ctz(uint32_t x) { int c = 0; while (!(x & 1u)) { x >>= 1; c++; } return c; }

static void tl_treelet(tl_tree *t, uint32_t r)
{
    uint32_t L[TL_LEAVES], I[TL_LEAVES - 1];
    int nl = 2, ni = 1;
    L[0] = t->left[r]; L[1] = t->right[r]; I[0] = r;
    while (nl < TL_LEAVES) {
        int best = -1;
        float ba = 0.0f;
        for (int i = 0; i < nl; i++) {
            if (t->right[L[i]] == NONE32) continue;
            float a = tl_half_area(t->box + 6 * (size_t)L[i]);
            if (best < 0 || a > ba) { best = i; ba = a; }
        }
        if (best < 0) break;
        uint32_t x = L[best];
        I[ni++] = x;
        L[best] = t->left[x];
        L[nl++] = t->right[x];
    }
    if (nl < 3) return;                 /* two leaves: one topology */
    const uint32_t full = (1u << nl) - 1u;
    float area[1u << TL_LEAVES], cost[1u << TL_LEAVES];
    uint32_t bestp[1u << TL_LEAVES];
    for (uint32_t S = 1; S <= full; S++) {
        float u[6];
        int have = 0;
        for (int i = 0; i < nl; i++) {
            if (!((S >> i) & 1u)) continue;
            const float *b = t->box + 6 * (size_t)L[i];
            if (!have) { memcpy(u, b, sizeof u); have = 1; }
            else tl_union(u, b, u);
        }
        area[S] = tl_half_area(u);
    }
    for (uint32_t S = 1; S <= full; S++) {
        if (tl_popc(S) == 1) { cost[S] = 0.0f; bestp[S] = 0; continue; }
        const uint32_t low = S & (~S + 1u);
        float best = 0.0f;
        uint32_t bp = 0;
        for (uint32_t P = 1; P < S; P++) {
            if ((P & S) != P || !(P & low)) continue;
            float c = cost[P] + cost[S ^ P];
            if (bp == 0 || c < best) { best = c; bp = P; }
        }
        cost[S] = area[S] + best;
        bestp[S] = bp;
    }
    /* the current topology's cost: expanded nodes' children were expanded
       later, so a reverse sweep sees children first */
    uint32_t mask[TL_LEAVES - 1];
    float cur[TL_LEAVES - 1];
    for (int j = ni - 1; j >= 0; j--) {
        uint32_t ch[2] = { t->left[I[j]], t->right[I[j]] }, m[2];
        float cc[2];
        for (int k = 0; k < 2; k++) {
            m[k] = 0; cc[k] = 0.0f;
            for (int i = 0; i < nl; i++) if (L[i] == ch[k]) m[k] = 1u << i;
            for (int q = j + 1; q < ni; q++) if (I[q] == ch[k]) { m[k] = mask[q]; cc[k] = cur[q]; }
        }
        mask[j] = m[0] | m[1];
        cur[j] = area[mask[j]] + (cc[0] + cc[1]);
    }
    if (!(cost[full] < cur[0])) return;
    /* rebuild: identities in pre-order, then boxes children first */
    uint32_t id_of[1u << TL_LEAVES], order[TL_LEAVES - 1], stack[TL_LEAVES];
    int sp = 0, no = 0, next = 1;
    stack[sp++] = full;
    while (sp) {
        uint32_t S = stack[--sp];
        id_of[S] = (S == full) ? r : I[next++];
        order[no++] = S;
        uint32_t P = bestp[S], Q = S ^ P;
        if (tl_popc(Q) > 1) stack[sp++] = Q;
        if (tl_popc(P) > 1) stack[sp++] = P;
    }
    for (int k = no - 1; k >= 0; k--) {
        uint32_t S = order[k], P = bestp[S], Q = S ^ P;
        uint32_t id = id_of[S];
        uint32_t l = tl_popc(P) == 1 ? L[tl_ctz(P)] : id_of[P];
        uint32_t rr = tl_popc(Q) == 1 ? L[tl_ctz(Q)] : id_of[Q];
        t->left[id] = l;
        t->right[id] = rr;
        tl_union(t->box + 6 * (size_t)l, t->box + 6 * (size_t)rr, t->box + 6 * (size_t)id);
    }
}

static void tl_visit(tl_tree *t, uint32_t v)
{
    if (t->right[v] == NONE32) return;
    tl_visit(t, t->left[v]);
    tl_visit(t, t->right[v]);
    tl_treelet(t, v);
}

typedef struct {
    const tl_tree *t;
    const uint32_t *perm_in;
    orc_bvh *out;
    uint32_t max_depth, tri;
    int error;
} tl_emit_ctx;

static void tl_emit(tl_emit_ctx *e, uint32_t v, uint32_t depth)
{
    orc_bvh *o = e->out;
    uint32_t node = o->num_nodes++;
    memcpy(o->box + 6 * (size_t)node, e->t->box + 6 * (size_t)v, 6 * sizeof(float));
    o->depth[node] = depth;
    if (e->t->right[v] == NONE32) {
        if (depth > e->max_depth) e->error = 1;
        o->right[node] = NONE32;
        o->first[node] = e->tri;
        o->count[node] = e->t->count[v];
        for (uint32_t k = 0; k < e->t->count[v]; k++) o->perm[e->tri++] = e->perm_in[e->t->first[v] + k];
        return;
    }
    o->first[node] = 0; o->count[node] = 0;
    tl_emit(e, e->t->left[v], depth + 1);
    o->right[node] = o->num_nodes;
    tl_emit(e, e->t->right[v], depth + 1);
}

/* `passes` treelet passes over a built tree (in place). */
static int tl_restructure(orc_bvh *out, uint32_t n, uint32_t max_depth, uint32_t passes)
{
    const uint32_t m = out->num_nodes;
    tl_tree t;
    t.left = (uint32_t *)malloc(sizeof(uint32_t) * m);
    t.right = (uint32_t *)malloc(sizeof(uint32_t) * m);
    t.first = (uint32_t *)malloc(sizeof(uint32_t) * m);
    t.count = (uint32_t *)malloc(sizeof(uint32_t) * m);
    t.box = (float *)malloc(sizeof(float) * 6 * (size_t)m);
    uint32_t *perm_in = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    memcpy(perm_in, out->perm, sizeof(uint32_t) * (size_t)n);
    memcpy(t.box, out->box, sizeof(float) * 6 * (size_t)m);
    for (uint32_t i = 0; i < m; i++) {
        t.right[i] = out->right[i];
        t.left[i] = out->right[i] == NONE32 ? NONE32 : i + 1;   /* pre-order: the left child is next */
        t.first[i] = out->first[i];
        t.count[i] = out->count[i];
    }
    for (uint32_t p = 0; p < passes; p++) tl_visit(&t, 0);
    tl_emit_ctx e = { &t, perm_in, out, max_depth, 0, 0 };
    out->num_nodes = 0;
    tl_emit(&e, 0, 0);
    free(t.left); free(t.right); free(t.first); free(t.count); free(t.box); free(perm_in);
    if (out->num_nodes != m || e.tri != n) return -1;
    return e.error ? -2 : 0;
}

/* The linear BVH of orc_build_lbvh after `passes` treelet passes.  Returns
   as orc_build_lbvh; -2 also when the restructured tree is deeper than
   max_depth. */
int orc_build_lbvh_treelet(const float *tris, uint32_t n, uint32_t leaf_max, uint32_t max_depth, uint32_t passes,
                           orc_bvh *out)
{
    if (passes > 16) return -1;
    /* the linear BVH first, deep enough for any radix tree */
    int rc = orc_build_lbvh(tris, n, leaf_max, 120, out);
    if (rc != 0) return rc;
    return tl_restructure(out, n, max_depth, passes);
}

/* The binned-SAH BVH of orc_build_sah after `passes` treelet passes (the
   SAH tree is built with max_depth, the result checked against it too). */
int orc_build_sah_treelet(const float *tris, uint32_t n, uint32_t leaf_max, uint32_t bins, uint32_t max_depth,
                          uint32_t passes, orc_bvh *out)
{
    if (passes > 16) return -1;
    int rc = orc_build_sah(tris, n, leaf_max, bins, max_depth, out);
    if (rc != 0) return rc;
    return tl_restructure(out, n, max_depth, passes);
}

/* ======================================================================== */
/* Ray primitives                                                           */
/* ======================================================================== */

/* A ray is valid when its origin and direction are finite, the direction is
   not the zero vector, neither bound is NaN and tmin < tmax (tmax may be
   +inf).  Invalid rays are misses that are never hashed or traversed. */
static int ray_valid(const float *r)
{
    for (int a = 0; a < 3; a++) if (!isfinite(r[a]) || !isfinite(r[4 + a])) return 0;
    if (r[4] == 0.0f && r[5] == 0.0f && r[6] == 0.0f) return 0;
    if (isnan(r[3]) || isnan(r[7])) return 0;
    return r[3] < r[7];
}

/* Slab test of one box against the interval [tmin, tcur].  The far distance
   is scaled by 1 + 3*2^-23 (>= 1 + 2*gamma_3), the conservative bound of
   Ize, "Robust BVH Ray Traversal" (JCGT 2013), so rounding in the slab
   distances never rejects a box the exact ray enters. */
static int slab(const float *b, const float *o, const float *inv, float tmin, float tcur, float *tnear_out)
{
    float lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        float t0 = (b[a] - o[a]) * inv[a];
        float t1 = (b[3 + a] - o[a]) * inv[a];
        lo[a] = min_num(t0, t1);
        hi[a] = max_num(t0, t1);
    }
    float tnear = max_num(max_num(max_num(lo[0], lo[1]), lo[2]), tmin);
    float tfar = min_num(min_num(min_num(hi[0], hi[1]), hi[2]), tcur) * bits_to_float(0x3F800003u);
    *tnear_out = tnear;
    return tnear <= tfar;
}

/* Moller-Trumbore ray/triangle test (Moller and Trumbore 1997), two-sided,
   in binary32: e1 = v1-v0, e2 = v2-v0, p = d x e2, det = e1.p; det == 0
   misses; inv = 1/det; s = o-v0; u = (s.p)*inv in [0,1]; q = s x e1;
   v = (d.q)*inv >= 0 with u+v <= 1; t = (e2.q)*inv.  dot(a,b) is
   (ax*bx + ay*by) + az*bz.  Returns 1 and (t,u,v) when inside the
   triangle; the caller applies its interval. */
static int moller_trumbore(const float *v0, const float *v1, const float *v2, const float *o,
                           const float *d, float *t_out, float *u_out, float *v_out)
{
    float e1[3] = { v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2] };
    float e2[3] = { v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2] };
    float p[3] = { d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0] };
    float det = (e1[0] * p[0] + e1[1] * p[1]) + e1[2] * p[2];
    if (det == 0.0f) return 0;
    float inv = 1.0f / det;
    float s[3] = { o[0] - v0[0], o[1] - v0[1], o[2] - v0[2] };
    float u = ((s[0] * p[0] + s[1] * p[1]) + s[2] * p[2]) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return 0;
    float q[3] = { s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0] };
    float v = ((d[0] * q[0] + d[1] * q[1]) + d[2] * q[2]) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return 0;
    *t_out = ((e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2]) * inv;
    *u_out = u;
    *v_out = v;
    return 1;
}

/* ======================================================================== */
/* Ray hash (our reading for the configured predictor: the paper's hash    */
/* maps origin and direction bits to an index, "HRPP Hash Function"; the   */
/* workloads here quantise the origin on a grid over the scene bounds and  */
/* the direction on an octahedral map (Meyer et al. 2010; Cigolle et al.,  */
/* JCGT 2014), then fold the key into the table by Fibonacci hashing).     */
/* ======================================================================== */
typedef struct {
    float bmin[3];
    float scale[3];
    uint32_t qo, qd, log2n;
    uint32_t mode;       /* 0 grid + octahedral, 1 the paper's IEEE-754 bit hash (precision qo) */
} hash_params;

static void hash_setup(hash_params *h, const float *root_box, uint32_t qo, uint32_t qd, uint32_t log2n)
{
    h->mode = 0;
    for (int a = 0; a < 3; a++) {
        float ext = root_box[3 + a] - root_box[a];
        float s = (float)(1u << qo) / ext;
        if (!(ext > 0.0f) || !isfinite(s)) s = 0.0f;
        h->bmin[a] = root_box[a];
        h->scale[a] = s;
    }
    h->qo = qo; h->qd = qd; h->log2n = log2n;
}

static uint32_t quantize(float x, float maxcell)
{
    float c = floorf(x);
    if (!(c >= 0.0f)) c = 0.0f;          /* also maps NaN to cell 0 */
    else if (c > maxcell) c = maxcell;
    return (uint32_t)c;
}

static float sign_not_neg(float x) { return x >= 0.0f ? 1.0f : -1.0f; }

/* The paper's hash ("HRPP Hash Function"): from each binary32 value keep
   the sign bit, the p most significant exponent bits and the p most
   significant mantissa bits, sign highest (2p+1 bits). */
static uint32_t ieee_hash(float x, uint32_t p)
{
    uint32_t u = float_to_bits(x);
    uint32_t sign = u >> 31, expo = (u >> 23) & 0xFFu, mant = u & 0x7FFFFFu;
    return (sign << (2 * p)) | ((expo >> (8 - p)) << p) | (mant >> (23 - p));
}

/* Swizzle origin with direction by XOR (o.x^d.z, o.y^d.y, o.z^d.x) and
   concatenate the three values at a stride of 8 bits (p <= 3, 2p+1 <= 7
   bits fit a byte) or 16 bits (4 <= p <= 7, at most 15 bits a field), at
   most 48 bits in all.  p is limited to 7 so that a field never exceeds
   the 16 bits the paper extracts per value. */
static uint64_t paper_key(const float *o, const float *d, uint32_t p)
{
    uint64_t h0 = ieee_hash(o[0], p) ^ ieee_hash(d[2], p);
    uint64_t h1 = ieee_hash(o[1], p) ^ ieee_hash(d[1], p);
    uint64_t h2 = ieee_hash(o[2], p) ^ ieee_hash(d[0], p);
    uint32_t stride = p <= 3 ? 8u : 16u;
    return h0 | (h1 << stride) | (h2 << (2 * stride));
}

static void hash_ray(const hash_params *h, const float *o, const float *d, uint64_t *key, uint32_t *idx)
{
    if (h->mode == 1) {
        uint64_t k = paper_key(o, d, h->qo);
        *key = k;
        *idx = (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> (64u - h->log2n));
        return;
    }
    uint32_t cell[3];
    float maxo = (float)((1u << h->qo) - 1u);
    for (int a = 0; a < 3; a++) cell[a] = quantize((o[a] - h->bmin[a]) * h->scale[a], maxo);
    /* octahedral map of d onto [-1,1]^2 */
    float l1 = (fabsf(d[0]) + fabsf(d[1])) + fabsf(d[2]);
    float inv = 1.0f / l1;
    float px = d[0] * inv, py = d[1] * inv;
    if (d[2] < 0.0f) {
        float fx = (1.0f - fabsf(py)) * sign_not_neg(px);
        float fy = (1.0f - fabsf(px)) * sign_not_neg(py);
        px = fx; py = fy;
    }
    float half = (float)(1u << (h->qd - 1u));
    float maxd = (float)((1u << h->qd) - 1u);
    uint32_t bu = quantize((px + 1.0f) * half, maxd);
    uint32_t bv = quantize((py + 1.0f) * half, maxd);
    uint64_t k = (uint64_t)cell[0] | ((uint64_t)cell[1] << h->qo) | ((uint64_t)cell[2] << (2 * h->qo))
               | ((uint64_t)bu << (3 * h->qo)) | ((uint64_t)bv << (3 * h->qo + h->qd));
    *key = k;
    *idx = (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> (64u - h->log2n));
}

/* Exported for the hash pins. */
void orc_hash(const float *root_box, uint32_t qo, uint32_t qd, uint32_t log2n, const float *rays,
              uint32_t n, uint64_t *keys, uint32_t *idxs, uint32_t mode)
{
    hash_params h;
    hash_setup(&h, root_box, qo, qd, log2n);
    h.mode = mode;
    for (uint32_t i = 0; i < n; i++) hash_ray(&h, rays + 8 * (size_t)i, rays + 8 * (size_t)i + 4, keys + i, idxs + i);
}

/* Exported for the Moller-Trumbore pin. */
int orc_mt(const float *tri9, const float *ray8, float *tuv)
{
    return moller_trumbore(tri9, tri9 + 3, tri9 + 6, ray8, ray8 + 4, tuv, tuv + 1, tuv + 2);
}

/* Exported for the slab pin. */
int orc_slab(const float *box6, const float *ray8, float tcur, float *tnear)
{
    float inv[3] = { 1.0f / ray8[4], 1.0f / ray8[5], 1.0f / ray8[6] };
    return slab(box6, ray8, inv, ray8[3], tcur, tnear);
}

/* ======================================================================== */
/* Traversal                                                                */
/* ======================================================================== */
typedef struct {
    const orc_bvh *bvh;
    const float *vtx;          /* 9 floats per BVH-ordered triangle */
    const uint32_t *leaf_node_by_first;  /* node index of the leaf starting at triangle k */
    const uint32_t *parent;    /* parent node of each node (NONE32 for the root) */
    const uint32_t *sub_lo;    /* BVH-ordered triangle range [sub_lo, sub_end) */
    const uint32_t *sub_end;   /*   of each node's subtree */
} scene;

typedef struct {
    float t, u, v;
    uint32_t prim;   /* original id; NONE32 = none */
    uint32_t leaf;   /* canonical leaf id holding prim */
} best_hit;

static uint32_t leaf_id(uint32_t first, uint32_t count) { return (first << 3) | (count - 1u); }

/* Test the triangles of one leaf.  ANY: returns 1 on the first hit inside
   (tmin, tmax).  CLOSEST: updates *b with the lexicographically smallest
   (t, prim) inside (tmin, tmax); returns 1 if *b changed. */
static int test_leaf(const scene *sc, uint32_t first, uint32_t count, const float *r, int closest,
                     best_hit *b, uint64_t *st)
{
    int changed = 0;
    for (uint32_t k = first; k < first + count; k++) {
        const float *v = sc->vtx + 9 * (size_t)k;
        float t, u, w;
        st[S_TRI_TESTS]++;
        if (!moller_trumbore(v, v + 3, v + 6, r, r + 4, &t, &u, &w)) continue;
        if (!(r[3] < t && t < r[7])) continue;
        uint32_t prim = sc->bvh->perm[k];
        if (!closest) {
            b->t = t; b->u = u; b->v = w; b->prim = prim; b->leaf = leaf_id(first, count);
            return 1;
        }
        if (t < b->t || (t == b->t && prim < b->prim)) {
            b->t = t; b->u = u; b->v = w; b->prim = prim; b->leaf = leaf_id(first, count);
            changed = 1;
        }
    }
    return changed;
}

/* Walk the subtree of `node`, whose own box the caller has already tested
   against [tmin, tcur].  With node = root this is the whole traversal; a
   predicted node ("Go Up Level") is walked the same way. */
static int walk(const scene *sc, uint32_t node, const float *r, const float *inv, int closest, best_hit *b,
                uint64_t *st)
{
    const orc_bvh *bvh = sc->bvh;
    uint32_t stack_node[128];
    float stack_t[128];
    int sp = 0;
    float tmin = r[3];
    float tcur = closest ? (b->prim != NONE32 ? b->t : r[7]) : r[7];
    int found = (b->prim != NONE32);
    const float pad = bits_to_float(0x3F800003u);
    for (;;) {
        st[S_NODES_VISITED]++;
        if (bvh->right[node] != NONE32) {
            uint32_t L = node + 1, R = bvh->right[node];
            float tl, tr;
            st[S_INTERIOR_VISITED]++;
            st[S_BOX_TESTS] += 2;
            int hl = slab(bvh->box + 6 * (size_t)L, r, inv, tmin, tcur, &tl);
            int hr = slab(bvh->box + 6 * (size_t)R, r, inv, tmin, tcur, &tr);
            if (hl && hr) {
                if (tr < tl) { stack_node[sp] = L; stack_t[sp] = tl; sp++; node = R; }
                else         { stack_node[sp] = R; stack_t[sp] = tr; sp++; node = L; }
                continue;
            }
            if (hl) { node = L; continue; }
            if (hr) { node = R; continue; }
        } else {
            st[S_LEAF_VISITED]++;
            if (test_leaf(sc, bvh->first[node], bvh->count[node], r, closest, b, st)) {
                found = 1;
                if (!closest) return 1;
                tcur = b->t;
            }
        }
        /* pop */
        for (;;) {
            if (sp == 0) return found;
            sp--;
            if (stack_t[sp] <= tcur * pad) break;
        }
        node = stack_node[sp];
    }
}

/* Plain stack traversal.  Order fully fixed:
   root box tested first (one box test); at an interior node both child
   boxes are tested against [tmin, tcur] (two box tests); with both hit,
   the child with the smaller entry distance is visited first (left on a
   tie) and the other is pushed with its entry distance; a popped node is
   visited only if its stored entry distance still passes the slab
   criterion against the current tcur (tnear <= tcur * (1 + 3*2^-23), which
   is exactly the slab test re-run with the shrunken interval).  Leaves test
   their triangles in BVH order.  Any-hit stops at the first hit. */
static int traverse(const scene *sc, const float *r, const float *inv, int closest, best_hit *b, uint64_t *st)
{
    float tcur = closest ? (b->prim != NONE32 ? b->t : r[7]) : r[7];
    float tn;
    st[S_TRAVERSALS]++;
    st[S_BOX_TESTS]++;
    if (!slab(sc->bvh->box, r, inv, r[3], tcur, &tn)) return b->prim != NONE32;
    return walk(sc, 0, r, inv, closest, b, st);
}

/* The node a record names at go-up level g: the leaf holding the result, or
   its ancestor g levels up (the root if the leaf has fewer ancestors). */
static uint32_t predicted_node_of(const scene *sc, uint32_t leaf, uint32_t go_up)
{
    uint32_t node = sc->leaf_node_by_first[leaf >> 3];
    for (uint32_t k = 0; k < go_up && sc->parent[node] != NONE32; k++) node = sc->parent[node];
    return node;
}

/* ======================================================================== */
/* HRPP per ray ("Overview" direct flow; "Precision and Recall")            */
/* ======================================================================== */
enum { Q_ANY = 0, Q_CLOSEST = 1 };
enum { C_PAPER = 0, C_EXACT = 1 };

typedef struct {
    uint64_t *tag;      /* [N] */
    uint32_t *slot;     /* [N * W] */
    uint32_t W;
    uint32_t go_up;     /* 0: slots hold leaf ids; g >= 1: node indices g levels above the leaf */
    uint32_t policy;    /* bit 0: FIFO eviction within an entry; bit 1: the resident tag keeps its entry */
    hash_params h;
} table;

typedef struct {
    uint8_t has;        /* record emitted */
    uint32_t idx;
    uint64_t key;
    uint32_t leaf;
} record;

/* per-ray outcome codes (optional output used by the pins) */
enum { OUT_INVALID = 0, OUT_TRAVERSED = 1, OUT_PRED_HIT = 2, OUT_FALSE_POS = 3 };

static void trace_one(const scene *sc, const table *tb, const float *r, int query, int cmode,
                      uint8_t *occ, float *hit4, record *rec, uint8_t *outcome, uint64_t *st)
{
    best_hit b = { INFINITY, 0.0f, 0.0f, NONE32, NONE32 };
    int closest = (query == Q_CLOSEST);
    rec->has = 0;
    if (outcome) *outcome = OUT_INVALID;
    st[S_RAYS]++;
    if (!ray_valid(r)) {
        st[S_INVALID]++;
        goto write;
    }
    float inv[3] = { 1.0f / r[4], 1.0f / r[5], 1.0f / r[6] };
    int hit = 0;
    if (tb) {
        uint64_t key; uint32_t idx;
        hash_ray(&tb->h, r, r + 4, &key, &idx);
        st[S_LOOKUPS]++;
        const uint32_t *slots = tb->slot + (size_t)idx * tb->W;
        int positive = (tb->tag[idx] == key && slots[0] != NONE32);
        uint32_t skip_depth = 0;
        if (positive) {
            st[S_POSITIVES]++;
            uint64_t box_before = st[S_BOX_TESTS], leaf_before = st[S_LEAF_VISITED], tri_before = st[S_TRI_TESTS];
            /* evaluate the predicted nodes in slot order: a node's box is
               tested against [tmin, tcur] (tcur = tmax, or the best hit so
               far for closest hit) and, if hit, its subtree is walked (a
               predicted leaf: its triangles).  The interior nodes above the
               node that produced the result count as skipped. */
            for (uint32_t s = 0; s < tb->W && slots[s] != NONE32; s++) {
                uint32_t node = tb->go_up ? slots[s] : sc->leaf_node_by_first[slots[s] >> 3];
                float tn;
                float tcur = (closest && b.prim != NONE32) ? b.t : r[7];
                st[S_BOX_TESTS]++;
                if (!slab(sc->bvh->box + 6 * (size_t)node, r, inv, r[3], tcur, &tn)) continue;
                float bt = b.t;
                uint32_t bp = b.prim;
                int f = walk(sc, node, r, inv, closest, &b, st);
                if (b.prim != bp || b.t != bt) skip_depth = sc->bvh->depth[node];
                if (f) {
                    hit = 1;
                    if (!closest) break;
                }
            }
            st[S_PRED_BOX_TESTS] += st[S_BOX_TESTS] - box_before;
            st[S_PRED_LEAF_VISITED] += st[S_LEAF_VISITED] - leaf_before;
            st[S_PRED_TRI_TESTS] += st[S_TRI_TESTS] - tri_before;
        }
        if (positive && hit && !(closest && cmode == C_EXACT)) {
            /* true positive: interior traversal skipped */
            st[S_PRED_HITS]++;
            st[S_NODES_SKIPPED] += skip_depth;
            if (outcome) *outcome = OUT_PRED_HIT;
        } else {
            if (positive && !(closest && cmode == C_EXACT)) st[S_FALSE_POS]++;
            if (outcome) *outcome = positive ? OUT_FALSE_POS : OUT_TRAVERSED;
            uint32_t seed_leaf = b.leaf;
            int found;
            if (closest && cmode == C_EXACT) {
                found = traverse(sc, r, inv, 1, &b, st);
            } else {
                b.t = INFINITY; b.prim = NONE32; b.leaf = NONE32;
                found = traverse(sc, r, inv, closest, &b, st);
            }
            if (closest && cmode == C_EXACT && positive) {
                /* success iff the final best lies in a predicted leaf, or in
                   the subtree of a predicted node */
                int in_pred = 0;
                for (uint32_t s = 0; s < tb->W && slots[s] != NONE32; s++) {
                    uint32_t node = tb->go_up ? slots[s] : sc->leaf_node_by_first[slots[s] >> 3];
                    if (found && sc->sub_lo[node] <= (b.leaf >> 3) && (b.leaf >> 3) < sc->sub_end[node]) in_pred = 1;
                }
                if (in_pred) st[S_PRED_HITS]++; else st[S_FALSE_POS]++;
                if (outcome) *outcome = in_pred ? OUT_PRED_HIT : OUT_FALSE_POS;
                (void)seed_leaf;
            }
            hit = found;
            if (found) {
                rec->has = 1; rec->idx = idx; rec->key = key;
                rec->leaf = tb->go_up ? predicted_node_of(sc, b.leaf, tb->go_up) : b.leaf;
                st[S_RECORDS]++;
            }
        }
    } else {
        hit = traverse(sc, r, inv, closest, &b, st);
        if (outcome) *outcome = OUT_TRAVERSED;
    }
    if (hit) st[S_HITS]++;
    else { b.t = INFINITY; b.u = 0.0f; b.v = 0.0f; b.prim = NONE32; }
write:
    if (occ) *occ = (uint8_t)(b.prim != NONE32);
    if (hit4) {
        if (b.prim == NONE32) { b.t = INFINITY; b.u = 0.0f; b.v = 0.0f; }
        hit4[0] = b.t; hit4[1] = b.u; hit4[2] = b.v; hit4[3] = bits_to_float(b.prim);
    }
}

/* ======================================================================== */
/* Epoch-end update: our batch-synchronous reading of the insertion rule   */
/* of section "HRPP Hash Function" (a conflicting ray's leaf joins the      */
/* existing entry unless already present).  Entries have W slots.  For     */
/* every entry touched by this epoch's records:                            */
/*  1. the owner key: the key of the record with the smallest ray id; with */
/*     the resident policy (bit 1) an entry that holds a tag keeps it, and  */
/*     only its own key's records count.  If the stored tag differs from    */
/*     the owner key, the tag is replaced and all slots emptied;            */
/*  2. records with another key are discarded (conflicts);                 */
/*  3. the owner key's ids not yet present are taken in the order of the  */
/*     smallest ray id that recorded each of them (the smallest ray id wins */
/*     any conflict, so an earlier ray's leaf goes before a later ray's).   */
/*     Without eviction (the paper: no replacement policy, section          */
/*     "Precision and Recall") they fill the empty slots front to back and */
/*     the rest are dropped.  With FIFO eviction (bit 0) the first W of     */
/*     them enter at the back and the oldest slots at the front make room.  */
/*     Every record whose id is absent from the final entry counts a drop.  */
/* The future-work sections ask for a replacement policy; bits 0 and 1 are  */
/* two simple, deterministic ones.                                          */
/* ======================================================================== */
typedef struct { uint32_t idx; uint32_t rid; } rec_ref;
static int rec_ref_cmp(const void *pa, const void *pb)
{
    const rec_ref *a = (const rec_ref *)pa, *b = (const rec_ref *)pb;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return a->rid < b->rid ? -1 : (a->rid > b->rid);
}

static void update_table(table *tb, const record *recs, uint32_t base, uint32_t count, uint64_t *st)
{
    rec_ref *refs = (rec_ref *)malloc(sizeof(rec_ref) * (count ? count : 1));
    uint32_t m = 0;
    for (uint32_t i = 0; i < count; i++) if (recs[i].has) { refs[m].idx = recs[i].idx; refs[m].rid = base + i; m++; }
    qsort(refs, m, sizeof(rec_ref), rec_ref_cmp);
    uint32_t W = tb->W;
    uint32_t *fresh = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    for (uint32_t g = 0; g < m;) {
        uint32_t e = g;
        while (e < m && refs[e].idx == refs[g].idx) e++;
        uint32_t idx = refs[g].idx;
        uint64_t kstar = recs[refs[g].rid - base].key;
        uint32_t *slots = tb->slot + (size_t)idx * W;
        if ((tb->policy & 2u) && tb->tag[idx] != EMPTY_TAG) {
            /* the resident key keeps the entry; other keys' records are conflicts */
            kstar = tb->tag[idx];
        }
        if (tb->tag[idx] != kstar) {
            tb->tag[idx] = kstar;
            for (uint32_t s = 0; s < W; s++) slots[s] = NONE32;
            st[S_TAG_CLAIMS]++;
        }
        uint32_t used = 0;
        while (used < W && slots[used] != NONE32) used++;
        /* distinct owner-key leaves not already present, each at the place
           of the first (smallest ray id) record that names it: the records
           of this entry are visited in increasing ray id */
        uint32_t nf = 0;
        for (uint32_t j = g; j < e; j++) {
            const record *r = &recs[refs[j].rid - base];
            if (r->key != kstar) { st[S_CONFLICTS]++; continue; }
            int present = 0;
            for (uint32_t s = 0; s < used; s++) if (slots[s] == r->leaf) present = 1;
            for (uint32_t f = 0; f < nf; f++) if (fresh[f] == r->leaf) present = 1;
            if (!present) fresh[nf++] = r->leaf;
        }
        if (tb->policy & 1u) {
            /* FIFO: the oldest (front) slots make room for the first W new ids */
            uint32_t take = nf < W ? nf : W;
            uint32_t evict = used + take > W ? used + take - W : 0;
            for (uint32_t s = 0; s + evict < used; s++) slots[s] = slots[s + evict];
            used -= evict;
            st[S_EVICTIONS] += evict;
            for (uint32_t f = 0; f < take; f++) { slots[used++] = fresh[f]; st[S_LEAF_INSERTS]++; }
            for (uint32_t s = used; s < W; s++) slots[s] = NONE32;
        } else {
            for (uint32_t f = 0; f < nf && used < W; f++) { slots[used++] = fresh[f]; st[S_LEAF_INSERTS]++; }
        }
        for (uint32_t j = g; j < e; j++) {
            const record *r = &recs[refs[j].rid - base];
            if (r->key != kstar) continue;
            int present = 0;
            for (uint32_t s = 0; s < used; s++) if (slots[s] == r->leaf) present = 1;
            if (!present) st[S_DROPPED]++;
        }
        g = e;
    }
    free(refs);
    free(fresh);
}

/* ======================================================================== */
/* Entry point                                                              */
/* ======================================================================== */

/* Trace n rays.  query: 0 any-hit, 1 closest.  cmode: 0 PAPER, 1 EXACT
   (closest only).  tags/slots NULL = plain traversal, otherwise the table
   (log2n entries of W slots) is read and updated in place, epochs of
   `epoch` rays in ray order, the first of them `first_epoch` rays long
   (0: `epoch`; at most `epoch`).  occ (n bytes) or hits (4 floats per ray: t,
   u, v, prim bits) receive the results; stats (STATS_SLOTS uint64) are
   accumulated; outcome (n bytes, optional) receives 0 invalid, 1 traversed
   without a positive prediction, 2 prediction hit, 3 false positive.
   nthreads <= 0 uses the OpenMP default.  Returns 0, or -1
   on bad arguments. */
int orc_trace(const orc_bvh *bvh, const float *vtx, const float *rays, uint32_t n, int query, int cmode,
              uint64_t *tags, uint32_t *slots, uint32_t log2n, uint32_t W, uint32_t qo, uint32_t qd,
              uint32_t epoch, uint8_t *occ, float *hits, uint64_t *stats, uint8_t *outcome, int nthreads,
              uint32_t hash_mode, uint32_t go_up, uint32_t policy, uint32_t first_epoch)
{
    if (!bvh || bvh->num_nodes == 0) return -1;
    if (tags && first_epoch > epoch) return -1;
    if (tags && (W < 1 || log2n < 1 || log2n > 31 || qo < 1 || qo > 10 || qd < 1 || qd > 10 || epoch < 1)) return -1;
    if (tags && (hash_mode > 1 || (hash_mode == 1 && (qo > 7 || qd != qo)))) return -1;
    if (tags && (go_up > 64 || policy > 3)) return -1;
    scene sc;
    sc.bvh = bvh;
    sc.vtx = vtx;
    uint32_t m = bvh->num_nodes;
    uint32_t *lnode = (uint32_t *)malloc(sizeof(uint32_t) * (bvh->num_tris + 1));
    uint32_t *parent = (uint32_t *)malloc(sizeof(uint32_t) * m);
    uint32_t *sub_lo = (uint32_t *)malloc(sizeof(uint32_t) * m);
    uint32_t *sub_end = (uint32_t *)malloc(sizeof(uint32_t) * m);
    for (uint32_t i = 0; i < m; i++) parent[i] = NONE32;
    for (uint32_t i = 0; i < m; i++) {
        if (bvh->right[i] == NONE32) lnode[bvh->first[i]] = i;
        else { parent[i + 1] = i; parent[bvh->right[i]] = i; }
    }
    /* children follow their parent in pre-order: a reverse sweep sees them first */
    for (uint32_t i = m; i-- > 0;) {
        if (bvh->right[i] == NONE32) { sub_lo[i] = bvh->first[i]; sub_end[i] = bvh->first[i] + bvh->count[i]; }
        else {
            uint32_t L = i + 1, R = bvh->right[i];
            sub_lo[i] = sub_lo[L] < sub_lo[R] ? sub_lo[L] : sub_lo[R];
            sub_end[i] = sub_end[L] > sub_end[R] ? sub_end[L] : sub_end[R];
        }
    }
    sc.leaf_node_by_first = lnode;
    sc.parent = parent;
    sc.sub_lo = sub_lo;
    sc.sub_end = sub_end;
    table tb, *ptb = NULL;
    if (tags) {
        tb.tag = tags; tb.slot = slots; tb.W = W; tb.go_up = go_up; tb.policy = policy;
        hash_setup(&tb.h, bvh->box, qo, qd, log2n);
        tb.h.mode = hash_mode;
        ptb = &tb;
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
    uint32_t E = ptb ? epoch : (n ? n : 1);
    uint32_t F = (ptb && first_epoch) ? first_epoch : E;   /* the first epoch's length */
    record *recs = (record *)malloc(sizeof(record) * (size_t)(E < n ? E : (n ? n : 1)));
    for (uint32_t base = 0; base < n;) {
        uint32_t len = base == 0 ? F : E;
        uint32_t cnt = (n - base < len) ? n - base : len;
        uint64_t acc[STATS_SLOTS];
        memset(acc, 0, sizeof acc);
        #pragma omp parallel
        {
            uint64_t loc[STATS_SLOTS];
            memset(loc, 0, sizeof loc);
            #pragma omp for schedule(dynamic, 256)
            for (uint32_t i = 0; i < cnt; i++) {
                uint32_t rid = base + i;
                trace_one(&sc, ptb, rays + 8 * (size_t)rid, query, cmode, occ ? occ + rid : NULL,
                          hits ? hits + 4 * (size_t)rid : NULL, &recs[i], outcome ? outcome + rid : NULL, loc);
            }
            #pragma omp critical
            for (int s = 0; s < STATS_SLOTS; s++) acc[s] += loc[s];
        }
        if (ptb) update_table(ptb, recs, base, cnt, acc);
        for (int s = 0; s < STATS_SLOTS; s++) stats[s] += acc[s];
        base += cnt;
    }
    free(recs);
    free(lnode);
    free(parent);
    free(sub_lo);
    free(sub_end);
    return 0;
}

/* Brute force over all triangles (original order), same binary32 test:
   the plain definition of the any-hit flag and of the exact closest hit
   (lexicographic (t, prim) minimum inside (tmin, tmax)). */
void orc_brute_force(const float *tris, uint32_t ntri, const float *rays, uint32_t n, int closest,
                     uint8_t *occ, float *hits, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 64)
    for (uint32_t i = 0; i < n; i++) {
        const float *r = rays + 8 * (size_t)i;
        float bt = INFINITY, bu = 0.0f, bv = 0.0f;
        uint32_t bp = NONE32;
        if (ray_valid(r)) {
            for (uint32_t k = 0; k < ntri; k++) {
                const float *v = tris + 9 * (size_t)k;
                float t, u, w;
                if (!moller_trumbore(v, v + 3, v + 6, r, r + 4, &t, &u, &w)) continue;
                if (!(r[3] < t && t < r[7])) continue;
                if (t < bt || (t == bt && k < bp)) { bt = t; bu = u; bv = w; bp = k; if (!closest) break; }
            }
        }
        if (occ) occ[i] = (uint8_t)(bp != NONE32);
        if (hits) {
            if (bp == NONE32 || !closest) { if (bp == NONE32) { bt = INFINITY; bu = 0.0f; bv = 0.0f; } }
            hits[4 * (size_t)i] = bt; hits[4 * (size_t)i + 1] = bu; hits[4 * (size_t)i + 2] = bv;
            hits[4 * (size_t)i + 3] = bits_to_float(bp);
        }
    }
}

uint32_t orc_float_bits(float f) { return float_to_bits(f); }
