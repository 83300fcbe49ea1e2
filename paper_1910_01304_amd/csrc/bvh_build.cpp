// Host BVH builder of the HRPP library: deterministic binned-SAH binary tree.
//
// The paper takes the binary BVH as given (section "Overview": a unified
// binary BVH whose interior nodes hold boxes and whose leaves hold
// triangles).  This builder fixes one deterministic construction so that
// every consumer of the tree (GPU layout, predictor leaf ids, counters) is
// reproducible:
//   * triangle bounds are the binary32 min/max of the three vertices and the
//     centroid is (min + max) * 0.5 in binary32;
//   * a node over more than leaf_max triangles is split by binned SAH on the
//     centroid bounds: per axis with positive, finitely invertible extent,
//     k = bins / extent, bin(c) = min(bins - 1, trunc((c - cmin) * k)); split
//     s (1 <= s < bins) costs A(left) * |left| + A(right) * |right| with A the
//     half surface area evaluated in double; the smallest cost wins, ties to
//     the lower axis and then the lower s; splits with an empty side are
//     skipped;
//   * if no axis qualifies (all centroids coincide) the range is halved;
//   * the partition is stable (original relative order kept on each side);
//   * nodes are numbered in depth-first pre-order, left subtree first.
// Optionally (desc.treelet_passes) the interior nodes are then rearranged by
// treelet restructuring (Karras and Aila, HPG 2013), with the rules the
// device builder applies to its linear BVH: a pass takes every interior node
// after all interior nodes below it; its treelet grows from its two children
// by opening the interior treelet leaf of largest half area (the first on
// ties; the left child takes its place, the right child goes last) up to 7
// leaves; the topology minimising the sum of interior half areas (binary32,
// by dynamic programming over leaf subsets, partitions tried in increasing
// bitmask order with the part holding the lowest leaf on the left, the first
// minimum kept) replaces the current one only when strictly cheaper, the
// root keeping its identity and the opened nodes taking the new interior
// positions in pre-order.  Boxes of rebuilt nodes are the union of their
// children's (the left child's value kept on ties); leaves do not change.
#include <array>
#include <cmath>
#include <cstring>
#include <limits>

#include "hrpp_internal.h"

namespace hrpp {
namespace {

struct Builder {
    const hrpp_bvh_desc &desc;
    std::vector<float> tb;        // 6 per triangle
    std::vector<float> tc;        // 3 per triangle
    std::vector<uint32_t> idx;
    std::vector<uint32_t> scratch;
    CanonTree &out;
    bool too_deep = false;

    // per-bin accumulators (reused)
    std::vector<uint32_t> cnt;
    std::vector<float> bmn, bmx, lmn, lmx, rmn, rmx;
    std::vector<uint32_t> lcount, rcount;

    Builder(const hrpp_bvh_desc &d, CanonTree &o) : desc(d), out(o) {}

    static double half_area(const float *mn, const float *mx) {
        double dx = (double)mx[0] - (double)mn[0];
        double dy = (double)mx[1] - (double)mn[1];
        double dz = (double)mx[2] - (double)mn[2];
        return dx * dy + dy * dz + dz * dx;
    }

    static inline uint32_t bin_index(float c, float cmin, float k, uint32_t bins) {
        uint32_t b = (uint32_t)((c - cmin) * k);
        return b > bins - 1 ? bins - 1 : b;
    }

    uint32_t node(uint32_t begin, uint32_t end, uint32_t depth) {
        const uint32_t id = (uint32_t)out.right.size();
        out.right.push_back(kNone);
        out.first.push_back(0);
        out.count.push_back(0);
        out.depth.push_back(depth);
        for (int a = 0; a < 6; a++) out.box.push_back(0.0f);

        const float inf = std::numeric_limits<float>::infinity();
        float mn[3] = {inf, inf, inf}, mx[3] = {-inf, -inf, -inf};
        float cmn[3] = {inf, inf, inf}, cmx[3] = {-inf, -inf, -inf};
        for (uint32_t i = begin; i < end; i++) {
            const float *b = &tb[6 * (size_t)idx[i]];
            const float *c = &tc[3 * (size_t)idx[i]];
            for (int a = 0; a < 3; a++) {
                if (b[a] < mn[a]) mn[a] = b[a];
                if (b[a + 3] > mx[a]) mx[a] = b[a + 3];
                if (c[a] < cmn[a]) cmn[a] = c[a];
                if (c[a] > cmx[a]) cmx[a] = c[a];
            }
        }
        for (int a = 0; a < 3; a++) {
            out.box[6 * (size_t)id + a] = mn[a];
            out.box[6 * (size_t)id + 3 + a] = mx[a];
        }
        const uint32_t n = end - begin;
        if (n <= desc.leaf_max || depth + 1 > desc.max_depth) {
            if (n > desc.leaf_max) too_deep = true;
            out.first[id] = begin;
            out.count[id] = n;
            if (depth > out.max_depth) out.max_depth = depth;
            return id;
        }

        const uint32_t B = desc.sah_bins;
        double best = inf;
        int best_axis = -1;
        uint32_t best_split = 0;
        float best_k = 0.0f;
        for (int a = 0; a < 3; a++) {
            float extent = cmx[a] - cmn[a];
            if (!(extent > 0.0f)) continue;
            float k = (float)B / extent;
            if (!std::isfinite(k)) continue;
            std::fill(cnt.begin(), cnt.end(), 0u);
            std::fill(bmn.begin(), bmn.end(), inf);
            std::fill(bmx.begin(), bmx.end(), -inf);
            for (uint32_t i = begin; i < end; i++) {
                const uint32_t t = idx[i];
                const uint32_t j = bin_index(tc[3 * (size_t)t + a], cmn[a], k, B);
                const float *b = &tb[6 * (size_t)t];
                cnt[j]++;
                float *pmn = &bmn[3 * j], *pmx = &bmx[3 * j];
                for (int q = 0; q < 3; q++) {
                    if (b[q] < pmn[q]) pmn[q] = b[q];
                    if (b[q + 3] > pmx[q]) pmx[q] = b[q + 3];
                }
            }
            // prefix (left of split s = bins [0, s)) and suffix (right = [s, B)) unions
            float accmn[3] = {inf, inf, inf}, accmx[3] = {-inf, -inf, -inf};
            uint32_t acc = 0;
            for (uint32_t s = 1; s < B; s++) {
                const uint32_t j = s - 1;
                acc += cnt[j];
                for (int q = 0; q < 3; q++) {
                    if (bmn[3 * j + q] < accmn[q]) accmn[q] = bmn[3 * j + q];
                    if (bmx[3 * j + q] > accmx[q]) accmx[q] = bmx[3 * j + q];
                    lmn[3 * s + q] = accmn[q];
                    lmx[3 * s + q] = accmx[q];
                }
                lcount[s] = acc;
            }
            for (int q = 0; q < 3; q++) { accmn[q] = inf; accmx[q] = -inf; }
            acc = 0;
            for (uint32_t s = B - 1; s >= 1; s--) {
                acc += cnt[s];
                for (int q = 0; q < 3; q++) {
                    if (bmn[3 * s + q] < accmn[q]) accmn[q] = bmn[3 * s + q];
                    if (bmx[3 * s + q] > accmx[q]) accmx[q] = bmx[3 * s + q];
                    rmn[3 * s + q] = accmn[q];
                    rmx[3 * s + q] = accmx[q];
                }
                rcount[s] = acc;
            }
            for (uint32_t s = 1; s < B; s++) {
                if (lcount[s] == 0 || rcount[s] == 0) continue;
                double cost = half_area(&lmn[3 * s], &lmx[3 * s]) * (double)lcount[s] +
                              half_area(&rmn[3 * s], &rmx[3 * s]) * (double)rcount[s];
                if (cost < best) { best = cost; best_axis = a; best_split = s; best_k = k; }
            }
        }

        uint32_t mid;
        if (best_axis < 0) {
            mid = begin + n / 2;
        } else {
            uint32_t w = begin, r = 0;
            const float cm = cmn[best_axis];
            for (uint32_t i = begin; i < end; i++) {
                const uint32_t t = idx[i];
                if (bin_index(tc[3 * (size_t)t + best_axis], cm, best_k, B) < best_split) idx[w++] = t;
                else scratch[r++] = t;
            }
            std::memcpy(&idx[w], scratch.data(), sizeof(uint32_t) * r);
            mid = w;
        }
        node(begin, mid, depth + 1);
        const uint32_t rc = node(mid, end, depth + 1);
        out.right[id] = rc;
        return id;
    }
};

// ---- treelet restructuring -------------------------------------------------

constexpr uint32_t kTreeletLeaves = 7;

// The tree with explicit children, for rearranging.
struct LinkedTree {
    std::vector<uint32_t> lc, rc;        // children; rc = kNone for a leaf
    std::vector<uint32_t> first, count;  // leaf triangles, in the input tree's order
    std::vector<float> box;              // 6 per node
    bool is_leaf(uint32_t v) const { return rc[v] == kNone; }
    float *bx(uint32_t v) { return &box[6 * (size_t)v]; }
};

inline float half_area32(const float *b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

// o = union of a and b; a's value is kept where they are equal.
inline void box_union(const float *a, const float *b, float *o) {
    float t[6];
    for (int k = 0; k < 3; k++) {
        t[k] = b[k] < a[k] ? b[k] : a[k];
        t[3 + k] = b[3 + k] > a[3 + k] ? b[3 + k] : a[3 + k];
    }
    std::memcpy(o, t, sizeof t);
}

void optimize_treelet(LinkedTree &t, uint32_t root) {
    std::array<uint32_t, kTreeletLeaves> leaf{};
    std::array<uint32_t, kTreeletLeaves - 1> opened{};
    uint32_t nl = 2, no = 1;
    leaf[0] = t.lc[root];
    leaf[1] = t.rc[root];
    opened[0] = root;
    for (; nl < kTreeletLeaves; nl++) {
        uint32_t pick = kNone;
        float pa = 0.0f;
        for (uint32_t i = 0; i < nl; i++) {
            if (t.is_leaf(leaf[i])) continue;
            const float a = half_area32(t.bx(leaf[i]));
            if (pick == kNone || a > pa) { pick = i; pa = a; }
        }
        if (pick == kNone) break;
        const uint32_t x = leaf[pick];
        opened[no++] = x;
        leaf[pick] = t.lc[x];
        leaf[nl] = t.rc[x];
    }
    if (nl < 3) return;
    const uint32_t all = (1u << nl) - 1u;
    std::array<float, 1u << kTreeletLeaves> area{}, best{};
    std::array<uint32_t, 1u << kTreeletLeaves> split{};
    for (uint32_t set = 1; set <= all; set++) {
        float u[6];
        bool started = false;
        for (uint32_t i = 0; i < nl; i++) {
            if (!(set & (1u << i))) continue;
            if (!started) { std::memcpy(u, t.bx(leaf[i]), sizeof u); started = true; }
            else box_union(u, t.bx(leaf[i]), u);
        }
        area[set] = half_area32(u);
    }
    // sets in increasing order: every proper subset comes first
    for (uint32_t set = 1; set <= all; set++) {
        if ((set & (set - 1u)) == 0u) continue;           // one leaf: cost 0
        const uint32_t lowest = set & (0u - set);
        uint32_t arg = 0;
        float m = 0.0f;
        for (uint32_t part = lowest; part != set; part = (part - set) & set) {
            if (!(part & lowest)) continue;
            const float c = best[part] + best[set ^ part];
            if (arg == 0 || c < m) { m = c; arg = part; }
        }
        best[set] = area[set] + m;
        split[set] = arg;
    }
    // the current topology's cost, children (opened later) first
    std::array<uint32_t, kTreeletLeaves - 1> set_of{};
    std::array<float, kTreeletLeaves - 1> cur{};
    for (uint32_t j = no; j-- > 0;) {
        const uint32_t kids[2] = {t.lc[opened[j]], t.rc[opened[j]]};
        uint32_t s2 = 0;
        float c2[2] = {0.0f, 0.0f};
        for (int k = 0; k < 2; k++) {
            for (uint32_t i = 0; i < nl; i++)
                if (leaf[i] == kids[k]) s2 |= 1u << i;
            for (uint32_t q = j + 1; q < no; q++)
                if (opened[q] == kids[k]) { s2 |= set_of[q]; c2[k] = cur[q]; }
        }
        set_of[j] = s2;
        cur[j] = area[s2] + (c2[0] + c2[1]);
    }
    if (!(best[all] < cur[0])) return;
    // identities in pre-order of the new topology; then links and boxes,
    // children before parents
    std::array<uint32_t, 1u << kTreeletLeaves> node_of{};
    std::array<uint32_t, kTreeletLeaves - 1> pre{};
    std::array<uint32_t, kTreeletLeaves> todo{};
    uint32_t ntodo = 0, npre = 0, next = 1;
    todo[ntodo++] = all;
    while (ntodo) {
        const uint32_t set = todo[--ntodo];
        node_of[set] = set == all ? root : opened[next++];
        pre[npre++] = set;
        const uint32_t a = split[set], b = set ^ a;
        if (b & (b - 1u)) todo[ntodo++] = b;
        if (a & (a - 1u)) todo[ntodo++] = a;
    }
    auto node = [&](uint32_t set) {
        return (set & (set - 1u)) ? node_of[set] : leaf[__builtin_ctz(set)];
    };
    for (uint32_t k = npre; k-- > 0;) {
        const uint32_t set = pre[k];
        const uint32_t v = node_of[set], l = node(split[set]), r = node(set ^ split[set]);
        t.lc[v] = l;
        t.rc[v] = r;
        box_union(t.bx(l), t.bx(r), t.bx(v));
    }
}

// Interior nodes in post-order (children before parents), root 0.
std::vector<uint32_t> interior_post_order(const LinkedTree &t) {
    std::vector<uint32_t> out, stack{0};
    std::vector<uint8_t> expanded(t.rc.size(), 0);
    while (!stack.empty()) {
        const uint32_t v = stack.back();
        if (t.is_leaf(v)) { stack.pop_back(); continue; }
        if (expanded[v]) { out.push_back(v); stack.pop_back(); continue; }
        expanded[v] = 1;
        stack.push_back(t.rc[v]);
        stack.push_back(t.lc[v]);
    }
    return out;
}

// Rewrite `tree` after `passes` passes; EDEPTH when the result is deeper
// than max_depth.
hrpp_status treelet_passes(CanonTree &tree, uint32_t passes, uint32_t max_depth) {
    const uint32_t m = (uint32_t)tree.right.size();
    LinkedTree t;
    t.rc = tree.right;
    t.lc.resize(m);
    for (uint32_t v = 0; v < m; v++) t.lc[v] = tree.right[v] == kNone ? kNone : v + 1;
    t.first = tree.first;
    t.count = tree.count;
    t.box = tree.box;
    for (uint32_t p = 0; p < passes; p++)
        for (uint32_t v : interior_post_order(t)) optimize_treelet(t, v);
    // depth-first pre-order, triangles in leaf order
    CanonTree out;
    out.box.reserve(tree.box.size());
    out.right.reserve(m); out.first.reserve(m); out.count.reserve(m); out.depth.reserve(m);
    out.perm.reserve(tree.perm.size());
    std::vector<std::pair<uint32_t, uint32_t>> stack{{0u, 0u}};   // (node, depth)
    std::vector<std::pair<uint32_t, uint32_t>> fix;                // (output node, right child input id)
    std::vector<uint32_t> out_id(m, kNone);
    while (!stack.empty()) {
        const auto [v, d] = stack.back();
        stack.pop_back();
        const uint32_t id = (uint32_t)out.right.size();
        out_id[v] = id;
        out.box.insert(out.box.end(), t.bx(v), t.bx(v) + 6);
        out.depth.push_back(d);
        out.right.push_back(kNone);
        if (t.is_leaf(v)) {
            out.first.push_back((uint32_t)out.perm.size());
            out.count.push_back(t.count[v]);
            for (uint32_t k = 0; k < t.count[v]; k++) out.perm.push_back(tree.perm[t.first[v] + k]);
            if (d > out.max_depth) out.max_depth = d;
        } else {
            out.first.push_back(0);
            out.count.push_back(0);
            fix.push_back({id, t.rc[v]});
            stack.push_back({t.rc[v], d + 1});
            stack.push_back({t.lc[v], d + 1});
        }
    }
    for (const auto &f : fix) out.right[f.first] = out_id[f.second];
    if (out.right.size() != m || out.perm.size() != tree.perm.size()) return HRPP_EINVAL;
    if (out.max_depth > max_depth) return HRPP_EDEPTH;
    tree = std::move(out);
    return HRPP_OK;
}

}  // namespace

hrpp_status build_sah_tree(const float *verts, uint32_t n, const hrpp_bvh_desc &desc, CanonTree &out) {
    if (!verts || n == 0 || n >= (1u << 28)) return HRPP_EINVAL;
    if (desc.leaf_max < 1 || desc.leaf_max > 8 || desc.sah_bins < 2 || desc.sah_bins > 256 ||
        desc.max_depth < 1 || desc.max_depth > (uint32_t)kMaxDepth || desc.treelet_passes > kMaxTreeletPasses)
        return HRPP_EINVAL;
    for (size_t i = 0; i < 9 * (size_t)n; i++)
        if (!std::isfinite(verts[i])) return HRPP_EINVAL;

    Builder b(desc, out);
    b.tb.resize(6 * (size_t)n);
    b.tc.resize(3 * (size_t)n);
    b.idx.resize(n);
    b.scratch.resize(n);
    const uint32_t B = desc.sah_bins;
    b.cnt.resize(B);
    b.bmn.resize(3 * B); b.bmx.resize(3 * B);
    b.lmn.resize(3 * B); b.lmx.resize(3 * B);
    b.rmn.resize(3 * B); b.rmx.resize(3 * B);
    b.lcount.resize(B); b.rcount.resize(B);
    for (uint32_t t = 0; t < n; t++) {
        const float *v = verts + 9 * (size_t)t;
        for (int a = 0; a < 3; a++) {
            float lo = v[a], hi = v[a];
            if (v[3 + a] < lo) lo = v[3 + a];
            if (v[6 + a] < lo) lo = v[6 + a];
            if (v[3 + a] > hi) hi = v[3 + a];
            if (v[6 + a] > hi) hi = v[6 + a];
            b.tb[6 * (size_t)t + a] = lo;
            b.tb[6 * (size_t)t + 3 + a] = hi;
            b.tc[3 * (size_t)t + a] = (lo + hi) * 0.5f;
        }
        b.idx[t] = t;
    }
    out = CanonTree();
    const size_t reserve = 2 * (size_t)n;
    out.right.reserve(reserve); out.first.reserve(reserve); out.count.reserve(reserve);
    out.depth.reserve(reserve); out.box.reserve(6 * reserve);
    b.node(0, n, 0);
    if (b.too_deep) return HRPP_EDEPTH;
    out.perm = std::move(b.idx);
    if (desc.treelet_passes) return treelet_passes(out, desc.treelet_passes, desc.max_depth);
    return HRPP_OK;
}

}  // namespace hrpp
