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

}  // namespace

hrpp_status build_sah_tree(const float *verts, uint32_t n, const hrpp_bvh_desc &desc, CanonTree &out) {
    if (!verts || n == 0 || n >= (1u << 28)) return HRPP_EINVAL;
    if (desc.leaf_max < 1 || desc.leaf_max > 8 || desc.sah_bins < 2 || desc.sah_bins > 256 ||
        desc.max_depth < 1 || desc.max_depth > (uint32_t)kMaxDepth)
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
    return HRPP_OK;
}

}  // namespace hrpp
