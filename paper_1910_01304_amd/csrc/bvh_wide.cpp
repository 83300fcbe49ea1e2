// 4-wide BVH for the plain-traversal baseline, collapsed from the binary
// SAH tree (a stronger plain baseline than binary traversal; the method
// itself predicts nodes of the binary tree).
//
// Collapse: a wide node starts from the two children of a binary interior
// node and, while it has fewer than 4 children, replaces its interior child
// of largest surface area (half area in double; ties to the earlier child)
// by that child's two children, in place.  Leaves stay the binary tree's
// leaves.  Wide nodes are numbered in depth-first pre-order.
//
// Node record, 32 words (128 B):
//   [0..3] min x of children 0..3   [4..7] max x   [8..11] min y  [12..15] max y
//   [16..19] min z                  [20..23] max z [24..27] child references
//   [28..31] zero
// A reference is a wide node index, kLeafFlag | leaf id, or kNone (no child).
#include <algorithm>
#include <cstring>

#include "hrpp_internal.h"

namespace hrpp {
namespace {

struct Collapser {
    const CanonTree &t;
    WideTree &w;

    double half_area(uint32_t i) const {
        const float *b = &t.box[6 * (size_t)i];
        const double dx = (double)b[3] - b[0], dy = (double)b[4] - b[1], dz = (double)b[5] - b[2];
        return dx * dy + dy * dz + dz * dx;
    }

    bool leaf(uint32_t i) const { return t.right[i] == kNone; }

    uint32_t leaf_ref(uint32_t i) const { return kLeafFlag | (t.first[i] << 3) | (t.count[i] - 1u); }

    // Emits the wide node over binary interior node i; returns its index and
    // the largest number of stack entries a traversal below it can hold.
    uint32_t emit(uint32_t i, uint32_t &need, uint32_t &depth) {
        uint32_t ch[4] = {i + 1, t.right[i], kNone, kNone};
        uint32_t n = 2;
        while (n < 4) {
            int pick = -1;
            double best = -1.0;
            for (uint32_t k = 0; k < n; k++) {
                if (leaf(ch[k])) continue;
                const double a = half_area(ch[k]);
                if (a > best) { best = a; pick = (int)k; }
            }
            if (pick < 0) break;
            const uint32_t c = ch[pick];
            for (uint32_t k = n; k > (uint32_t)pick + 1; k--) ch[k] = ch[k - 1];
            ch[pick] = c + 1;
            ch[pick + 1] = t.right[c];
            n++;
        }
        const uint32_t id = (uint32_t)(w.words.size() / 32);
        w.words.resize(w.words.size() + 32, 0u);
        uint32_t sub_need = 0, sub_depth = 0;
        for (uint32_t k = 0; k < 4; k++) {
            uint32_t ref = kNone;
            float box[6] = {0, 0, 0, 0, 0, 0};
            if (k < n) {
                std::memcpy(box, &t.box[6 * (size_t)ch[k]], sizeof box);
                if (leaf(ch[k])) {
                    ref = leaf_ref(ch[k]);
                } else {
                    uint32_t cn = 0, cd = 0;
                    ref = emit(ch[k], cn, cd);
                    sub_need = std::max(sub_need, cn);
                    sub_depth = std::max(sub_depth, cd);
                }
            }
            uint32_t *p = &w.words[(size_t)id * 32];
            const int order[6] = {0, 3, 1, 4, 2, 5};   // min x, max x, min y, max y, min z, max z
            for (int a = 0; a < 6; a++) std::memcpy(&p[4 * a + k], &box[order[a]], 4);
            p[24 + k] = ref;
        }
        need = (n - 1) + sub_need;      // every child hit: n - 1 pushed, one taken
        depth = 1 + sub_depth;
        return id;
    }
};

}  // namespace

void collapse_wide(const CanonTree &t, WideTree &w) {
    w.words.clear();
    w.stack_need = 1;
    w.depth = 0;
    if (t.right.empty()) return;
    if (t.right[0] == kNone) {
        w.root_ref = kLeafFlag | (t.first[0] << 3) | (t.count[0] - 1u);
        return;
    }
    Collapser c{t, w};
    uint32_t need = 0, depth = 0;
    w.root_ref = c.emit(0, need, depth);
    w.stack_need = std::max(1u, need);
    w.depth = depth;
}

}  // namespace hrpp
