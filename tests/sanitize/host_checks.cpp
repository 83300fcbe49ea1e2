// Host-only checks of the library's CPU code -- the binned-SAH builder, the
// 4-wide collapse and the serving pool allocator -- for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
// Exits non-zero on the first broken invariant; the sanitizers abort on the
// first memory or undefined-behaviour error.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hrpp_internal.h"
#include "pool_alloc.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what, uint32_t n, uint32_t leaf_max) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (n=%u, leaf_max=%u)\n", what, n, leaf_max);
        failures++;
    }
}

// Random triangle soup in the unit cube, with degenerate variants.
std::vector<float> scene(std::mt19937 &g, uint32_t n, int kind) {
    std::uniform_real_distribution<float> u(0.0f, 1.0f);
    std::vector<float> v(9 * (size_t)n);
    for (uint32_t i = 0; i < n; i++) {
        const float cx = u(g), cy = u(g), cz = u(g);
        for (int k = 0; k < 3; k++) {
            float *p = &v[9 * (size_t)i + 3 * k];
            p[0] = cx + 0.05f * (u(g) - 0.5f);
            p[1] = cy + 0.05f * (u(g) - 0.5f);
            p[2] = cz + 0.05f * (u(g) - 0.5f);
            if (kind == 1) p[1] = 0.25f;                       // a flat axis
            if (kind == 2) { p[0] = cx; p[1] = cy; p[2] = cz; } // point triangles
        }
        if (kind == 3 && i > 0)                                  // every triangle the same
            for (int k = 0; k < 9; k++) v[9 * (size_t)i + k] = v[k];
    }
    return v;
}

void check_tree(const std::vector<float> &v, uint32_t n, uint32_t leaf_max, uint32_t passes = 0) {
    hrpp_bvh_desc d{leaf_max, 32, 64, passes};
    hrpp::CanonTree t;
    const hrpp_status st = hrpp::build_sah_tree(v.data(), n, d, t);
    if (st == HRPP_EDEPTH) return;
    expect(st == HRPP_OK, "build status", n, leaf_max);
    if (st != HRPP_OK) return;
    const size_t m = t.right.size();
    expect(t.box.size() == 6 * m && t.first.size() == m && t.count.size() == m && t.depth.size() == m,
           "array sizes", n, leaf_max);
    expect(t.perm.size() == n, "perm size", n, leaf_max);
    std::vector<uint8_t> seen(n, 0);
    for (uint32_t p : t.perm) {
        expect(p < n && !seen[p], "perm is a permutation", n, leaf_max);
        if (p < n) seen[p] = 1;
    }
    // leaves in depth-first order tile [0, n)
    uint32_t next = 0;
    for (size_t i = 0; i < m; i++) {
        if (t.right[i] != hrpp::kNone) {
            expect(t.right[i] > i + 1 && t.right[i] < m, "right child after the left subtree", n, leaf_max);
            if (t.right[i] < m)
                for (int a = 0; a < 3; a++) {
                    const float *l = &t.box[6 * (i + 1)], *r = &t.box[6 * (size_t)t.right[i]], *b = &t.box[6 * i];
                    expect(b[a] == std::min(l[a], r[a]) && b[3 + a] == std::max(l[3 + a], r[3 + a]),
                           "interior box is the union of its children", n, leaf_max);
                }
            continue;
        }
        expect(t.count[i] >= 1 && t.count[i] <= leaf_max, "leaf size", n, leaf_max);
        expect(t.first[i] == next, "leaves in order", n, leaf_max);
        next = t.first[i] + t.count[i];
        for (uint32_t k = t.first[i]; k < next && k < n; k++) {
            const float *tri = &v[9 * (size_t)t.perm[k]];
            for (int c = 0; c < 9; c++)
                expect(tri[c] >= t.box[6 * i + c % 3] && tri[c] <= t.box[6 * i + 3 + c % 3], "leaf box holds its triangles",
                       n, leaf_max);
        }
        expect(t.depth[i] <= t.max_depth, "depth bound", n, leaf_max);
    }
    expect(next == n, "leaves cover every triangle", n, leaf_max);
    hrpp::WideTree w;
    hrpp::collapse_wide(t, w);
    expect(w.words.size() % 32 == 0, "wide node records", n, leaf_max);
    const size_t wn = w.words.size() / 32;
    uint32_t leaves = 0;
    for (size_t i = 0; i < wn; i++)
        for (int k = 0; k < 4; k++) {
            const uint32_t ref = w.words[32 * i + 24 + k];
            if (ref == hrpp::kNone) continue;
            if (ref & hrpp::kLeafFlag) leaves++;
            else expect(ref > i && ref < wn, "wide child after its parent", n, leaf_max);
        }
    uint32_t binary_leaves = 0;
    for (size_t i = 0; i < m; i++) binary_leaves += t.right[i] == hrpp::kNone;
    if (m > 1) expect(leaves == binary_leaves, "wide tree keeps every leaf", n, leaf_max);
}

void check_pool(std::mt19937 &g) {
    const size_t size = 1u << 20;
    hrpp::PoolAllocator pool(size);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    std::uniform_int_distribution<size_t> len(1, 40000);
    for (int step = 0; step < 20000; step++) {
        if (live.empty() || g() % 3 != 0) {
            const size_t b = len(g);
            size_t off = 0;
            if (pool.alloc(b, off)) {
                const size_t ab = hrpp::align256(b);
                expect(off % 256 == 0 && off + ab <= size, "allocation inside the pool", (uint32_t)b, 0);
                for (const Live &l : live)
                    expect(off + ab <= l.off || l.off + hrpp::align256(l.bytes) <= off, "no overlap", (uint32_t)b, 0);
                live.push_back({off, b});
            }
        } else {
            const size_t k = g() % live.size();
            pool.release(live[k].off, live[k].bytes);
            live[k] = live.back();
            live.pop_back();
        }
        size_t used = 0;
        for (const Live &l : live) used += hrpp::align256(l.bytes);
        expect(pool.used() == used, "used bytes", (uint32_t)live.size(), 0);
    }
    for (const Live &l : live) pool.release(l.off, l.bytes);
    size_t off = 0;
    expect(pool.used() == 0 && pool.alloc(size, off) && off == 0, "free ranges merge back into one", 0, 0);
}

}  // namespace

int main() {
    std::mt19937 g(12345);
    const uint32_t sizes[] = {1, 2, 3, 5, 8, 17, 64, 255, 1000, 4097};
    for (uint32_t n : sizes)
        for (uint32_t leaf_max = 1; leaf_max <= 8; leaf_max++)
            for (int kind = 0; kind < 4; kind++) check_tree(scene(g, n, kind), n, leaf_max);
    // the same checks after treelet restructuring
    for (uint32_t n : sizes)
        for (uint32_t leaf_max : {1u, 2u, 4u})
            for (uint32_t passes = 1; passes <= 3; passes++)
                for (int kind = 0; kind < 4; kind++) check_tree(scene(g, n, kind), n, leaf_max, passes);
    check_pool(g);
    // invalid input is refused, not read out of bounds
    {
        std::vector<float> v = scene(g, 10, 0);
        v[13] = 1.0f / 0.0f;
        hrpp_bvh_desc d{4, 32, 64};
        hrpp::CanonTree t;
        expect(hrpp::build_sah_tree(v.data(), 10, d, t) == HRPP_EINVAL, "non-finite vertex refused", 10, 4);
    }
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
