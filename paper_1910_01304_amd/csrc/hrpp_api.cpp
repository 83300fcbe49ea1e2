// C ABI of the HRPP library: argument checking, device layout, epoch
// sequencing.  Every step of the query path runs in the kernels of
// hrpp_kernels.hip; this file only validates, lays out memory and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hrpp.h"
#include "hrpp_internal.h"
#include "hrpp_kernels.h"

using namespace hrpp;

namespace {

std::atomic<uint64_t> g_uid{1};

constexpr size_t kHeaderBytes = 256;   // BVH buffer header: [0] device error word

uint32_t max_persistent_blocks() {
    static uint32_t cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached = (uint32_t)cus * 16u;
    }
    return cached;
}

bool desc_ok(const hrpp_predictor_desc *d) {
    return d && d->log2_entries >= 1 && d->log2_entries <= 26 && d->ways >= 1 && d->ways <= 8 &&
           d->origin_bits >= 1 && d->origin_bits <= 10 && d->dir_bits >= 1 && d->dir_bits <= 10 &&
           d->epoch_rays >= 1 && d->epoch_rays <= (1u << 22) && d->go_up_level <= 64 && d->inline_lanes <= 65 &&
           d->replace_policy <= 3 && d->first_epoch_rays <= d->epoch_rays &&
           (d->hash_mode == 0 || (d->hash_mode == 1 && d->origin_bits <= 7 && d->dir_bits == d->origin_bits));
}

uint32_t entry_bytes_for(uint32_t ways) { return ways <= 4 ? 32u : 64u; }

struct PredLayout {
    size_t table, topw, topw_rows, pairs, rec_key, rec_idx, rec_leaf, rec_status, queue, dirty, ctrl, total;
};

PredLayout pred_layout(const hrpp_predictor_desc *d) {
    PredLayout L{};
    const size_t N = size_t(1) << d->log2_entries, E = d->epoch_rays, W = d->ways;
    size_t off = 0;
    L.table = off; off += align256(N * entry_bytes_for(d->ways));
    const size_t H = size_t(1) << pair_hash_bits_for((uint32_t)E);
    // one fresh-id list per claimed entry of an epoch: indexed by the entry when
    // the table is no larger than an epoch, else by the claiming ray's offset
    L.topw_rows = N <= E ? N : E;
    L.topw = off; off += align256(L.topw_rows * W * 8);
    L.pairs = off; off += align256(H * sizeof(PairSlot));
    L.rec_key = off; off += align256(E * 8);
    L.rec_idx = off; off += align256(E * 4);
    L.rec_leaf = off; off += align256(E * 4);
    L.rec_status = off; off += align256(E * 4);
    L.queue = off; off += align256((size_t)kSubQueues * queue_subcap_for((uint32_t)E) * 8);
    L.dirty = off; off += align256((N + kResetGroup - 1) / kResetGroup);
    L.ctrl = off; off += 256;
    L.total = off;
    return L;
}

hrpp_status check(hipError_t e) { return e == hipSuccess ? HRPP_OK : HRPP_EDEVICE; }

}  // namespace

extern "C" {

const char *hrpp_status_string(hrpp_status s) {
    switch (s) {
        case HRPP_OK: return "ok";
        case HRPP_EINVAL: return "invalid argument";
        case HRPP_ENOMEM: return "buffer too small or out of memory";
        case HRPP_EDEVICE: return "HIP runtime error";
        case HRPP_EDEPTH: return "BVH deeper than max_depth";
        case HRPP_EBUSY: return "busy";
    }
    return "unknown status";
}

size_t hrpp_bvh_required_bytes(uint32_t num_tris, const hrpp_bvh_desc *desc) {
    if (num_tris == 0 || !desc) return 0;
    const size_t interior = num_tris > 1 ? (size_t)num_tris - 1 : 0;   // at most n - 1 interior nodes
    const size_t nodes = 2 * (size_t)num_tris - 1;                      // at most 2n - 1 nodes
    // a wide node takes at least one binary interior node: at most n - 1 (1 for a one-leaf tree)
    const size_t wide = std::max<size_t>(1, interior);
    return kHeaderBytes + align256(interior * kNodeBytes) + align256((size_t)num_tris * kTriBytes) +
           align256((size_t)num_tris * kLeafBoxBytes) + align256(nodes * kCNodeBytes) +
           align256(wide * kWideNodeBytes);
}

hrpp_status hrpp_bvh_build_host(const float *h_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                hrpp_bvh **out) {
    if (!h_verts || !desc || !out || num_tris == 0 || num_tris >= (1u << 28)) return HRPP_EINVAL;
    *out = nullptr;
    hrpp_bvh *b = new (std::nothrow) hrpp_bvh();
    if (!b) return HRPP_ENOMEM;
    hrpp_status st = build_sah_tree(h_verts, num_tris, *desc, b->canon);
    if (st != HRPP_OK) { delete b; return st; }
    collapse_wide(b->canon, b->wide);
    const CanonTree &t = b->canon;
    b->uid = g_uid.fetch_add(1);
    b->num_tris = num_tris;
    b->num_nodes = (uint32_t)t.right.size();
    b->max_depth = t.max_depth;
    b->leaf_max = desc->leaf_max;
    for (int a = 0; a < 6; a++) b->root_box[a] = t.box[a];
    uint32_t ni = 0;
    for (uint32_t i = 0; i < b->num_nodes; i++)
        if (t.right[i] != kNone) ni++;
    b->num_interior = ni;
    b->verts.assign(h_verts, h_verts + 9 * (size_t)num_tris);
    b->d_nodes = nullptr;
    b->d_tris = nullptr;
    b->d_leafbox = nullptr;
    b->d_cnode = nullptr;
    b->d_wide = nullptr;
    *out = b;
    return HRPP_OK;
}

// Region offsets of a device-built BVH inside its buffer: sized for the
// largest tree over n triangles, since the node counts are known only after
// the build.
struct DeviceBvhLayout {
    size_t nodes, tris, leafbox, cnode, total;
};

static DeviceBvhLayout device_bvh_layout(uint32_t n) {
    DeviceBvhLayout L{};
    L.nodes = kHeaderBytes;
    L.tris = L.nodes + align256((size_t)(n - 1) * kNodeBytes);
    L.leafbox = L.tris + align256((size_t)n * kTriBytes);
    L.cnode = L.leafbox + align256((size_t)n * kLeafBoxBytes);
    L.total = L.cnode + align256((2 * (size_t)n - 1) * kCNodeBytes);
    return L;
}

size_t hrpp_bvh_device_bytes(const hrpp_bvh *bvh) {
    if (!bvh) return 0;
    if (bvh->device_built) return device_bvh_layout(bvh->num_tris).total;
    return kHeaderBytes + align256((size_t)bvh->num_interior * kNodeBytes) +
           align256((size_t)bvh->num_tris * kTriBytes) + align256((size_t)bvh->num_tris * kLeafBoxBytes) +
           align256((size_t)bvh->num_nodes * kCNodeBytes) + align256(bvh->wide.words.size() * 4);
}

hrpp_status hrpp_bvh_upload(hrpp_bvh *b, void *d_buf, size_t bytes, void *stream) {
    if (!b || !d_buf || b->verts.empty()) return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_buf) % 256) return HRPP_EINVAL;
    if (bytes < hrpp_bvh_device_bytes(b)) return HRPP_ENOMEM;
    const CanonTree &t = b->canon;
    const uint32_t m = b->num_nodes, n = b->num_tris;
    const float *h_verts = b->verts.data();
    // interior nodes keep their DFS order
    std::vector<uint32_t> iid(m, kNone);
    uint32_t ni = 0;
    for (uint32_t i = 0; i < m; i++)
        if (t.right[i] != kNone) iid[i] = ni++;
    auto ref_of = [&](uint32_t node) -> uint32_t {
        if (t.right[node] == kNone) return kLeafFlag | (t.first[node] << 3) | (t.count[node] - 1u);
        return iid[node];
    };
    b->root_ref = ref_of(0);
    std::vector<float> hn((size_t)ni * 16);
    for (uint32_t i = 0; i < m; i++) {
        if (t.right[i] == kNone) continue;
        float *p = &hn[(size_t)iid[i] * 16];
        const float *L = &t.box[6 * (size_t)(i + 1)];
        const float *R = &t.box[6 * (size_t)t.right[i]];
        for (int a = 0; a < 6; a++) { p[a] = L[a]; p[6 + a] = R[a]; }
        const uint32_t refs[4] = {ref_of(i + 1), ref_of(t.right[i]), 0u, 0u};
        std::memcpy(p + 12, refs, sizeof refs);
    }
    std::vector<uint32_t> leaf_depth(n, 0);
    for (uint32_t i = 0; i < m; i++)
        if (t.right[i] == kNone)
            for (uint32_t k = t.first[i]; k < t.first[i] + t.count[i]; k++) leaf_depth[k] = t.depth[i];
    // triangle record: v0 + prim | e1 + leaf depth | e2 + 0, with e = v - v0 in binary32
    std::vector<float> ht((size_t)n * 12);
    for (uint32_t k = 0; k < n; k++) {
        const uint32_t prim = t.perm[k];
        const float *v = h_verts + 9 * (size_t)prim;
        float *p = &ht[(size_t)k * 12];
        p[0] = v[0]; p[1] = v[1]; p[2] = v[2];
        std::memcpy(&p[3], &prim, 4);
        p[4] = v[3] - v[0]; p[5] = v[4] - v[1]; p[6] = v[5] - v[2];
        std::memcpy(&p[7], &leaf_depth[k], 4);
        p[8] = v[6] - v[0]; p[9] = v[7] - v[1]; p[10] = v[8] - v[2];
        p[11] = 0.0f;
    }
    // leaf boxes, indexed by the leaf's first triangle: min xyz, max x | max yz, depth, canonical node
    std::vector<float> hl((size_t)n * 8, 0.0f);
    for (uint32_t i = 0; i < m; i++) {
        if (t.right[i] != kNone) continue;
        float *p = &hl[(size_t)t.first[i] * 8];
        for (int a = 0; a < 6; a++) p[a] = t.box[6 * (size_t)i + a];
        std::memcpy(&p[6], &t.depth[i], 4);
        std::memcpy(&p[7], &i, 4);
    }
    // canonical node records (go-up levels >= 1 name nodes by canonical index):
    // min xyz, max x | max yz, reference, depth | parent, subtree triangle range
    std::vector<uint32_t> parent(m, kNone), lo(m), hi(m);
    for (uint32_t i = 0; i < m; i++)
        if (t.right[i] != kNone) { parent[i + 1] = i; parent[t.right[i]] = i; }
    for (uint32_t i = m; i-- > 0;) {
        if (t.right[i] == kNone) { lo[i] = t.first[i]; hi[i] = t.first[i] + t.count[i]; continue; }
        lo[i] = std::min(lo[i + 1], lo[t.right[i]]);
        hi[i] = std::max(hi[i + 1], hi[t.right[i]]);
    }
    std::vector<uint32_t> hc((size_t)m * 12, 0u);
    for (uint32_t i = 0; i < m; i++) {
        uint32_t *p = &hc[(size_t)i * 12];
        std::memcpy(p, &t.box[6 * (size_t)i], 6 * sizeof(float));
        p[6] = ref_of(i);
        p[7] = t.depth[i];
        p[8] = parent[i];
        p[9] = lo[i];
        p[10] = hi[i];
    }
    char *base = static_cast<char *>(d_buf);
    char *d_nodes = base + kHeaderBytes;
    char *d_tris = d_nodes + align256((size_t)ni * kNodeBytes);
    char *d_leafbox = d_tris + align256((size_t)n * kTriBytes);
    char *d_cnode = d_leafbox + align256((size_t)n * kLeafBoxBytes);
    char *d_wide = d_cnode + align256((size_t)m * kCNodeBytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemsetAsync(base, 0, kHeaderBytes, s);
    if (e == hipSuccess && ni) e = hipMemcpyAsync(d_nodes, hn.data(), hn.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tris, ht.data(), ht.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_leafbox, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_cnode, hc.data(), hc.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !b->wide.words.empty())
        e = hipMemcpyAsync(d_wide, b->wide.words.data(), b->wide.words.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // host staging buffers die here
    if (e != hipSuccess) return HRPP_EDEVICE;
    b->d_nodes = d_nodes;
    b->d_tris = d_tris;
    b->d_leafbox = d_leafbox;
    b->d_cnode = d_cnode;
    b->d_wide = d_wide;
    return HRPP_OK;
}

hrpp_status hrpp_build_bvh(const float *h_verts, uint32_t num_tris, const hrpp_bvh_desc *desc, void *d_buf,
                           size_t bytes, void *stream, hrpp_bvh **out) {
    if (!h_verts || !desc || !d_buf || !out || num_tris == 0 || num_tris >= (1u << 28)) return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_buf) % 256) return HRPP_EINVAL;
    if (bytes < hrpp_bvh_required_bytes(num_tris, desc)) return HRPP_ENOMEM;
    hrpp_bvh *b = nullptr;
    hrpp_status st = hrpp_bvh_build_host(h_verts, num_tris, desc, &b);
    if (st != HRPP_OK) return st;
    st = hrpp_bvh_upload(b, d_buf, bytes, stream);
    if (st != HRPP_OK) { delete b; *out = nullptr; return st; }
    *out = b;
    return HRPP_OK;
}

size_t hrpp_bvh_device_build_scratch_bytes(uint32_t num_tris) {
    if (num_tris == 0 || num_tris >= (1u << 28)) return 0;
    return lbvh_scratch_bytes(num_tris);
}

// The device build on a given scratch region (both entry points below).
static hrpp_status device_build(const float *d_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                void *d_scratch, size_t scratch_bytes, void *d_buf, size_t bytes, void *stream,
                                hrpp_bvh **out) {
    if (!out) return HRPP_EINVAL;
    *out = nullptr;
    if (!d_verts || !desc || !d_scratch || !d_buf || num_tris == 0 || num_tris >= (1u << 28)) return HRPP_EINVAL;
    if (desc->leaf_max < 1 || desc->leaf_max > 8 || desc->max_depth < 1 || desc->max_depth > (uint32_t)kMaxDepth ||
        desc->treelet_passes > kMaxTreeletPasses)
        return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_buf) % 256 || reinterpret_cast<uintptr_t>(d_scratch) % 256 ||
        reinterpret_cast<uintptr_t>(d_verts) % 4)
        return HRPP_EINVAL;
    const size_t need = lbvh_scratch_bytes(num_tris);
    if (need == 0) return HRPP_EDEVICE;
    const DeviceBvhLayout L = device_bvh_layout(num_tris);
    if (scratch_bytes < need || bytes < hrpp_bvh_required_bytes(num_tris, desc)) return HRPP_ENOMEM;
    char *base = static_cast<char *>(d_buf);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemsetAsync(base, 0, kHeaderBytes, s) != hipSuccess) return HRPP_EDEVICE;
    LbvhOut o{base + L.nodes, base + L.tris, base + L.leafbox, base + L.cnode};
    LbvhResult r{};
    if (lbvh_build(d_verts, num_tris, desc->leaf_max, desc->max_depth, desc->treelet_passes, d_scratch, o, s, &r) !=
        hipSuccess)
        return HRPP_EDEVICE;
    if (r.bad & 1u) return HRPP_EINVAL;
    const uint32_t m = r.num_nodes;
    if ((r.bad & 6u) || m == 0 || m % 2 == 0 || m > 2 * num_tris - 1) return HRPP_EDEVICE;
    if (r.max_depth > desc->max_depth) return HRPP_EDEPTH;
    hrpp_bvh *b = new (std::nothrow) hrpp_bvh();
    if (!b) return HRPP_ENOMEM;
    b->uid = g_uid.fetch_add(1);
    b->device_built = true;
    b->num_tris = num_tris;
    b->num_nodes = m;
    b->num_interior = (m - 1) / 2;
    b->max_depth = r.max_depth;
    b->leaf_max = desc->leaf_max;
    for (int a = 0; a < 6; a++) b->root_box[a] = r.root_box[a];
    b->root_ref = m == 1 ? (kLeafFlag | (num_tris - 1u)) : 0u;
    b->d_nodes = o.nodes;
    b->d_tris = o.tris;
    b->d_leafbox = o.leafbox;
    b->d_cnode = o.cnode;
    b->d_wide = nullptr;
    *out = b;
    return HRPP_OK;
}

hrpp_status hrpp_build_bvh_device(const float *d_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                  void *d_scratch, size_t scratch_bytes, void *d_buf, size_t bytes, void *stream,
                                  hrpp_bvh **out) {
    return device_build(d_verts, num_tris, desc, d_scratch, scratch_bytes, d_buf, bytes, stream, out);
}

hrpp_status hrpp_build_bvh_device_static(const float *d_verts, uint32_t num_tris, const hrpp_bvh_desc *desc,
                                         void *d_buf, size_t bytes, void *stream, hrpp_bvh **out) {
    if (!out) return HRPP_EINVAL;
    *out = nullptr;
    if (num_tris == 0 || num_tris >= (1u << 28)) return HRPP_EINVAL;
    const size_t need = lbvh_scratch_bytes(num_tris);
    if (need == 0) return HRPP_EDEVICE;
    if (need > kStaticBuildScratchBytes) return HRPP_ENOMEM;   // more triangles than the static scratch holds
    void *d_scratch = nullptr;
    if (lbvh_static_scratch(&d_scratch) != hipSuccess || !d_scratch) return HRPP_EDEVICE;
    return device_build(d_verts, num_tris, desc, d_scratch, kStaticBuildScratchBytes, d_buf, bytes, stream, out);
}

hrpp_status hrpp_bvh_info(const hrpp_bvh *bvh, uint32_t *num_nodes, uint32_t *num_tris, uint32_t *max_depth) {
    if (!bvh) return HRPP_EINVAL;
    if (num_nodes) *num_nodes = bvh->num_nodes;
    if (num_tris) *num_tris = bvh->num_tris;
    if (max_depth) *max_depth = bvh->max_depth;
    return HRPP_OK;
}

hrpp_status hrpp_bvh_wide_info(const hrpp_bvh *bvh, uint32_t *num_nodes, uint32_t *root_ref, uint32_t *stack_need,
                               uint32_t *depth) {
    if (!bvh) return HRPP_EINVAL;
    if (num_nodes) *num_nodes = (uint32_t)(bvh->wide.words.size() / 32);
    if (root_ref) *root_ref = bvh->wide.root_ref;
    if (stack_need) *stack_need = bvh->wide.stack_need;
    if (depth) *depth = bvh->wide.depth;
    return HRPP_OK;
}

hrpp_status hrpp_bvh_wide_export(const hrpp_bvh *bvh, uint32_t *h_words, size_t words) {
    if (!bvh || (!h_words && !bvh->wide.words.empty()) || words < bvh->wide.words.size()) return HRPP_EINVAL;
    if (!bvh->wide.words.empty()) std::memcpy(h_words, bvh->wide.words.data(), bvh->wide.words.size() * 4);
    return HRPP_OK;
}

hrpp_status hrpp_bvh_export(const hrpp_bvh *bvh, hrpp_bvh_canon *o) {
    if (!bvh || !o || !o->box || !o->right || !o->first_tri || !o->count || !o->depth || !o->tri_perm)
        return HRPP_EINVAL;
    if (bvh->device_built) {
        // read the canonical node records and triangle records back
        const uint32_t m = bvh->num_nodes, n = bvh->num_tris;
        std::vector<uint32_t> hc((size_t)m * 12), ht((size_t)n * 12);
        if (hipMemcpy(hc.data(), bvh->d_cnode, hc.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(ht.data(), bvh->d_tris, ht.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return HRPP_EDEVICE;
        for (uint32_t i = 0; i < m; i++) {
            const uint32_t *p = &hc[(size_t)i * 12];
            std::memcpy(&o->box[6 * (size_t)i], p, 6 * sizeof(float));
            const uint32_t ref = p[6];
            const bool leaf = (ref & kLeafFlag) != 0;
            o->right[i] = kNone;
            o->first_tri[i] = leaf ? (ref & ~kLeafFlag) >> 3 : 0u;
            o->count[i] = leaf ? (ref & 7u) + 1u : 0u;
            o->depth[i] = p[7];
        }
        for (uint32_t j = 1; j < m; j++) {   // a child that is not the next node is its parent's right child
            const uint32_t par = hc[(size_t)j * 12 + 8];
            if (par >= m) return HRPP_EDEVICE;
            if (j != par + 1) o->right[par] = j;
        }
        for (uint32_t k = 0; k < n; k++) o->tri_perm[k] = ht[(size_t)k * 12 + 3];
        return HRPP_OK;
    }
    const CanonTree &t = bvh->canon;
    std::memcpy(o->box, t.box.data(), t.box.size() * 4);
    std::memcpy(o->right, t.right.data(), t.right.size() * 4);
    std::memcpy(o->first_tri, t.first.data(), t.first.size() * 4);
    std::memcpy(o->count, t.count.data(), t.count.size() * 4);
    std::memcpy(o->depth, t.depth.data(), t.depth.size() * 4);
    std::memcpy(o->tri_perm, t.perm.data(), t.perm.size() * 4);
    return HRPP_OK;
}

void hrpp_bvh_destroy(hrpp_bvh *bvh) { delete bvh; }

size_t hrpp_predictor_required_bytes(const hrpp_predictor_desc *desc) {
    if (!desc_ok(desc)) return 0;
    return pred_layout(desc).total;
}

size_t hrpp_predictor_table_bytes(const hrpp_predictor_desc *desc) {
    if (!desc_ok(desc)) return 0;
    return (size_t(1) << desc->log2_entries) * entry_bytes_for(desc->ways);
}

hrpp_status hrpp_predictor_reset(hrpp_predictor *p, void *stream) {
    if (!p) return HRPP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the update marks the group of every entry it tags while empty (see
    // k_update_apply): clear the marked groups, or everything when an entry
    // may have been written without a mark
    launch_reset_table(p->d_table, p->entry_bytes, 1u << p->desc.log2_entries, p->d_dirty,
                       p->table_unmarked || p->scratch_dirty, s);
    const bool scratch = p->scratch_dirty;
    if (scratch) {
        // every epoch leaves the fresh-id lists, record slots and sub-queue
        // counts cleared; they are cleared here only at creation and after a
        // failed launch
        const size_t E = p->desc.epoch_rays;
        launch_fill32(p->d_ctrl, 64, 0u, s);
        const PredLayout L = pred_layout(&p->desc);
        launch_fill32(reinterpret_cast<uint32_t *>(p->d_topw), 2 * L.topw_rows * p->desc.ways, kNone, s);
        const size_t H = size_t(1) << pair_hash_bits_for((uint32_t)E);
        launch_fill32(static_cast<uint32_t *>(p->d_pairs), 4 * H, kNone, s);
        launch_fill32(p->d_rec_idx, E, kNone, s);
    }
    const hrpp_status st = check(hipGetLastError());
    if (st == HRPP_OK) {
        // only a reset whose launches were accepted establishes a clean state;
        // otherwise the next reset clears everything again
        p->table_unmarked = false;
        p->scratch_dirty = false;
        p->empty = true;
    }
    return st;
}

hrpp_status hrpp_predictor_create(const hrpp_bvh *bvh, const hrpp_predictor_desc *desc, void *d_buf, size_t bytes,
                                  void *stream, hrpp_predictor **out) {
    if (!bvh || !bvh->d_nodes || !desc_ok(desc) || !d_buf || !out) return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_buf) % 256) return HRPP_EINVAL;
    const PredLayout L = pred_layout(desc);
    if (bytes < L.total) return HRPP_ENOMEM;
    *out = nullptr;
    hrpp_predictor *p = new (std::nothrow) hrpp_predictor();
    if (!p) return HRPP_ENOMEM;
    char *base = static_cast<char *>(d_buf);
    p->bvh_uid = bvh->uid;
    p->bvh_tris = bvh->num_tris;
    p->bvh_nodes = bvh->num_nodes;
    p->desc = *desc;
    p->entry_bytes = entry_bytes_for(desc->ways);
    p->table_bytes = (size_t(1) << desc->log2_entries) * p->entry_bytes;
    p->d_table = base + L.table;
    p->d_topw = reinterpret_cast<uint64_t *>(base + L.topw);
    p->topw_by_entry = L.topw_rows == (size_t(1) << desc->log2_entries);
    p->d_pairs = base + L.pairs;
    p->d_rec_key = reinterpret_cast<uint64_t *>(base + L.rec_key);
    p->d_rec_idx = reinterpret_cast<uint32_t *>(base + L.rec_idx);
    p->d_rec_leaf = reinterpret_cast<uint32_t *>(base + L.rec_leaf);
    p->d_rec_status = reinterpret_cast<uint32_t *>(base + L.rec_status);
    p->d_queue = reinterpret_cast<uint64_t *>(base + L.queue);
    p->d_dirty = reinterpret_cast<uint8_t *>(base + L.dirty);
    p->d_ctrl = reinterpret_cast<uint32_t *>(base + L.ctrl);
    // hash grid over the scene box: scale = 2^qo / extent (0 for a flat or
    // degenerate axis), computed once in binary32
    for (int a = 0; a < 3; a++) {
        const float ext = bvh->root_box[3 + a] - bvh->root_box[a];
        float sc = (float)(1u << desc->origin_bits) / ext;
        if (!(ext > 0.0f) || !std::isfinite(sc)) sc = 0.0f;
        p->bmin[a] = bvh->root_box[a];
        p->scale[a] = sc;
    }
    hrpp_status st = hrpp_predictor_reset(p, stream);
    if (st != HRPP_OK) { delete p; return st; }
    *out = p;
    return HRPP_OK;
}

hrpp_status hrpp_predictor_export(const hrpp_predictor *p, void *h_dst, size_t bytes, void *stream) {
    if (!p || !h_dst || bytes < p->table_bytes) return HRPP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(h_dst, p->d_table, p->table_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return check(e);
}

hrpp_status hrpp_predictor_import(hrpp_predictor *p, const void *h_src, size_t bytes, void *stream) {
    if (!p || !h_src || bytes < p->table_bytes) return HRPP_EINVAL;
    // every slot must stay inside this predictor's BVH (a leaf id's triangle
    // range, or a node index at go-up levels >= 1) and no claim may be held,
    // so that the kernels never index outside the scene arrays
    const char *src = static_cast<const char *>(h_src);
    const size_t entries = size_t(1) << p->desc.log2_entries;
    for (size_t i = 0; i < entries; i++) {
        const char *e = src + i * p->entry_bytes;
        uint32_t w[9];
        std::memcpy(w, e + 8, 4 * (p->desc.ways + 1));
        if (w[p->desc.ways] != kNone) return HRPP_EINVAL;
        for (uint32_t k = 0; k < p->desc.ways; k++) {
            const uint32_t v = w[k];
            if (v == kNone) continue;
            if (p->desc.go_up_level > 0) {
                if (v >= p->bvh_nodes) return HRPP_EINVAL;
            } else if ((v >> 3) + (v & 7u) + 1u > p->bvh_tris) {
                return HRPP_EINVAL;
            }
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(p->d_table, h_src, p->table_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    p->empty = false;
    p->table_unmarked = true;      // imported entries carry no reset marks
    return check(e);
}

void hrpp_predictor_destroy(hrpp_predictor *p) { delete p; }

// Kernel arguments of one trace (shared by single calls and batches).
// Touch bitmap of the measurement mode (hrpp_profile_touch): which BVH and
// predictor it is for, and its layout.
namespace {
struct TouchState {
    uint32_t *bits = nullptr;
    size_t words = 0;
    const hrpp_bvh *bvh = nullptr;
    const hrpp_predictor *pred = nullptr;
    uint32_t layout[1 + 2 * kTouchRegions] = {};
};
TouchState g_touch;

// Block size and region offsets (words) of the touch bitmap for a BVH and
// predictor: regions of 128-byte lines of the interior nodes, triangles, leaf
// boxes, table entries and canonical nodes.
void touch_layout(const hrpp_bvh *bvh, const hrpp_predictor *pred, uint32_t *out) {
    const size_t bytes[kTouchRegions] = {
        (size_t)bvh->num_interior * kNodeBytes, (size_t)bvh->num_tris * kTriBytes,
        (size_t)bvh->num_tris * kLeafBoxBytes, pred ? pred->table_bytes : 0, (size_t)bvh->num_nodes * kCNodeBytes};
    uint32_t off = 0;
    for (int r = 0; r < kTouchRegions; r++) {
        const uint32_t lines = (uint32_t)((bytes[r] + 127) / 128);
        out[1 + r] = off;
        out[1 + kTouchRegions + r] = lines;
        off += (lines + 31) / 32;
    }
    out[0] = off;
}
}  // namespace

static TraceArgs make_args(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint8_t *d_occ,
                           hrpp_hit *d_hits, hrpp_stats *d_stats) {
    TraceArgs a{};
    a.nodes = bvh->d_nodes;
    a.tris = bvh->d_tris;
    a.leafbox = bvh->d_leafbox;
    a.cnode = bvh->d_cnode;
    for (int i = 0; i < 6; i++) a.root_box[i] = bvh->root_box[i];
    a.root_ref = bvh->root_ref;
    a.stack_cap = std::max<uint32_t>(1u, bvh->max_depth);
    a.max_blocks = max_persistent_blocks();
    a.rays = d_rays;
    a.occluded = d_occ;
    a.hits = d_hits;
    a.stats = reinterpret_cast<unsigned long long *>(d_stats);
    a.error = reinterpret_cast<uint32_t *>(static_cast<char *>(const_cast<void *>(bvh->d_nodes)) - kHeaderBytes);
    if (pred) {
        const hrpp_predictor_desc &d = pred->desc;
        a.table = pred->d_table;
        a.entry_bytes = pred->entry_bytes;
        a.ways = d.ways;
        for (int i = 0; i < 3; i++) { a.hash.bmin[i] = pred->bmin[i]; a.hash.scale[i] = pred->scale[i]; }
        a.hash.maxo = (float)((1u << d.origin_bits) - 1u);
        a.hash.maxd = (float)((1u << d.dir_bits) - 1u);
        a.hash.half = (float)(1u << (d.dir_bits - 1u));
        a.hash.qo = d.origin_bits;
        a.hash.qd = d.dir_bits;
        a.hash.log2n = d.log2_entries;
        a.hash.mode = d.hash_mode;
        a.go_up = d.go_up_level;
        a.inline_min = d.inline_lanes ? d.inline_lanes : kDefaultInlineLanes;
        a.policy = d.replace_policy;
        a.hash.stride = d.origin_bits <= 3 ? 8u : 16u;
        a.ctrl = pred->d_ctrl;
        a.dirty = pred->d_dirty;
        a.queue = pred->d_queue;
        a.queue_subcap = queue_subcap_for(d.epoch_rays);
        a.rec_key = pred->d_rec_key;
        a.rec_idx = pred->d_rec_idx;
        a.rec_leaf = pred->d_rec_leaf;
        a.rec_status = pred->d_rec_status;
        a.topw = pred->d_topw;
        a.topw_by_entry = pred->topw_by_entry ? 1u : 0u;
        a.pairs = static_cast<PairSlot *>(pred->d_pairs);
        a.hash_bits = pair_hash_bits_for(d.epoch_rays);
    }
    if (g_touch.bits && d_stats && g_touch.bvh == bvh && g_touch.pred == pred) {
        a.touch = g_touch.bits;
        a.touch_kind_words = g_touch.layout[0];
        for (int r = 0; r < kTouchRegions; r++) a.touch_off[r] = g_touch.layout[1 + r];
    }
    return a;
}

static hrpp_status check_trace_args(const hrpp_bvh *bvh, const hrpp_predictor *pred, const void *d_rays, uint32_t n,
                                    bool any, const void *d_out) {
    if (!bvh || !bvh->d_nodes) return HRPP_EINVAL;
    if (n == 0) return HRPP_OK;
    if (n >= (1u << 31) || !d_rays || !d_out) return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_rays) % 16 || (!any && reinterpret_cast<uintptr_t>(d_out) % 16))
        return HRPP_EINVAL;
    if (pred && pred->bvh_uid != bvh->uid) return HRPP_EINVAL;
    return HRPP_OK;
}

static hrpp_status trace_common(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint32_t n,
                                bool any, bool exact, uint8_t *d_occ, hrpp_hit *d_hits, hrpp_stats *d_stats,
                                void *stream) {
    const hrpp_status st = check_trace_args(bvh, pred, d_rays, n, any, any ? (const void *)d_occ : d_hits);
    if (st != HRPP_OK || n == 0) return st;
    // after a failed launch the epoch scratch (record list, claims, queue
    // counts) may hold stale words: the predictor needs a reset first
    if (pred && pred->scratch_dirty) return HRPP_EINVAL;
    const TraceArgs a = make_args(bvh, pred, d_rays, d_occ, d_hits, d_stats);
    const uint32_t epoch = pred ? pred->desc.epoch_rays : n;
    const uint32_t first = pred && pred->desc.first_epoch_rays ? pred->desc.first_epoch_rays : epoch;
    launch_trace(a, n, any, exact, pred != nullptr, epoch, first, pred && pred->empty,
                 static_cast<hipStream_t>(stream));
    const hrpp_status ls = check(hipGetLastError());
    if (pred) {
        pred->empty = false;
        if (ls != HRPP_OK) pred->scratch_dirty = pred->table_unmarked = true;
    }
    return ls;
}

hrpp_status hrpp_trace_anyhit(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint32_t n,
                              uint8_t *d_occluded, hrpp_stats *d_stats, void *stream) {
    return trace_common(bvh, pred, d_rays, n, true, false, d_occluded, nullptr, d_stats, stream);
}

hrpp_status hrpp_trace_closest(const hrpp_bvh *bvh, hrpp_predictor *pred, const hrpp_ray *d_rays, uint32_t n,
                               uint32_t mode, hrpp_hit *d_hits, hrpp_stats *d_stats, void *stream) {
    if (mode != HRPP_CLOSEST_PAPER && mode != HRPP_CLOSEST_EXACT) return HRPP_EINVAL;
    return trace_common(bvh, pred, d_rays, n, false, mode == HRPP_CLOSEST_EXACT, nullptr, d_hits, d_stats, stream);
}

static hrpp_status trace_wide(const hrpp_bvh *bvh, const hrpp_ray *d_rays, uint32_t n, bool any, uint8_t *d_occ,
                              hrpp_hit *d_hits, hrpp_stats *d_stats, void *stream) {
    const hrpp_status st = check_trace_args(bvh, nullptr, d_rays, n, any, any ? (const void *)d_occ : d_hits);
    if (st != HRPP_OK || n == 0) return st;
    if (!bvh->d_wide) return HRPP_EINVAL;
    TraceArgs a = make_args(bvh, nullptr, d_rays, d_occ, d_hits, d_stats);
    a.wide = bvh->d_wide;
    a.wide_root = bvh->wide.root_ref;
    a.stack_cap = std::max<uint32_t>(1u, bvh->wide.stack_need);
    launch_wide(a, n, any, static_cast<hipStream_t>(stream));
    return check(hipGetLastError());
}

hrpp_status hrpp_trace_wide_anyhit(const hrpp_bvh *bvh, const hrpp_ray *d_rays, uint32_t n, uint8_t *d_occluded,
                                   hrpp_stats *d_stats, void *stream) {
    return trace_wide(bvh, d_rays, n, true, d_occluded, nullptr, d_stats, stream);
}

hrpp_status hrpp_trace_wide_closest(const hrpp_bvh *bvh, const hrpp_ray *d_rays, uint32_t n, hrpp_hit *d_hits,
                                    hrpp_stats *d_stats, void *stream) {
    return trace_wide(bvh, d_rays, n, false, nullptr, d_hits, d_stats, stream);
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct hrpp_batch {
    std::vector<BatchJob> jobs;
    std::vector<hrpp_predictor *> preds;    // the jobs' predictors (host state: scheduling hints, scratch)
    std::vector<uint32_t> ids;
    std::vector<BatchGroup> groups;
    uint32_t max_rounds = 0;
    BatchJob *d_jobs = nullptr;
    uint32_t *d_ids = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;   // the legacy default stream cannot be captured
};

static bool bj_inline(const hrpp_predictor *p) {
    const uint32_t v = p->desc.inline_lanes ? p->desc.inline_lanes : kDefaultInlineLanes;
    return v <= 64;
}

// Block offsets: count + 1 per group for the two plain groups, and three
// arrays of count + 1 per predictor group that runs in rounds (at most six
// such groups; groups of small-epoch jobs need none).
static size_t batch_offset_words(uint32_t njobs) { return ((size_t)njobs + 2) + 3 * ((size_t)njobs + 6); }

size_t hrpp_batch_required_bytes(uint32_t njobs) {
    // job table, job ids, and the groups' block offsets
    return align256((size_t)njobs * sizeof(BatchJob)) + align256((size_t)njobs * sizeof(uint32_t)) +
           align256(batch_offset_words(njobs) * sizeof(uint32_t));
}

hrpp_status hrpp_batch_create(const hrpp_batch_job *jobs, uint32_t njobs, void *d_buf, size_t bytes, void *stream,
                              hrpp_batch **out) {
    if (!jobs || njobs == 0 || !d_buf || !out) return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_buf) % 256) return HRPP_EINVAL;
    if (bytes < hrpp_batch_required_bytes(njobs)) return HRPP_ENOMEM;
    *out = nullptr;
    hrpp_batch *b = new (std::nothrow) hrpp_batch();
    if (!b) return HRPP_ENOMEM;
    std::vector<uint32_t> kind_of(njobs);
    for (uint32_t j = 0; j < njobs; j++) {
        const hrpp_batch_job &J = jobs[j];
        const bool any = (J.query == 0);
        if (J.query > 1 || (!any && J.mode != HRPP_CLOSEST_PAPER && J.mode != HRPP_CLOSEST_EXACT)) {
            delete b;
            return HRPP_EINVAL;
        }
        hrpp_status st = check_trace_args(J.bvh, J.pred, J.d_rays, J.n, any, J.d_out);
        if (st != HRPP_OK) { delete b; return st; }
        for (uint32_t k = 0; k < j; k++)
            if (J.pred && jobs[k].pred == J.pred) { delete b; return HRPP_EINVAL; }   // predictors must be distinct
        BatchJob bj{};
        bj.a = make_args(J.bvh, J.pred, J.d_rays, any ? static_cast<uint8_t *>(J.d_out) : nullptr,
                         any ? nullptr : static_cast<hrpp_hit *>(J.d_out), J.d_stats);
        bj.n = J.n;
        bj.epoch = J.pred ? J.pred->desc.epoch_rays : std::max(1u, J.n);
        bj.first = J.pred && J.pred->desc.first_epoch_rays ? J.pred->desc.first_epoch_rays : bj.epoch;
        b->jobs.push_back(bj);
        if (J.pred) b->preds.push_back(J.pred);
        if (J.pred) kind_of[j] = any ? kBatchAnyHrpp : (J.mode == HRPP_CLOSEST_EXACT ? kBatchExactHrpp : kBatchPaperHrpp);
        else kind_of[j] = any ? kBatchAnyPlain : kBatchClosestPlain;
    }
    // groups: by kind; predictor kinds also by go-up level (bit 0 of sub) and
    // by whether the job's epochs are small enough for one workgroup (bit 1)
    for (int kind = kBatchAnyHrpp; kind <= kBatchClosestPlain; kind++)
    for (int sub = 0; sub < 4; sub++) {
        const bool hrpp_kind = (kind == kBatchAnyHrpp || kind == kBatchPaperHrpp || kind == kBatchExactHrpp);
        if (sub && !hrpp_kind) continue;
        BatchGroup g{};
        g.kind = kind;
        g.subtree = (sub & 1) != 0;
        g.block_epochs = (sub & 2) != 0;
        g.first_id = (uint32_t)b->ids.size();
        for (uint32_t j = 0; j < njobs; j++) {
            if ((int)kind_of[j] != kind || jobs[j].n == 0) continue;
            if (hrpp_kind && (jobs[j].pred->desc.go_up_level > 0) != g.subtree) continue;
            if (hrpp_kind && (b->jobs[j].first <= kBlockEpochRays && b->jobs[j].epoch <= kBlockEpochRays) !=
                                 g.block_epochs)
                continue;
            if (hrpp_kind && bj_inline(jobs[j].pred)) g.inline_any = true;
            const BatchJob &bj = b->jobs[j];
            b->ids.push_back(j);
            g.count++;
            g.rounds = std::max(g.rounds, bj.n <= bj.first ? 1u : 1u + (bj.n - bj.first + bj.epoch - 1) / bj.epoch);
            if (bj.a.stats) g.stats = true;
        }
        if (g.count == 0) continue;
        if (kind == kBatchAnyPlain || kind == kBatchClosestPlain || g.block_epochs) g.rounds = 0;
        b->max_rounds = std::max(b->max_rounds, g.rounds);
        b->groups.push_back(g);
    }
    char *base = static_cast<char *>(d_buf);
    b->d_jobs = reinterpret_cast<BatchJob *>(base);
    b->d_ids = reinterpret_cast<uint32_t *>(base + align256((size_t)njobs * sizeof(BatchJob)));
    uint32_t *d_off = reinterpret_cast<uint32_t *>(base + align256((size_t)njobs * sizeof(BatchJob)) +
                                                   align256((size_t)njobs * sizeof(uint32_t)));
    // flat grids: plain groups get one lane per ray of each job; predictor
    // groups one lane per ray of each job's longest epoch (the first epoch is
    // never longer than the others), which every round reuses
    std::vector<uint32_t> offs;
    auto add_offsets = [&](const BatchGroup &g, uint32_t lanes, uint32_t cap, bool whole) {
        const uint32_t at = (uint32_t)offs.size();
        uint32_t acc = 0;
        for (uint32_t k = 0; k < g.count; k++) {
            const BatchJob &bj = b->jobs[b->ids[g.first_id + k]];
            const uint32_t rays = whole ? bj.n : std::min(bj.epoch, bj.n);
            offs.push_back(acc);
            acc += std::min(cap, std::max(1u, (rays + lanes - 1u) / lanes));
        }
        offs.push_back(acc);
        return std::make_pair(at, acc);
    };
    for (BatchGroup &g : b->groups) {
        if (g.block_epochs) continue;   // one workgroup per job: no block offsets
        if (g.kind == kBatchAnyPlain || g.kind == kBatchClosestPlain) {
            const auto p = add_offsets(g, 128u, ~0u, true);
            g.d_block_off = d_off + p.first;
            g.total_blocks = p.second;
        } else {
            const auto p128 = add_offsets(g, 128u, ~0u, false);
            const auto p256 = add_offsets(g, 256u, ~0u, false);
            const auto pq = add_offsets(g, 128u, kQueueBlocks, false);
            g.d_off128 = d_off + p128.first;
            g.d_off256 = d_off + p256.first;
            g.d_offq = d_off + pq.first;
            g.blocks128 = p128.second;
            g.blocks256 = p256.second;
            g.blocksq = pq.second;
        }
    }
    if (offs.size() > batch_offset_words(njobs)) { delete b; return HRPP_EINVAL; }   // cannot happen
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(b->d_jobs, b->jobs.data(), b->jobs.size() * sizeof(BatchJob),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !b->ids.empty())
        e = hipMemcpyAsync(b->d_ids, b->ids.data(), b->ids.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !offs.empty())
        e = hipMemcpyAsync(d_off, offs.data(), offs.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete b; return HRPP_EDEVICE; }
    *out = b;
    return HRPP_OK;
}

static hrpp_status batch_launch(hrpp_batch *b, uint32_t use_graph, hipStream_t s);

hrpp_status hrpp_batch_launch(hrpp_batch *b, uint32_t use_graph, void *stream) {
    if (!b) return HRPP_EINVAL;
    for (const hrpp_predictor *p : b->preds)
        if (p->scratch_dirty) return HRPP_EINVAL;   // reset the predictor after a failed launch first
    const hrpp_status st = batch_launch(b, use_graph, static_cast<hipStream_t>(stream));
    for (hrpp_predictor *p : b->preds) {
        p->empty = false;
        if (st != HRPP_OK) p->scratch_dirty = p->table_unmarked = true;
    }
    return st;
}

static hrpp_status batch_launch(hrpp_batch *b, uint32_t use_graph, hipStream_t s) {
    if (!use_graph) {
        launch_batch(b->d_jobs, b->d_ids, b->groups, b->max_rounds, max_persistent_blocks(), s);
        return check(hipGetLastError());
    }
    if (!b->exec) {
        const uint32_t max_blocks = max_persistent_blocks();   // query outside the capture
        if (!b->capture_stream && hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return HRPP_EDEVICE;
        hipStream_t cs = b->capture_stream;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return HRPP_EDEVICE;
        launch_batch(b->d_jobs, b->d_ids, b->groups, b->max_rounds, max_blocks, cs);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) return HRPP_EDEVICE;
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return HRPP_EDEVICE;
        }
        b->graph = g;
        b->exec = x;
    }
    return check(hipGraphLaunch(b->exec, s));
}

void hrpp_batch_destroy(hrpp_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    delete b;
}

hrpp_status hrpp_profile_touch(const hrpp_bvh *bvh, const hrpp_predictor *pred, uint32_t *d_bits, size_t words,
                               uint32_t *h_layout) {
    if (!d_bits) {
        g_touch = TouchState{};
        if (bvh && h_layout) {                    // the layout only, to size a bitmap
            if (!bvh->d_nodes || (pred && pred->bvh_uid != bvh->uid)) return HRPP_EINVAL;
            touch_layout(bvh, pred, h_layout);
        }
        return HRPP_OK;
    }
    if (!bvh || !bvh->d_nodes || (pred && pred->bvh_uid != bvh->uid)) return HRPP_EINVAL;
    TouchState t;
    touch_layout(bvh, pred, t.layout);
    if (words < (size_t)kTouchKinds * t.layout[0]) return HRPP_EINVAL;
    t.bits = d_bits;
    t.words = words;
    t.bvh = bvh;
    t.pred = pred;
    g_touch = t;
    if (h_layout) std::memcpy(h_layout, t.layout, sizeof t.layout);
    return HRPP_OK;
}

hrpp_status hrpp_profile_start(void) {
    profile_start();
    return HRPP_OK;
}

hrpp_status hrpp_profile_stop(hrpp_kernel_time *out, uint32_t capacity, uint32_t *count) {
    double ms[kNumKernelKinds];
    uint64_t launches[kNumKernelKinds];
    const int err = profile_stop(ms, launches);
    uint32_t n = 0;
    for (int k = 0; k < kNumKernelKinds; k++) {
        if (launches[k] == 0) continue;
        if (out && n < capacity) {
            std::memset(&out[n], 0, sizeof(hrpp_kernel_time));
            std::strncpy(out[n].name, kernel_kind_name(k), sizeof(out[n].name) - 1);
            out[n].launches = launches[k];
            out[n].total_ms = ms[k];
        }
        n++;
    }
    if (count) *count = n;
    return err ? HRPP_EDEVICE : HRPP_OK;
}

hrpp_status hrpp_get_error(const hrpp_bvh *bvh, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return HRPP_EDEVICE;
    if (hipGetLastError() != hipSuccess) return HRPP_EDEVICE;
    if (bvh && bvh->d_nodes) {
        uint32_t word = 0;
        const void *err = static_cast<const char *>(bvh->d_nodes) - kHeaderBytes;
        if (hipMemcpy(&word, err, 4, hipMemcpyDeviceToHost) != hipSuccess) return HRPP_EDEVICE;
        if (word & 1u) return HRPP_EDEPTH;
    }
    return HRPP_OK;
}

}  // extern "C"
