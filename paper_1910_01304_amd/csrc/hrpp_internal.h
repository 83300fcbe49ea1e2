// Internal definitions shared by the host builder and the HIP kernels of the
// HRPP library.  Not part of the public ABI (see include/hrpp.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hrpp.h"

namespace hrpp {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kLeafFlag = 0x80000000u;   // node reference names a leaf
constexpr uint64_t kEmptyTag = 0xFFFFFFFFFFFFFFFFull;
constexpr int kMaxDepth = 64;                  // deepest leaf the kernels accept
constexpr uint32_t kMaxTreeletPasses = 8;      // treelet restructuring passes a build accepts

// Counter slots, in the order of hrpp_stats.
enum Stat : int {
    kRays, kInvalid, kHits, kLookups, kPositives, kPredHits, kFalsePos, kTraversals,
    kNodesVisited, kInteriorVisited, kLeafVisited, kBoxTests, kTriTests, kNodesSkipped,
    kRecords, kTagClaims, kLeafInserts, kDropped, kConflicts, kPredLeafVisited, kPredTriTests, kPredBoxTests,
    kEvictions, kQueueTraversals, kQueueInteriorVisited, kQueueTriTests, kQueueRecords, kEmptyLookups,
    kEmptyRays, kEmptyInteriorVisited, kEmptyTriTests, kEmptyRecords, kNumStats
};

static_assert(kNumStats <= HRPP_STATS_SLOTS, "hrpp_stats has a slot for every counter");

// Canonical depth-first pre-order tree, as produced by the builder.
struct CanonTree {
    std::vector<float> box;        // 6 per node
    std::vector<uint32_t> right;   // kNone for leaves
    std::vector<uint32_t> first;
    std::vector<uint32_t> count;
    std::vector<uint32_t> depth;
    std::vector<uint32_t> perm;    // BVH position -> original primitive id
    uint32_t max_depth = 0;
};

// Deterministic binned-SAH build; returns HRPP_OK, HRPP_EINVAL or HRPP_EDEPTH.
hrpp_status build_sah_tree(const float *verts, uint32_t n, const hrpp_bvh_desc &desc, CanonTree &out);

// 4-wide tree collapsed from the binary one (plain-traversal baseline).
struct WideTree {
    std::vector<uint32_t> words;   // 32 per node (128 B), layout in bvh_wide.cpp
    uint32_t root_ref = kNone;     // node 0, or kLeafFlag | leaf id for a one-leaf tree
    uint32_t stack_need = 1;       // most stack entries any traversal can hold
    uint32_t depth = 0;            // wide interior levels
};
void collapse_wide(const CanonTree &t, WideTree &w);

// GPU layout sizes.
constexpr size_t kNodeBytes = 64;   // two child boxes + two references
constexpr size_t kTriBytes = 48;    // v0+prim | e1+leaf depth | e2+pad
constexpr size_t kLeafBoxBytes = 32;  // per BVH triangle position: box of the leaf starting there, depth, node
constexpr size_t kCNodeBytes = 48;    // per canonical node: box, reference, depth, parent, triangle range
constexpr size_t kWideNodeBytes = 128; // per 4-wide node: child boxes (structure of arrays) + references
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace hrpp

// Opaque handles (defined here so the builder and the API share them).
struct hrpp_bvh {
    uint64_t uid;
    uint32_t num_tris, num_nodes, num_interior, max_depth, leaf_max;
    float root_box[6];
    uint32_t root_ref;          // kLeafFlag|leaf id when the root is a leaf, else 0
    const void *d_nodes;        // num_interior * 64 B
    const void *d_tris;         // num_tris * 48 B
    const void *d_leafbox;      // num_tris * 32 B (valid at leaf start positions)
    const void *d_cnode;        // num_nodes * 48 B, canonical (depth-first pre-order) node records
    const void *d_wide;         // 4-wide nodes, 128 B each (plain-traversal baseline)
    bool device_built = false;  // built by hrpp_build_bvh_device: no host tree, no 4-wide tree
    hrpp::CanonTree canon;
    hrpp::WideTree wide;
    std::vector<float> verts;   // host copy of the input, used by the upload
};

struct hrpp_predictor {
    uint64_t bvh_uid;
    uint32_t bvh_tris, bvh_nodes;  // sizes of the BVH the table indexes (import checks slots against them)
    bool empty = true;             // reset and not traced or imported since (scheduling hint only)
    bool scratch_dirty = true;     // fresh-id lists / record slots need clearing (creation, failed launch)
    bool table_unmarked = true;    // the table may hold entries whose reset group is not marked
                                   // (creation, import, failed launch): the next reset clears all of it
    hrpp_predictor_desc desc;
    uint32_t entry_bytes;       // 32 or 64
    float bmin[3], scale[3];    // hash grid over the BVH root box
    // device regions inside the caller's buffer
    void *d_table;              // 2^T entries
    uint64_t *d_topw;           // min(2^T, E) * W fresh-id lists, ray id << 32 | id
    bool topw_by_entry;         // lists indexed by table entry (2^T <= E) or by claiming ray
    void *d_pairs;              // 2^hash_bits 16-byte slots: (claiming ray, id) pair + smallest ray id
    uint64_t *d_rec_key;        // E
    uint32_t *d_rec_idx;        // E (kNone = no record)
    uint32_t *d_rec_leaf;       // E
    uint32_t *d_rec_status;     // E
    uint64_t *d_queue;          // E fallback entries: ray id | seed leaf << 32
    uint8_t *d_dirty;           // ceil(2^T / 16) reset marks
    uint32_t *d_ctrl;           // [0, 8) sub-queue counts
    size_t table_bytes;
};
