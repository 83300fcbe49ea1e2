// Kernel argument blocks and launchers of the HRPP library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hrpp {

// Hash grid of one predictor (see hash_ray in hrpp_kernels.hip).
struct HashArgs {
    float bmin[3];
    float scale[3];     // 2^qo / extent per axis (0 for a flat axis)
    float maxo;         // 2^qo - 1
    float maxd;         // 2^qd - 1
    float half;         // 2^(qd - 1)
    uint32_t qo, qd, log2n;
    uint32_t mode;      // 0 grid + octahedral; 1 IEEE-754 bit fields at precision qo
    uint32_t stride;    // mode 1: field stride of the key, 8 or 16 bits
};

constexpr uint32_t kSubQueues = 8;     // striped fallback sub-queues per epoch
constexpr uint32_t kResetGroup = 16;   // table entries per reset mark
constexpr uint32_t kDefaultInlineLanes = 48;   // failing lanes of a wave that traverse at once

// Capacity of one sub-queue, sized as if prediction blocks held 256 rays:
// block b appends to sub-queue (b % kSubQueues), so with blocks of 128 rays a
// sub-queue receives at most ceil(ceil(E/128) / kSubQueues) * 128 rays, which
// never exceeds ceil(ceil(E/256) / kSubQueues) * 256.
// Size of the per-epoch (claiming ray, id) set: the power of two >= 2 E, so
// that it is at most half full.
inline uint32_t pair_hash_bits_for(uint32_t epoch) {
    uint32_t b = 1;
    while ((1ull << b) < 2ull * epoch) b++;
    return b;
}

inline uint32_t queue_subcap_for(uint32_t epoch) {
    const uint32_t blocks = (epoch + 255u) / 256u;
    return ((blocks + kSubQueues - 1u) / kSubQueues) * 256u;
}

// One slot of the per-epoch set of (claiming ray, id) pairs: the pair and the
// smallest ray id that recorded it, in one 16-byte record, so that a probe, its
// compare-and-swap and its minimum touch one cache line.
struct PairSlot {
    unsigned long long key;
    uint32_t min;
    uint32_t pad;
};

struct TraceArgs {
    // scene
    const void *nodes;            // interior nodes, 64 B each
    const void *tris;             // triangles, 48 B each
    const void *leafbox;          // leaf boxes by first triangle, 32 B each
    const void *cnode;            // canonical node records, 48 B each (predicted interior nodes)
    const void *wide;             // 4-wide nodes, 128 B each (plain-traversal baseline)
    uint32_t wide_root;           // wide node 0, or kLeafFlag | leaf id
    float root_box[6];
    uint32_t root_ref;
    uint32_t stack_cap;           // traversal stack slots per lane (>= deepest leaf)
    uint32_t max_blocks;          // grid cap of the persistent plain traversal
    // rays and results
    const void *rays;             // hrpp_ray[n]
    uint8_t *occluded;            // any-hit output
    void *hits;                   // closest-hit output (hrpp_hit[n])
    unsigned long long *stats;    // hrpp_stats or null
    uint32_t *error;              // device error word
    // predictor (null table = plain)
    void *table;
    uint32_t entry_bytes;
    uint32_t ways;
    uint32_t go_up;               // 0: slots hold leaf ids; g: canonical node g levels above the leaf
    uint32_t inline_min;          // failing lanes of a wave that traverse at once (65 = never)
    uint32_t policy;              // bit 0: FIFO eviction; bit 1: the resident tag keeps its entry
    HashArgs hash;
    uint32_t *ctrl;               // [0 .. kSubQueues) sub-queue counts
    uint8_t *dirty;               // reset marks, one per kResetGroup entries
    uint64_t *queue;              // kSubQueues sub-queues of queue_subcap entries
    uint32_t queue_subcap;
    uint64_t *rec_key;
    uint32_t *rec_idx;
    uint32_t *rec_leaf;
    uint32_t *rec_status;         // status | free slots << 2 | (hash slot + 1) << 8
    uint64_t *topw;               // W fresh (ray id << 32 | id), increasing, per claimed entry: indexed by
    uint32_t topw_by_entry;       // ... the entry (1, when the table has no more entries than an epoch
                                  // has rays) or by the claiming ray's offset in the epoch (0)
    PairSlot *pairs;              // per-epoch set of (claiming ray - base) << 32 | id
    uint32_t hash_bits;           // log2 of the set's size (>= 2 x the epoch)
    // measurement only (kernels with counters): a bitmap of the 128-byte lines
    // of the scene and table arrays each kernel kind touched (null = off)
    uint32_t *touch;
    uint32_t touch_kind_words;    // words per kernel kind (kTouchKinds blocks)
    uint32_t touch_off[5];        // word offset of each region within a block
};

// Regions and kernel kinds of the touch bitmap (hrpp_profile_touch).
enum TouchRegion : int { kTouchNodes, kTouchTris, kTouchLeafbox, kTouchEntries, kTouchCnode, kTouchRegions };
enum TouchKind : int { kTouchPredict, kTouchEmpty, kTouchQueue, kTouchPlain, kTouchKinds };

// One job of a batch (see hrpp_batch_create): its arguments, ray count, epoch
// size and the length of its first epoch (<= epoch).
struct BatchJob {
    TraceArgs a;
    uint32_t n, epoch, first, pad1;
};

enum BatchKind : int { kBatchAnyHrpp, kBatchPaperHrpp, kBatchExactHrpp, kBatchAnyPlain, kBatchClosestPlain };

// Jobs of one kind, listed in ids[first_id .. first_id + count).  Every
// launch of a group is one flat grid in which job k owns the blocks
// [off[k], off[k + 1]); offsets are increasing (every job has a block).
struct BatchGroup {
    int kind;
    uint32_t first_id, count, rounds;
    bool stats;
    bool subtree;                 // predictors of go-up level >= 1
    bool inline_any;              // some job traverses failing waves in place
    bool block_epochs;            // every job's epochs hold at most kBlockEpochRays rays: one
                                  // workgroup per job runs all of its epochs, in one launch
    // plain groups: blocks of 128 lanes covering each job's rays
    uint32_t total_blocks;
    const uint32_t *d_block_off;
    // predictor groups, per round: blocks of 128 lanes and of 256 lanes covering
    // each job's longest epoch, and the queue kernel's grid (128 lanes, at most
    // kQueueBlocks per job)
    uint32_t blocks128, blocks256, blocksq;
    const uint32_t *d_off128, *d_off256, *d_offq;
};

constexpr uint32_t kQueueBlocks = 4096;   // grid cap of one epoch's queue traversal
constexpr uint32_t kBlockEpochRays = 256; // epochs this small run a whole call in one workgroup

void launch_batch(const BatchJob *jobs, const uint32_t *ids, const std::vector<BatchGroup> &groups,
                  uint32_t max_rounds, uint32_t max_blocks, hipStream_t s);

enum KernelKind : int {
    kKindPredict, kKindTraverseQueue, kKindTraversePlain, kKindUpdateClassify, kKindUpdateApply,
    kKindUpdateFinish, kKindFill, kKindTraverseWide, kKindEpochEmpty, kKindResetTable, kKindUpdateRank,
    kKindEpochsBlock, kNumKernelKinds
};
const char *kernel_kind_name(int k);
void profile_start();
int profile_stop(double *ms, uint64_t *launches);   // synchronises the recorded events

// empty_table: the predictor was reset and not traced since (its first epoch
// then traverses in place).
// Epochs of `epoch` rays, the first one `first_epoch` rays long (<= epoch).
void launch_trace(const TraceArgs &a, uint32_t n, bool any, bool exact, bool hrpp, uint32_t epoch,
                  uint32_t first_epoch, bool empty_table, hipStream_t s);
void launch_fill32(uint32_t *p, size_t n, uint32_t value, hipStream_t s);
// Empties every group of kResetGroup entries whose mark is set (all groups
// when `full`) and clears the marks.
void launch_reset_table(void *table, uint32_t entry_bytes, uint32_t n_entries, uint8_t *dirty, bool full,
                        hipStream_t s);

// Device build of a linear BVH (bvh_device.hip).  The output regions are
// sized for the largest tree over n triangles: n - 1 interior nodes, n
// triangles and leaf-box slots, 2n - 1 canonical node records.
struct LbvhOut {
    void *nodes, *tris, *leafbox, *cnode;
};
struct LbvhResult {
    uint32_t bad;          // bit 0: non-finite vertex; bits 1-2: internal inconsistency
    uint32_t max_depth, num_nodes;
    float root_box[6];
};
// Scratch bytes for n triangles (0 for n = 0).
size_t lbvh_scratch_bytes(uint32_t n);
// The device build's static scratch (one per GPU, kStaticBuildScratchBytes):
// its device address on the current device, looked up on first use.
constexpr size_t kStaticBuildScratchBytes = size_t(64) << 20;
hipError_t lbvh_static_scratch(void **ptr);
// Enqueues the build on `s` and synchronises it: once to read the linear
// BVH's depth (a tree deeper than max_depth, or a non-finite vertex, ends
// the build there; with treelet passes, deeper than the walk limit), once
// per treelet pass and after the last one to read the levels' sizes and
// the depth, and once at the end.
hipError_t lbvh_build(const float *d_verts, uint32_t n, uint32_t leaf_max, uint32_t max_depth, uint32_t passes,
                      void *d_scratch, const LbvhOut &out, hipStream_t s, LbvhResult *res);

// Plain traversal of the 4-wide tree (a.wide, a.wide_root; a.stack_cap = the
// tree's stack need); closest hit is the exact one.
void launch_wide(const TraceArgs &a, uint32_t n, bool any, hipStream_t s);

}  // namespace hrpp
