// Device sort and prefix sum of the linear-BVH build (internal).
//
// radix_sort_pairs: a stable least-significant-digit radix sort of (64-bit
// key, 32-bit value) pairs, 8-bit digits, three launches per digit and no
// workgroup ever waiting on another:
//   k_sort_count    each wave counts the digits of its sub-tile of 1024 items
//                   into counts[digit][sub-tile] (digit-major);
//   k_sort_scan     block d scans row d of that table in place, so that it
//                   holds where sub-tile w's run of digit d starts among the
//                   items of digit d, and writes the row's total;
//   k_sort_scatter  each wave ranks its sub-tile stably (peers of a digit found
//                   with eight wave ballots), stages it in LDS in digit order,
//                   and writes each digit's run to its place, so that lanes of
//                   a wave store consecutive addresses.
// exclusive_scan_u32: tile sums, a scan of the sums, and a scan of each tile.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>

#include "device_sort.h"

namespace hrpp {
namespace {

constexpr uint32_t kDigitBits = 8;
constexpr uint32_t kDigits = 1u << kDigitBits;
constexpr uint32_t kLaneDigits = kDigits / 64;       // consecutive digits owned by one lane
constexpr uint32_t kWaveItems = 1024;               // items of one wave's sub-tile
constexpr uint32_t kRounds = kWaveItems / 64;       // rounds of one item per lane
constexpr uint32_t kSortWaves = 2;                  // waves per block of the count and scatter kernels
constexpr uint32_t kSortThreads = 64 * kSortWaves;
constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kRowThreads = 1024;              // threads of the per-digit row scan
constexpr uint32_t kScanTile = kScanThreads * 16;   // items per block of the prefix sum


inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// LDS accesses of one wave are performed in issue order; this keeps the
// compiler from moving them across the point.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive sum over the THREADS threads of a block (all must call it);
// *total receives the block's sum.  Uses wsum[THREADS / 64].
template <uint32_t THREADS>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const uint32_t incl = wave_inclusive_sum(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t k = 0; k < THREADS / 64; k++) {
        if (k < wave) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();   // wsum may be reused at once
    *total = all;
    return before + incl - v;
}

// The lanes of the wave that hold a valid item of digit d (meaningful for
// valid lanes only).
__device__ __forceinline__ uint64_t digit_peers(bool valid, uint32_t d) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (uint32_t b = 0; b < kDigitBits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t set = __ballot(valid && bit);
        m &= bit ? set : ~set;
    }
    return m;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint64_t *__restrict__ keys, uint32_t n,
                                                             uint32_t shift, uint32_t ntw,
                                                             uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[kSortWaves][kDigits];
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const uint32_t w = blockIdx.x * kSortWaves + wave;
    if (w >= ntw) return;                              // uniform per wave; no block barrier follows
    for (uint32_t d = lane; d < kDigits; d += 64) hist[wave][d] = 0;
    wave_lds_order();
    const size_t first = (size_t)w * kWaveItems;
    uint32_t digit[kRounds];                           // all loads in flight before the first count
#pragma unroll
    for (uint32_t r = 0; r < kRounds; r++) {
        const size_t i = first + r * 64u + lane;
        digit[r] = i < n ? (uint32_t)(keys[i] >> shift) & (kDigits - 1) : kDigits;
    }
#pragma unroll
    for (uint32_t r = 0; r < kRounds; r++)
        if (digit[r] < kDigits) atomicAdd(&hist[wave][digit[r]], 1u);
    wave_lds_order();
    for (uint32_t d = lane; d < kDigits; d += 64) counts[(size_t)d * ntw + w] = hist[wave][d];
}

__global__ __launch_bounds__(kRowThreads) void k_sort_scan(uint32_t *__restrict__ counts, uint32_t ntw,
                                                           uint32_t *__restrict__ totals) {
    __shared__ uint32_t wsum[kRowThreads / 64];
    uint32_t *row = counts + (size_t)blockIdx.x * ntw;
    uint32_t carry = 0;
    for (uint32_t c = 0; c < ntw; c += kRowThreads) {
        const uint32_t i = c + threadIdx.x;
        const uint32_t v = i < ntw ? row[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_sum<kRowThreads>(v, wsum, &total);
        if (i < ntw) row[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t *__restrict__ kin,
                                                               const uint32_t *__restrict__ vin,
                                                               uint64_t *__restrict__ kout,
                                                               uint32_t *__restrict__ vout, uint32_t n,
                                                               uint32_t shift, uint32_t ntw,
                                                               const uint32_t *__restrict__ counts,
                                                               const uint32_t *__restrict__ totals) {
    __shared__ uint32_t s_base[kDigits];                 // first position of each digit in the output
    __shared__ uint32_t s_run[kSortWaves][kDigits];      // next staging slot of each digit
    __shared__ uint32_t s_delta[kSortWaves][kDigits];    // output position minus staging slot, per digit
    __shared__ uint64_t s_key[kSortWaves][kWaveItems];
    __shared__ uint32_t s_val[kSortWaves][kWaveItems];
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (wave == 0) {
        // exclusive sum of the digit totals; lane L owns digits
        // kLaneDigits * L .. kLaneDigits * (L + 1) - 1
        uint32_t t[kLaneDigits], s = 0;
#pragma unroll
        for (uint32_t k = 0; k < kLaneDigits; k++) {
            t[k] = totals[kLaneDigits * lane + k];
            s += t[k];
        }
        uint32_t at = wave_inclusive_sum(s) - s;
#pragma unroll
        for (uint32_t k = 0; k < kLaneDigits; k++) {
            s_base[kLaneDigits * lane + k] = at;
            at += t[k];
        }
    }
    __syncthreads();
    const uint32_t w = blockIdx.x * kSortWaves + wave;
    if (w >= ntw) return;                              // uniform per wave; no block barrier follows
    // every lane's items in registers first, so that their loads are in flight
    // together (and with the counts below) rather than one round at a time
    const size_t first = (size_t)w * kWaveItems;
    uint64_t keys[kRounds];
    uint32_t vals[kRounds];
#pragma unroll
    for (uint32_t r = 0; r < kRounds; r++) {
        const size_t i = first + r * 64u + lane;
        keys[r] = i < n ? kin[i] : 0ull;
        vals[r] = i < n ? vin[i] : 0u;
    }
    // this sub-tile's count of each digit (differences of the scanned row) and
    // the start of its run in staging and in the output
    uint32_t cnt[kLaneDigits], out_at[kLaneDigits], s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kLaneDigits; k++) {
        const uint32_t d = kLaneDigits * lane + k;
        const uint32_t *row = counts + (size_t)d * ntw;
        const uint32_t at = row[w];
        const uint32_t next = w + 1 < ntw ? row[w + 1] : totals[d];
        cnt[k] = next - at;
        out_at[k] = s_base[d] + at;
        s += cnt[k];
    }
    uint32_t stage = wave_inclusive_sum(s) - s;
#pragma unroll
    for (uint32_t k = 0; k < kLaneDigits; k++) {
        const uint32_t d = kLaneDigits * lane + k;
        s_run[wave][d] = stage;
        s_delta[wave][d] = out_at[k] - stage;
        stage += cnt[k];
    }
    wave_lds_order();
    // stage the items in digit order, each digit's items in input order
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (uint32_t r = 0; r < kRounds; r++) {
        const bool valid = first + r * 64u + lane < n;
        const uint64_t key = keys[r];
        const uint32_t val = vals[r];
        const uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1);
        const uint64_t peers = digit_peers(valid, d);
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        const uint32_t slot = valid ? s_run[wave][d] + rank : 0u;
        wave_lds_order();                              // every lane has read its digit's slot
        if (valid) {
            if (rank == 0) s_run[wave][d] += (uint32_t)__popcll(peers);
            s_key[wave][slot] = key;
            s_val[wave][slot] = val;
        }
        wave_lds_order();
    }
    // write the staged items out: consecutive slots of one digit go to
    // consecutive output positions
    const uint32_t items = (uint32_t)((size_t)n - first < kWaveItems ? (size_t)n - first : kWaveItems);
    for (uint32_t p = lane; p < items; p += 64) {
        const uint64_t key = s_key[wave][p];
        const uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1);
        const uint32_t o = s_delta[wave][d] + p;
        kout[o] = key;
        vout[o] = s_val[wave][p];
    }
}

// Prefix sum: per-tile sums, their exclusive scan (one block), then each tile.
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(const uint32_t *__restrict__ in, uint32_t n,
                                                                 uint32_t *__restrict__ sums) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t first = (size_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (uint32_t r = 0; r < kScanTile / kScanThreads; r++) {
        const size_t i = first + r * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t total;
    (void)block_exclusive_sum<kScanThreads>(s, wsum, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t *__restrict__ sums, uint32_t m) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < m; c += kScanThreads) {
        const uint32_t i = c + threadIdx.x;
        const uint32_t v = i < m ? sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_sum<kScanThreads>(v, wsum, &total);
        if (i < m) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const uint32_t *__restrict__ in,
                                                             uint32_t *__restrict__ out, uint32_t n,
                                                             const uint32_t *__restrict__ sums) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t first = (size_t)blockIdx.x * kScanTile;
    uint32_t carry = sums[blockIdx.x];
    for (uint32_t r = 0; r < kScanTile / kScanThreads; r++) {
        const size_t i = first + r * kScanThreads + threadIdx.x;
        const uint32_t v = i < n ? in[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_sum<kScanThreads>(v, wsum, &total);
        if (i < n) out[i] = carry + ex;
        carry += total;
    }
}

inline uint32_t sort_subtiles(uint32_t n) { return (uint32_t)(((size_t)n + kWaveItems - 1) / kWaveItems); }
inline uint32_t scan_tiles(uint32_t n) { return (uint32_t)(((size_t)n + kScanTile - 1) / kScanTile); }

}  // namespace

size_t radix_sort_scratch_bytes(uint32_t n) {
    const size_t ntw = sort_subtiles(n);
    return align256(kDigits * ntw * sizeof(uint32_t)) + align256(kDigits * sizeof(uint32_t));
}

hipError_t radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t n, uint32_t end_bit,
                            void *scratch, hipStream_t s, uint32_t *result_in) {
    *result_in = 0;
    if (n == 0 || end_bit == 0) return hipSuccess;
    if (end_bit > 64) return hipErrorInvalidValue;
    const uint32_t ntw = sort_subtiles(n);
    auto *counts = static_cast<uint32_t *>(scratch);
    auto *totals = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) +
                                                align256(kDigits * (size_t)ntw * sizeof(uint32_t)));
    const dim3 grid((ntw + kSortWaves - 1) / kSortWaves);
    uint64_t *kin = k0, *kout = k1;
    uint32_t *vin = v0, *vout = v1;
    for (uint32_t shift = 0; shift < end_bit; shift += kDigitBits) {
        hipLaunchKernelGGL(k_sort_count, grid, dim3(kSortThreads), 0, s, kin, n, shift, ntw, counts);
        hipLaunchKernelGGL(k_sort_scan, dim3(kDigits), dim3(kRowThreads), 0, s, counts, ntw, totals);
        hipLaunchKernelGGL(k_sort_scatter, grid, dim3(kSortThreads), 0, s, kin, vin, kout, vout, n, shift, ntw,
                           counts, totals);
        std::swap(kin, kout);
        std::swap(vin, vout);
        *result_in ^= 1u;
    }
    return hipGetLastError();
}

size_t exclusive_scan_scratch_bytes(uint32_t n) { return align256((size_t)scan_tiles(n) * sizeof(uint32_t)); }

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, void *scratch, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t m = scan_tiles(n);
    auto *sums = static_cast<uint32_t *>(scratch);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(m), dim3(kScanThreads), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, m);
    hipLaunchKernelGGL(k_scan_tiles, dim3(m), dim3(kScanThreads), 0, s, in, out, n, sums);
    return hipGetLastError();
}

}  // namespace hrpp
