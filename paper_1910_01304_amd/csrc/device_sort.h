// Device sort and prefix sum of the linear-BVH build (internal; device_sort.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hrpp {

// Scratch bytes of radix_sort_pairs for n pairs.
size_t radix_sort_scratch_bytes(uint32_t n);
// Stable sort of n (key, value) pairs by the key's bits [0, end_bit), 8 bits
// per pass, enqueued on s.  The pairs start in (k0, v0); passes alternate
// between (k0, v0) and (k1, v1), and *result_in says which of the two holds
// the sorted pairs at the end (0 or 1).  scratch: radix_sort_scratch_bytes(n)
// bytes, 256-byte aligned.
hipError_t radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t n, uint32_t end_bit,
                            void *scratch, hipStream_t s, uint32_t *result_in);

// Scratch bytes of exclusive_scan_u32 for n words.
size_t exclusive_scan_scratch_bytes(uint32_t n);
// out[i] = in[0] + ... + in[i - 1] (modulo 2^32), enqueued on s; out may not
// alias in.
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, void *scratch, hipStream_t s);

}  // namespace hrpp
