// First-fit allocator of the serving pool (internal; host only, no HIP).
#pragma once

#include <algorithm>
#include <cstddef>
#include <map>

#include "hrpp_internal.h"

namespace hrpp {

// First-fit allocator over [0, size) with 256-byte granularity.
class PoolAllocator {
  public:
    explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t &off) {
        bytes = hrpp::align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = hrpp::align256(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

}  // namespace hrpp
