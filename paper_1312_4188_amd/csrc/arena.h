// First-fit allocator over the offsets [0, size) of one memory block, with
// coalescing frees.  Host-only code (no HIP): the serving runtime places
// in-flight groups of requests with it.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace fw {

class Arena {
   public:
    explicit Arena(size_t size) {
        if (size) free_[0] = size;
    }

    // Lowest free offset with `need` bytes after it; false if none.
    bool alloc(size_t need, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need, at = it->first + need;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }

    // Return [off, off + size), merging it with free neighbours.
    void release(size_t off, size_t size) {
        if (size == 0) return;
        auto it = free_.emplace(off, size).first;
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

    // Size of the largest free block (0 when full).
    size_t largest() const {
        size_t m = 0;
        for (const auto& kv : free_)
            if (kv.second > m) m = kv.second;
        return m;
    }

    // Free blocks as (offset, size), in offset order.
    const std::map<size_t, size_t>& blocks() const { return free_; }

   private:
    std::map<size_t, size_t> free_;
};

}  // namespace fw
