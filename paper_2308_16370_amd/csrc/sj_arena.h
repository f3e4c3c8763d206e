// First-fit allocator over the offsets of a caller-provided device buffer (host-side
// bookkeeping only). Used by the serving extension and by the filter catalogue.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace sj {

inline uint64_t round256(uint64_t b) { return (b + 255) & ~uint64_t(255); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(uint64_t size) : size_(size) {
        if (size_) free_[0] = size_;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = round256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = round256(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

   private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_, used_ = 0, peak_ = 0;
};

}  // namespace sj
