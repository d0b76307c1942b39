// First-fit range allocator over a fixed byte range: the serving arena's HBM
// budget for result slots.  Host-only, not thread-safe (the server holds its
// lock around every call).  Offsets and sizes are rounded up to `align`.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace dare {

class RangeAlloc {
public:
    RangeAlloc() = default;
    RangeAlloc(uint64_t base, uint64_t size, uint64_t align = 256) { reset(base, size, align); }

    void reset(uint64_t base, uint64_t size, uint64_t align = 256) {
        align_ = align ? align : 1;
        const uint64_t b = round_up(base);
        const uint64_t end = base + size;
        free_.clear();
        base_ = b;
        capacity_ = end > b ? (end - b) / align_ * align_ : 0;
        if (capacity_) free_[b] = capacity_;
        used_ = 0;
    }

    // Offset of a new block, or UINT64_MAX when no free range is large enough.
    uint64_t alloc(uint64_t bytes) {
        const uint64_t need = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const uint64_t off = it->first;
            const uint64_t rest = it->second - need;
            free_.erase(it);
            if (rest) free_[off + need] = rest;
            used_ += need;
            return off;
        }
        return UINT64_MAX;
    }

    // Return a block; neighbouring free ranges are merged.
    void release(uint64_t off, uint64_t bytes) {
        const uint64_t len = round_up(bytes ? bytes : 1);
        used_ -= len;
        auto it = free_.emplace(off, len).first;
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
                it = prev;
            }
        }
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
    }

    bool fits_ever(uint64_t bytes) const { return round_up(bytes ? bytes : 1) <= capacity_; }
    uint64_t capacity() const { return capacity_; }
    uint64_t used() const { return used_; }
    size_t free_ranges() const { return free_.size(); }

private:
    uint64_t round_up(uint64_t x) const { return (x + align_ - 1) / align_ * align_; }
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t base_ = 0, capacity_ = 0, used_ = 0, align_ = 256;
};

}  // namespace dare
