// Host memory of bricks moved out of a volume's HBM pool (out-of-core bricks).  Host-only C++, no
// HIP, so that it is also built and tested on its own.  Not thread-safe: a volume's calls do not
// overlap.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <memory>
#include <unordered_map>
#include <vector>

namespace dare {

// Host memory of bricks moved out of HBM: each brick's 512 exact accumulators in a 4 KB block,
// blocks carved from 16 MB chunks and reused once their brick comes back (the chunks stay until
// clear() or the volume's end).
class HeldStore {
public:
    static constexpr uint32_t kChunkBlocks = 4096;
    static constexpr size_t kBlockWords = 512;

    bool empty() const { return index_.empty(); }
    size_t size() const { return index_.size(); }
    const std::unordered_map<int64_t, uint32_t>& index() const { return index_; }

    // The block of `entry`, or nullptr when it holds none.
    unsigned long long* find(int64_t entry) {
        auto it = index_.find(entry);
        return it == index_.end() ? nullptr : block(it->second);
    }
    // The block of `entry`, a new one (contents undefined, `fresh` set) when it held none.
    unsigned long long* add(int64_t entry, bool& fresh) {
        auto it = index_.find(entry);
        fresh = it == index_.end();
        if (!fresh) return block(it->second);
        uint32_t b;
        if (!free_.empty()) {
            b = free_.back();
            free_.pop_back();
        } else {
            if (next_ == chunks_.size() * kChunkBlocks)
                chunks_.emplace_back(new unsigned long long[(size_t)kChunkBlocks * kBlockWords]);
            b = next_++;
        }
        index_.emplace(entry, b);
        return block(b);
    }
    void erase(int64_t entry) {
        auto it = index_.find(entry);
        if (it == index_.end()) return;
        free_.push_back(it->second);
        index_.erase(it);
    }
    void clear() {
        index_.clear();
        free_.clear();
        chunks_.clear();
        next_ = 0;
    }

private:
    unsigned long long* block(uint32_t b) { return chunks_[b / kChunkBlocks].get() + (size_t)(b % kChunkBlocks) * kBlockWords; }
    std::unordered_map<int64_t, uint32_t> index_;
    std::vector<std::unique_ptr<unsigned long long[]>> chunks_;
    std::vector<uint32_t> free_;
    uint32_t next_ = 0;
};

}  // namespace dare
