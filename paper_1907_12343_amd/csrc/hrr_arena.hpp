// hrr_arena.hpp -- first-fit allocator over one device arena (offsets only;
// no device calls), used by the serving loop to carve its HBM budget into
// request eye copies and result arrays.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace hrr {

// Blocks are kAlign-aligned and rounded up to kAlign bytes; a zero-byte
// request takes one kAlign block.  Free blocks are kept by offset and
// coalesced with their neighbours on release.  Not thread-safe.
class Arena {
public:
    static constexpr uint64_t kAlign = 256;
    static uint64_t round_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

    void init(uint64_t size) {
        size_ = size / kAlign * kAlign;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }
    // Lowest-offset free block that fits; false if none.
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = round_up(std::max<uint64_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    // Return a block obtained from alloc (same byte count).
    void release(uint64_t off, uint64_t bytes) {
        bytes = round_up(std::max<uint64_t>(bytes, 1));
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        uint64_t lo = off, hi = off + bytes;
        if (next != free_.end() && next->first == hi) {
            hi += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == lo) {
                lo = prev->first;
                free_.erase(prev);
            }
        }
        free_[lo] = hi - lo;
    }
    // Keep the first new_bytes of a block of old_bytes, free the rest.
    void shrink(uint64_t off, uint64_t old_bytes, uint64_t new_bytes) {
        old_bytes = round_up(std::max<uint64_t>(old_bytes, 1));
        new_bytes = round_up(std::max<uint64_t>(new_bytes, 1));
        if (new_bytes < old_bytes) release(off + new_bytes, old_bytes - new_bytes);
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

private:
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace hrr
