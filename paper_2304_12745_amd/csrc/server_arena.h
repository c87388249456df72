// Offsets-only allocator of the serving arena (host code, no HIP).
//
// The arena is one device buffer allocated when the server is created.  Query
// scratch takes the lowest free block that fits (first fit).  Resident data
// (deployment geometry and the DMIMO_PA schedule), which stays for the
// server's life, is one stack at the top: a resident block is taken from the
// free block just below the stack, or not at all.  Resident blocks therefore
// never sit between query blocks: once no query is running, the space below
// the stack is one free block, so a query whose scratch fits the budget left
// by the resident data always finds room.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace dmimo {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

class Arena {
  public:
    // the usable size is rounded down to a multiple of 256 bytes
    void init(size_t size) {
        free_.clear();
        size_ = size & ~size_t(255);
        floor_ = size_;
        if (size_) free_[0] = size_;
    }

    size_t size() const { return size_; }
    // lowest offset of the resident stack (size() when it is empty)
    size_t resident_floor() const { return floor_; }

    // lowest free block that holds `bytes` (rounded up to 256)
    bool alloc_low(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }

    // the top of the free block just below the resident stack, which grows
    // down by `bytes` (rounded up to 256); false if that block is missing or
    // too small (queries hold the space under the stack)
    bool alloc_high(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        if (bytes == 0) bytes = 256;
        auto it = free_.lower_bound(floor_);
        if (it == free_.begin()) return false;
        --it;
        if (it->first + it->second != floor_ || it->second < bytes) return false;
        const size_t start = it->first;
        const size_t len = it->second;
        *off = start + len - bytes;
        if (len == bytes)
            free_.erase(start);
        else
            it->second = len - bytes;
        floor_ = *off;
        return true;
    }

    // give back a block from alloc_low, or the lowest block of the resident
    // stack (same byte count)
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        if (bytes == 0) bytes = 256;
        if (off == floor_) floor_ += bytes;
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

    size_t free_bytes() const {
        size_t s = 0;
        for (const auto& kv : free_) s += kv.second;
        return s;
    }

    size_t largest_free() const {
        size_t s = 0;
        for (const auto& kv : free_) s = kv.second > s ? kv.second : s;
        return s;
    }

    size_t blocks() const { return free_.size(); }

    // the free blocks, in address order (for checks)
    const std::map<size_t, size_t>& free_list() const { return free_; }

  private:
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, coalesced
    size_t size_ = 0;
    size_t floor_ = 0;                // resident stack: [floor_, size_)
};

}  // namespace dmimo
