// arena.h -- first-fit allocator over one caller-provided byte range, used by
// the request server to place each admitted solve's workspace and outputs.
// Host-only logic (no HIP calls): offsets are handed out, the caller adds the
// base address.  Blocks are aligned to 256 bytes; freeing coalesces with both
// neighbours, so a fully released arena is again one free block.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>

namespace htree {

class Arena {
  public:
    static constexpr size_t kAlign = 256;
    static constexpr size_t kNone = ~(size_t)0;

    // The usable range is [0, bytes) rounded down to the alignment.
    explicit Arena(size_t bytes) : size_(bytes & ~(kAlign - 1)) {
        if (size_) free_[0] = size_;
    }

    static size_t round_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

    // Offset of a block of at least `bytes` (lowest address that fits), or
    // kNone when no free block is large enough.
    size_t alloc(size_t bytes) {
        if (bytes == 0) bytes = kAlign;
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            if (used_ > peak_) peak_ = used_;
            live_[off] = bytes;
            return off;
        }
        return kNone;
    }

    // Returns false (and changes nothing) for an offset that is not live.
    bool release(size_t off) {
        auto lv = live_.find(off);
        if (lv == live_.end()) return false;
        size_t bytes = lv->second;
        live_.erase(lv);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return true;
            }
        }
        free_[off] = bytes;
        return true;
    }

    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const {
        size_t b = 0;
        for (auto &f : free_)
            if (f.second > b) b = f.second;
        return b;
    }
    size_t free_blocks() const { return free_.size(); }
    size_t live_blocks() const { return live_.size(); }

  private:
    size_t size_;
    size_t used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;    // offset -> bytes, disjoint, never adjacent
    std::map<size_t, size_t> live_;    // offset -> bytes
};

}  // namespace htree
