// The request loop's device-memory arena (host-side bookkeeping only).
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace aesgpu {

// Next-fit arena allocator with coalescing of free neighbours: the search
// starts where the previous allocation ended and wraps around, so memory is
// reused in roughly the order it was taken (requests finish roughly in
// arrival order) and a freed region is not handed out again at once.
class Arena {
  public:
    explicit Arena(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off) {
        // 1. from the cursor on, inside the free block that holds it
        auto it = free_.upper_bound(cursor_);
        if (it != free_.begin()) {
            auto p = std::prev(it);
            const uint64_t start = p->first, end = p->first + p->second;
            if (start <= cursor_ && end > cursor_ && end - cursor_ >= n) {
                free_.erase(p);
                if (cursor_ > start)
                    free_[start] = cursor_ - start;
                if (end > cursor_ + n)
                    free_[cursor_ + n] = end - cursor_ - n;
                *off = cursor_;
                cursor_ += n;
                return true;
            }
        }
        // 2. the first block after the cursor that fits, then 3. wrap around
        for (it = free_.upper_bound(cursor_); it != free_.end(); ++it)
            if (it->second >= n)
                return take(it, n, off);
        for (it = free_.begin(); it != free_.end() && it->first <= cursor_; ++it)
            if (it->second >= n)
                return take(it, n, off);
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

    // Free blocks as (offset, size), in address order.
    const std::map<uint64_t, uint64_t> &free_blocks() const { return free_; }

  private:
    bool take(std::map<uint64_t, uint64_t>::iterator it, uint64_t n, uint64_t *off) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest)
            free_[at] = rest;
        cursor_ = at;
        return true;
    }

    std::map<uint64_t, uint64_t> free_;
    uint64_t cursor_ = 0;
};

}  // namespace aesgpu
