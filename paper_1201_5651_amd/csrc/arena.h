// arena.h -- first-fit placement of byte ranges inside one allocation of
// `size` bytes, in 256-byte granules, with neighbouring free ranges merged on
// release.  Host bookkeeping only (no device calls), so it is testable alone.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace pi {

struct ArenaMap {
    size_t size = 0;
    size_t used = 0;
    std::map<size_t, size_t> free_;   // offset -> length of each free range

    static size_t round(size_t n) { return (n + 255) & ~size_t(255); }

    void init(size_t bytes)
    {
        size = bytes & ~size_t(255);
        used = 0;
        free_.clear();
        if (size) free_[0] = size;
    }

    // Lowest-offset free range that holds n bytes; false if none does.
    bool alloc(size_t n, size_t* off)
    {
        n = round(n);
        if (n == 0) n = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[o + n] = len - n;
            used += n;
            *off = o;
            return true;
        }
        return false;
    }

    // Returns [off, off + n) (as allocated) to the free ranges.
    void release(size_t off, size_t n)
    {
        n = round(n);
        if (n == 0) n = 256;
        used -= n;
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
};

}  // namespace pi
