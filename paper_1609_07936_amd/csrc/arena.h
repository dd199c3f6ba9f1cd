// arena.h -- the served loop's device-memory arena: first-fit placement of
// job blocks in one caller-sized allocation, 4 KiB granules, freed blocks
// merged with free neighbours.  Pure host code (offsets only; the memory is
// never touched), so it is tested on the CPU as well.
#ifndef SAIL_ARENA_H
#define SAIL_ARENA_H

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace sail_arena {

// base/size: the allocation the arena hands out; free_: offset -> bytes of
// every free extent, none adjacent to another; used/peak: bytes handed out
// now and at most.  Set up with base, size and free_[0] = size.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    static size_t round_up(size_t n) { return (n + 4095) & ~(size_t)4095; }
    char *take(size_t n)
    {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used += n;
            peak = std::max(peak, used);
            return base + off;
        }
        return nullptr;
    }
    void give(char *q, size_t n)
    {
        n = round_up(n);
        size_t off = (size_t)(q - base);
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

}  // namespace sail_arena

#endif
