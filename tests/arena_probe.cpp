// Host-only C entry points over the served loop's arena, for the CPU tests.
// The arena works on a real host buffer of the given size, which it never
// reads or writes (it hands out offsets into it).
#include <cstdint>
#include <cstdlib>

#include "../paper_1609_07936_amd/csrc/arena.h"

namespace {
struct Probe {
    char *buf = nullptr;
    sail_arena::Arena a;
};
}  // namespace

extern "C" {

void *arena_new(size_t size)
{
    Probe *p = new Probe;
    p->buf = static_cast<char *>(std::malloc(size));
    p->a.base = p->buf;
    p->a.size = size;
    p->a.free_[0] = size;
    return p;
}

void arena_delete(void *h)
{
    Probe *p = static_cast<Probe *>(h);
    std::free(p->buf);
    delete p;
}

// offset of a new block of n bytes, or -1 when no free extent holds it
int64_t arena_take(void *h, size_t n)
{
    Probe *p = static_cast<Probe *>(h);
    char *q = p->a.take(n);
    return q ? (int64_t)(q - p->buf) : -1;
}

void arena_give(void *h, int64_t off, size_t n)
{
    Probe *p = static_cast<Probe *>(h);
    p->a.give(p->buf + off, n);
}

size_t arena_used(void *h) { return static_cast<Probe *>(h)->a.used; }
size_t arena_peak(void *h) { return static_cast<Probe *>(h)->a.peak; }

// the free extents in offset order; returns their count (at most max written)
int arena_free_extents(void *h, int64_t *off, int64_t *len, int max)
{
    Probe *p = static_cast<Probe *>(h);
    int k = 0;
    for (const auto &e : p->a.free_) {
        if (k < max) {
            off[k] = (int64_t)e.first;
            len[k] = (int64_t)e.second;
        }
        ++k;
    }
    return k;
}

}  // extern "C"
