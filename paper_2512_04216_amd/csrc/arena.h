// arena.h -- first-fit sub-allocator over one device block (host code, no
// HIP calls: it only hands out offsets of a block the context owns).
#pragma once

#include <cstdint>
#include <map>
#include <mutex>

namespace svh {

class Arena {
  public:
    void init(char *base, uint64_t size);
    // lowest extent that fits; nullptr when none does
    void *alloc(uint64_t bytes, uint64_t align = 256);
    // highest extent that fits, taken at its top end (small long-lived
    // objects, kept away from the space that large ones grow into)
    void *alloc_high(uint64_t bytes, uint64_t align = 256);
    // extend the allocation at p in place to `bytes` when the free extent
    // right after it is large enough; false (nothing changed) otherwise
    bool grow(void *p, uint64_t bytes);
    // extend the allocation at p (currently `unit` bytes) to units * unit
    // bytes around itself: the old bytes end up at unit position *k of the new
    // allocation, with k * unit taken from the free extent just below p and the
    // rest from the one just above (the lowest k that fits and keeps the new
    // start aligned). Returns the new start, nullptr (nothing changed) if no k
    // fits.
    void *grow_around(void *p, uint64_t units, uint64_t unit, uint64_t align, uint64_t *k);
    // give back the part of the allocation at p beyond `bytes`
    void shrink(void *p, uint64_t bytes);
    void free(void *p);
    uint64_t free_bytes() const;
    uint64_t largest_free() const;
    uint64_t used_bytes() const;
    uint64_t size() const { return size_; }
    bool contains(const void *p) const;

  private:
    void insert_free(uint64_t start, uint64_t len);   // with coalescing; caller holds mu_
    mutable std::mutex mu_;
    char *base_ = nullptr;
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    std::map<uint64_t, uint64_t> used_;   // offset -> length
};

}  // namespace svh
