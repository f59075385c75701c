// Host-only checks of the context's sub-allocator (arena.cpp): random
// alloc / alloc_high / grow / shrink / free sequences against a shadow map of
// the allocations, with the arena's own accounting checked after every step.
#include "arena.h"

#include <cstdio>
#include <map>
#include <random>
#include <vector>

using svh::Arena;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);            \
            if (++failures > 20) return 1;                              \
        }                                                               \
    } while (0)

static uint64_t r256(uint64_t b) { return ((b ? b : 1) + 255) & ~255ull; }

int main() {
    static char region[1];   // only its address is used: the arena hands out offsets
    char *base = region;
    const uint64_t size = 1ull << 30;
    Arena a;
    a.init(base, size);
    std::map<uint64_t, uint64_t> shadow;   // offset -> bytes
    std::mt19937_64 rng(7);
    auto check_all = [&]() -> int {
        uint64_t used = 0, end = 0;
        for (auto &kv : shadow) {
            CHECK(kv.first >= end);   // no overlap, sorted
            end = kv.first + kv.second;
            used += kv.second;
        }
        CHECK(end <= size);
        CHECK(a.used_bytes() == used);
        CHECK(a.free_bytes() + used == size);
        return 0;
    };
    for (int step = 0; step < 20000; ++step) {
        const int op = (int)(rng() % 6);
        if (op <= 1 || shadow.empty()) {
            const uint64_t b = 1 + rng() % (1ull << (8 + rng() % 16));
            const uint64_t al = 1ull << (8 + rng() % 9);
            void *p = op == 0 ? a.alloc(b, al) : a.alloc_high(b, al);
            if (p) {
                const uint64_t off = (uint64_t)((char *)p - base);
                CHECK(off % al == 0);
                CHECK(shadow.find(off) == shadow.end());
                shadow[off] = r256(b);
            }
        } else {
            auto it = shadow.begin();
            std::advance(it, rng() % shadow.size());
            char *p = base + it->first;
            if (op == 2) {
                a.free(p);
                shadow.erase(it);
            } else if (op == 3) {
                const uint64_t nb = it->second + 1 + rng() % (1ull << 20);
                // expected: the next allocation (or the end) leaves room
                auto nx = std::next(it);
                const uint64_t limit = nx == shadow.end() ? size : nx->first;
                const bool room = it->first + r256(nb) <= limit;
                const bool ok = a.grow(p, nb);
                CHECK(ok == room);
                if (ok) it->second = r256(nb);
            } else if (op == 4) {
                const uint64_t nb = 1 + rng() % it->second;
                a.shrink(p, nb);
                it->second = std::min(it->second, r256(nb));
            } else {
                CHECK(a.contains(p));
            }
        }
        if (check_all()) return 1;
    }
    // freeing everything coalesces back to one extent
    for (auto &kv : shadow) a.free(base + kv.first);
    CHECK(a.free_bytes() == size && a.largest_free() == size);
    // alloc_high takes the top end; grow into the space a shrink returned
    void *lo = a.alloc(1 << 20), *hi = a.alloc_high(4096);
    CHECK((char *)hi - base == (int64_t)(size - 4096));
    CHECK(lo == base);
    a.shrink(lo, 1 << 19);
    CHECK(a.grow(lo, 1 << 20));
    CHECK(a.grow(lo, size - 4096));
    CHECK(!a.grow(lo, size - 4096 + 256));
    // grow_around: room above only, below only, and split between the two
    a.free(lo);
    a.free(hi);
    {
        const uint64_t U = 1 << 20;
        char *b1 = (char *)a.alloc(U, U);           // [0, 1M)
        char *blk = (char *)a.alloc(U, U);          // [1M, 2M)
        char *b3 = (char *)a.alloc(U, U);           // [2M, 3M)
        uint64_t k = 99;
        CHECK(a.grow_around(blk, 2, U, U, &k) == nullptr);   // no room on either side
        a.free(b3);                                  // room above
        CHECK(a.grow_around(blk, 4, U, U, &k) == blk && k == 0);
        a.shrink(blk, U);
        a.free(b1);                                  // room below too: k = 0 still first
        char *big = (char *)a.alloc(U << 3, U);      // fill above from 2M on
        CHECK(big == blk + U);
        CHECK(a.grow_around(blk, 2, U, U, &k) == blk - U && k == 1);   // only below
        CHECK(a.used_bytes() == (2 * U) + (U << 3));
        a.free(blk - U);
        a.free(big);
        CHECK(a.free_bytes() == size && a.largest_free() == size);
    }
    if (failures) return 1;
    std::printf("all checks passed\n");
    return 0;
}
