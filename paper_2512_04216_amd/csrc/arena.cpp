// arena.cpp -- the context's device-memory sub-allocator (offsets only).
#include "arena.h"

#include <algorithm>

namespace svh {

namespace {
uint64_t round256(uint64_t b) { return ((b ? b : 1) + 255) & ~255ull; }
}  // namespace

void Arena::init(char *base, uint64_t size) {
    std::lock_guard<std::mutex> g(mu_);
    base_ = base;
    size_ = size;
    free_.clear();
    used_.clear();
    if (size) free_[0] = size;
}

void *Arena::alloc(uint64_t bytes, uint64_t align) {
    std::lock_guard<std::mutex> g(mu_);
    bytes = round256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        const uint64_t off = it->first, len = it->second;
        const uint64_t a = (off + align - 1) / align * align;
        if (a + bytes > off + len) continue;
        free_.erase(it);
        if (a > off) free_[off] = a - off;
        if (a + bytes < off + len) free_[a + bytes] = off + len - (a + bytes);
        used_[a] = bytes;
        return base_ + a;
    }
    return nullptr;
}

void *Arena::alloc_high(uint64_t bytes, uint64_t align) {
    std::lock_guard<std::mutex> g(mu_);
    bytes = round256(bytes);
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
        const uint64_t off = it->first, len = it->second;
        if (len < bytes) continue;
        const uint64_t a = (off + len - bytes) / align * align;
        if (a < off) continue;
        free_.erase(off);
        if (a > off) free_[off] = a - off;
        if (a + bytes < off + len) free_[a + bytes] = off + len - (a + bytes);
        used_[a] = bytes;
        return base_ + a;
    }
    return nullptr;
}

bool Arena::grow(void *p, uint64_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    const uint64_t off = (uint64_t)((char *)p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    bytes = round256(bytes);
    const uint64_t cur = u->second;
    if (bytes <= cur) return true;
    auto nx = free_.find(off + cur);
    if (nx == free_.end() || nx->second < bytes - cur) return false;
    const uint64_t rest = nx->second - (bytes - cur);
    free_.erase(nx);
    if (rest) free_[off + bytes] = rest;
    u->second = bytes;
    return true;
}

void *Arena::grow_around(void *p, uint64_t units, uint64_t unit, uint64_t align, uint64_t *k) {
    std::lock_guard<std::mutex> g(mu_);
    const uint64_t off = (uint64_t)((char *)p - base_);
    auto u = used_.find(off);
    if (u == used_.end() || u->second != unit || units == 0) return nullptr;
    auto nx = free_.find(off + unit);
    const uint64_t after = nx == free_.end() ? 0 : nx->second;
    auto pv = free_.lower_bound(off);
    uint64_t before = 0, bstart = off;
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            before = pv->second;
            bstart = pv->first;
        }
    }
    for (uint64_t kk = 0; kk < units; ++kk) {
        const uint64_t lo = kk * unit, hi = (units - 1 - kk) * unit;
        if (lo > before || hi > after || (off - lo) % align != 0) continue;
        if (lo) {
            free_.erase(bstart);
            if (before > lo) free_[bstart] = before - lo;
        }
        if (hi) {
            free_.erase(off + unit);
            if (after > hi) free_[off + unit + hi] = after - hi;
        }
        used_.erase(u);
        used_[off - lo] = units * unit;
        *k = kk;
        return base_ + (off - lo);
    }
    return nullptr;
}

void Arena::shrink(void *p, uint64_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    const uint64_t off = (uint64_t)((char *)p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    bytes = round256(bytes);
    const uint64_t cur = u->second;
    if (bytes >= cur) return;
    u->second = bytes;
    insert_free(off + bytes, cur - bytes);
}

void Arena::insert_free(uint64_t start, uint64_t len) {
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && nx->first == start + len) {
        len += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(start);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == start) {
            start = pv->first;
            len += pv->second;
            free_.erase(pv);
        }
    }
    free_[start] = len;
}

void Arena::free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    const uint64_t off = (uint64_t)((char *)p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    const uint64_t len = u->second;
    used_.erase(u);
    insert_free(off, len);
}

uint64_t Arena::free_bytes() const {
    std::lock_guard<std::mutex> g(mu_);
    uint64_t t = 0;
    for (auto &f : free_) t += f.second;
    return t;
}

uint64_t Arena::largest_free() const {
    std::lock_guard<std::mutex> g(mu_);
    uint64_t t = 0;
    for (auto &f : free_) t = std::max(t, f.second);
    return t;
}

uint64_t Arena::used_bytes() const {
    std::lock_guard<std::mutex> g(mu_);
    uint64_t t = 0;
    for (auto &u : used_) t += u.second;
    return t;
}

bool Arena::contains(const void *p) const { return (const char *)p >= base_ && (const char *)p < base_ + size_; }

}  // namespace svh
