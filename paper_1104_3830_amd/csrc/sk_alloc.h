// First-fit range allocator with coalescing, used by the serving scheduler to
// place requests in the device arena and W copies in the pinned staging ring.
// Offsets only: it never touches the memory it manages. Not thread-safe.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace sk {

struct RangeAlloc {
    static constexpr size_t kGranule = 256;
    std::map<size_t, size_t> free_;  // offset -> length of each free range

    static size_t round(size_t x) { return (x + kGranule - 1) / kGranule * kGranule; }
    void init(size_t base, size_t cap) {
        free_.clear();
        if (cap > base) free_[base] = cap - base;
    }
    bool alloc(size_t len, size_t &off) {
        len = round(len);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                off = it->first;
                const size_t rest = it->second - len;
                free_.erase(it);
                if (rest) free_[off + len] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t len) {
        len = round(len);
        auto it = free_.emplace(off, len).first;
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
        for (const auto &kv : free_) s += kv.second;
        return s;
    }
};

}  // namespace sk
