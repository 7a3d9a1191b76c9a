// First-fit device-memory arena (host bookkeeping only) used by the
// serving engine: one allocation carved into 256-byte-aligned blocks.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace tmi {

// First-fit arena over one device allocation, 256-byte granules.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    std::map<size_t, size_t> live_;  // offset -> bytes

    void init(char *b, size_t n)
    {
        base = b;
        size = n;
        free_.clear();
        live_.clear();
        free_[0] = n;
        used = 0;
    }
    void *alloc(size_t n)
    {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            size_t off = it->first, rem = it->second - n;
            free_.erase(it);
            if (rem) free_[off + n] = rem;
            live_[off] = n;
            used += n;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p)
    {
        if (!p) return;
        size_t off = (char *)p - base;
        auto it = live_.find(off);
        if (it == live_.end()) return;
        size_t n = it->second;
        live_.erase(it);
        used -= n;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + n == nx->first) {
            n += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t largest_free() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};


}  // namespace tmi
