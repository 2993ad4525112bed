// Device-memory arena of the serving engine (host bookkeeping only).
#include "arena.h"

#include <algorithm>
#include <iterator>

namespace jac {

Arena::Arena(SlabAlloc alloc, SlabFree free, void* user, size_t slab_min, size_t limit)
    : alloc_(alloc), free_(free), user_(user), slab_min_(round(slab_min)), limit_(limit) {}

Arena::~Arena() {
    for (Slab& s : slabs_) free_(s.base, user_);
}

bool Arena::add_slab(size_t bytes) {
    if (reserved_ + bytes > limit_) return false;
    size_t size = std::max(bytes, slab_min_);
    if (reserved_ + size > limit_) size = limit_ - reserved_;  // what is left of the limit
    void* p = alloc_(size, user_);
    if (!p) return false;
    Slab s;
    s.base = static_cast<char*>(p);
    s.size = size;
    s.free[0] = size;
    slabs_.push_back(std::move(s));
    reserved_ += size;
    return true;
}

void Arena::release_empty() {
    for (size_t i = 0; i < slabs_.size();) {
        Slab& s = slabs_[i];
        if (s.free.size() == 1 && s.free.begin()->first == 0 && s.free.begin()->second == s.size) {
            free_(s.base, user_);
            reserved_ -= s.size;
            slabs_.erase(slabs_.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

void* Arena::alloc(size_t bytes) {
    bytes = round(std::max<size_t>(bytes, 1));
    for (int attempt = 0; attempt < 3; ++attempt) {
        // best fit: the smallest free block that holds the request
        Slab* best_slab = nullptr;
        std::map<size_t, size_t>::iterator best;
        for (Slab& s : slabs_)
            for (auto it = s.free.begin(); it != s.free.end(); ++it)
                if (it->second >= bytes && (!best_slab || it->second < best->second)) {
                    best_slab = &s;
                    best = it;
                }
        if (best_slab) {
            const size_t off = best->first, len = best->second;
            best_slab->free.erase(best);
            if (len > bytes) best_slab->free[off + bytes] = len - bytes;
            in_use_ += bytes;
            return best_slab->base + off;
        }
        if (attempt == 0) {
            if (!add_slab(bytes)) continue;
        } else if (attempt == 1) {
            // empty slabs may be too small: give them back and reserve anew
            release_empty();
            if (!add_slab(bytes)) return nullptr;
        }
    }
    return nullptr;
}

void Arena::free(void* p, size_t bytes) {
    if (!p) return;
    bytes = round(std::max<size_t>(bytes, 1));
    char* c = static_cast<char*>(p);
    for (Slab& s : slabs_) {
        if (c < s.base || c >= s.base + s.size) continue;
        size_t off = (size_t)(c - s.base), len = bytes;
        auto next = s.free.lower_bound(off);
        if (next != s.free.end() && off + len == next->first) {  // merge with the following block
            len += next->second;
            next = s.free.erase(next);
        }
        if (next != s.free.begin()) {  // merge with the preceding block
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                len += prev->second;
                s.free.erase(prev);
            }
        }
        s.free[off] = len;
        in_use_ -= bytes;
        return;
    }
}

size_t Arena::largest_free() const {
    size_t m = 0;
    for (const Slab& s : slabs_)
        for (const auto& kv : s.free) m = std::max(m, kv.second);
    return m;
}

}  // namespace jac
