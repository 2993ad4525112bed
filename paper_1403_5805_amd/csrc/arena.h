// Device-memory arena of the serving engine (host bookkeeping, no HIP here).
//
// Requests are placed best-fit into slabs that are reserved on demand and
// kept until the arena is destroyed, so steady-state serving never calls the
// device allocator: a new request reuses the space of retired ones.  Blocks
// are 256-byte aligned; freeing coalesces with free neighbours.  The caller
// frees a block only once the device no longer uses it.
#pragma once

#include <stddef.h>

#include <map>
#include <vector>

namespace jac {

class Arena {
public:
    using SlabAlloc = void* (*)(size_t bytes, void* user);  // nullptr on failure
    using SlabFree = void (*)(void* p, void* user);

    // slab_min: smallest slab reserved at once; limit: cap on reserved bytes.
    Arena(SlabAlloc alloc, SlabFree free, void* user, size_t slab_min, size_t limit);
    ~Arena();
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;

    // A block of at least `bytes`, or nullptr when no free block fits and no
    // slab can be added within the limit (after releasing empty slabs).
    void* alloc(size_t bytes);
    // Return a block obtained from alloc with the same `bytes`.
    void free(void* p, size_t bytes);

    size_t reserved() const { return reserved_; }
    size_t in_use() const { return in_use_; }
    size_t slabs() const { return slabs_.size(); }
    // Largest free block (for tests and diagnostics).
    size_t largest_free() const;

    static size_t round(size_t bytes) { return (bytes + 255) / 256 * 256; }

private:
    struct Slab {
        char* base;
        size_t size;
        std::map<size_t, size_t> free;  // offset -> length, disjoint, not adjacent
    };
    bool add_slab(size_t bytes);
    void release_empty();

    SlabAlloc alloc_;
    SlabFree free_;
    void* user_;
    size_t slab_min_, limit_;
    size_t reserved_ = 0, in_use_ = 0;
    std::vector<Slab> slabs_;
};

}  // namespace jac
