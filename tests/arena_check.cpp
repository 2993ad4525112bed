// Test driver for the serving engine's device-memory arena
// (paper_1403_5805_amd/csrc/arena.cpp), run on the CPU with host memory
// standing in for device slabs.  Usage: arena_check SEED OPS LIMIT_MB SLAB_MB
// Prints "ok <stats>" or the first violated property, exit status 0 / 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../paper_1403_5805_amd/csrc/arena.h"

static std::map<char*, size_t> g_slabs;  // live fake slabs

static void* slab_alloc(size_t bytes, void*) {
    void* p = nullptr;
    if (posix_memalign(&p, 256, bytes) != 0) return nullptr;
    g_slabs[(char*)p] = bytes;
    return p;
}
static void slab_free(void* p, void*) {
    g_slabs.erase((char*)p);
    std::free(p);
}

static int fail(const char* what, long op) {
    std::printf("FAIL %s at op %ld\n", what, op);
    return 1;
}

int main(int argc, char** argv) {
    if (argc != 5) return 2;
    const unsigned seed = (unsigned)std::atoi(argv[1]);
    const long ops = std::atol(argv[2]);
    const size_t limit = (size_t)std::atol(argv[3]) << 20, slab = (size_t)std::atol(argv[4]) << 20;
    std::mt19937_64 rng(seed);
    std::vector<std::pair<char*, size_t>> live;
    long nulls = 0, allocs = 0;
    {
        jac::Arena a(slab_alloc, slab_free, nullptr, slab, limit);
        for (long op = 0; op < ops; ++op) {
            const bool do_alloc = live.empty() || (rng() % 100) < 55;
            if (do_alloc) {
                // sizes log-uniform from 1 KiB to a quarter of the limit
                const double lo = 10.0, hi = std::log2((double)limit / 4);
                const double e = lo + (hi - lo) * (double)(rng() % 1000000) / 1e6;
                const size_t bytes = (size_t)std::exp2(e) + rng() % 300;
                char* p = (char*)a.alloc(bytes);
                ++allocs;
                if (!p) {
                    ++nulls;
                    // only allowed when no free block holds the request
                    if (a.largest_free() >= jac::Arena::round(bytes))
                        return fail("refused although a free block fits", op);
                    continue;
                }
                if ((uintptr_t)p % 256 != 0) return fail("misaligned block", op);
                bool inside = false;
                for (auto& kv : g_slabs)
                    if (p >= kv.first && p + bytes <= kv.first + kv.second) inside = true;
                if (!inside) return fail("block outside every slab", op);
                for (auto& l : live)
                    if (p < l.first + jac::Arena::round(l.second) && l.first < p + jac::Arena::round(bytes))
                        return fail("overlapping blocks", op);
                live.push_back({p, bytes});
            } else {
                const size_t i = rng() % live.size();
                a.free(live[i].first, live[i].second);
                live[i] = live.back();
                live.pop_back();
            }
            size_t used = 0, res = 0;
            for (auto& l : live) used += jac::Arena::round(l.second);
            for (auto& kv : g_slabs) res += kv.second;
            if (used != a.in_use()) return fail("in_use mismatch", op);
            if (res != a.reserved()) return fail("reserved mismatch", op);
            if (a.reserved() > limit) return fail("limit exceeded", op);
        }
        for (auto& l : live) a.free(l.first, l.second);
        live.clear();
        if (a.in_use() != 0) return fail("in_use after freeing all", ops);
        size_t biggest = 0;
        for (auto& kv : g_slabs) biggest = std::max(biggest, kv.second);
        if (a.largest_free() != biggest) return fail("free blocks not coalesced", ops);
        // a freed block is reused without reserving more
        const size_t before = a.reserved();
        void* p = a.alloc(biggest / 2 + 1);
        if (!p || a.reserved() != before) return fail("no reuse of freed space", ops);
        a.free(p, biggest / 2 + 1);
    }
    if (!g_slabs.empty()) return fail("slabs leaked at destruction", ops);
    std::printf("ok allocs %ld refused %ld\n", allocs, nulls);
    return 0;
}
