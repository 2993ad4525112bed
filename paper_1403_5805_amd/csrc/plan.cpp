// Workgroup plan of the persistent batched kernel (host code, no HIP).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <utility>

namespace jac {

// Modelled time of one sweep of rows [0, rows) of an n-column system on one
// workgroup: ceil(tiles / tpp) passes, each taking ceil(blocks / U) load
// round trips (a round trip covers bw columns of every tile of the pass) plus
// its epilogue.  Units are arbitrary; only ratios matter.
static double job_cost(int64_t n, int64_t rows, int tpp, int unroll, int bw) {
    const double passes = std::ceil(std::ceil((double)rows / 16.0) / tpp);
    const double blocks = std::ceil((double)n / bw);
    return passes * (1.0 + std::ceil(blocks / unroll)) + 1.0;
}

// Split big systems over several workgroups (by the modelled sweep time
// above) and queue the small ones, largest first, for whichever workgroup is
// free.  A workgroup that shares a system with others
// owns nothing else, so barrier waits only involve workgroups that are certain
// to arrive.
Plan make_plan(const std::vector<int64_t>& n, int capacity, int tpp, int unroll, int bw,
               int max_split) {
    Plan p;
    const int count = (int)n.size();
    p.nwg.assign(count, 1);
    if (count == 0) {
        p.job_off.push_back(0);
        return p;
    }
    std::vector<double> cost(count);
    double total = 0.0;
    for (int i = 0; i < count; ++i) {
        cost[i] = job_cost(n[i], n[i], tpp, unroll, bw);
        total += cost[i];
    }
    const double target = total / std::max(1, capacity);
    std::vector<int> big, small;
    int g_big = 0;
    for (int i = 0; i < count; ++i) {
        const int64_t tiles = (n[i] + 15) / 16;
        int want = (int)std::lround(cost[i] / target);
        // no share smaller than one full pass of tiles
        want = (int)std::min<int64_t>(want, (tiles + tpp - 1) / tpp);
        want = std::min(want, std::max(1, max_split));
        if (want >= 2) {
            p.nwg[i] = want;
            big.push_back(i);
            g_big += want;
        } else {
            small.push_back(i);
        }
    }
    // workgroups kept free for the systems that run whole (recomputed as
    // shrinking moves systems into that group)
    auto reserve = [&]() {
        return small.empty() ? 0 : std::max(1, std::min((int)small.size(), capacity / 8));
    };
    while (g_big > capacity - reserve() && !big.empty()) {
        // shrink the largest shares until the plan fits the resident grid
        int best = big[0];
        for (int i : big)
            if (p.nwg[i] > p.nwg[best]) best = i;
        p.nwg[best] -= 1;
        g_big -= 1;
        if (p.nwg[best] == 1) {
            big.erase(std::find(big.begin(), big.end(), best));
            small.push_back(best);
            g_big -= 1;
        }
    }
    std::vector<std::vector<BJob>> wg_jobs;
    for (int i : big) {
        const int64_t tiles = (n[i] + 15) / 16;
        for (int r = 0; r < p.nwg[i]; ++r) {
            const int64_t t0 = tiles * r / p.nwg[i], t1 = tiles * (r + 1) / p.nwg[i];
            BJob j;
            j.sys = i;
            j.rank = r;
            j.r0 = (int32_t)(16 * t0);
            j.r1 = (int32_t)std::min<int64_t>(n[i], 16 * t1);
            wg_jobs.push_back({j});
        }
    }
    // Systems that run whole are not bound to workgroups: they wait in a
    // queue, largest first, and every workgroup takes the next one when it
    // is free (its own split share done, or none).  Workgroups set aside for
    // the queue carry no fixed job.
    const int pool = std::max(small.empty() ? 0 : 1,
                              std::min((int)small.size(), capacity - (int)wg_jobs.size()));
    std::stable_sort(small.begin(), small.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int i : small) p.queue.push_back(i);
    wg_jobs.resize(wg_jobs.size() + pool);
    p.job_off.push_back(0);
    for (auto& v : wg_jobs) {
        for (auto& j : v) p.jobs.push_back(j);
        p.job_off.push_back((int32_t)p.jobs.size());
    }
    p.grid = (int)p.job_off.size() - 1;
    p.max_nwg = 1;
    for (int v : p.nwg) p.max_nwg = std::max(p.max_nwg, v);
    return p;
}

// About eight items per workgroup and round (per_wg, tuned per batch class)
// keeps the round's tail short (the last items are the small systems'); the
// floor keeps the per-item ticket and pipeline start small next to the item's
// loads.
// Grouping by XCD: all items of a system run on one XCD (while its own
// workgroups have work), so the system's iterate, which every one of its
// items reads in full, stays in that XCD's L2 instead of being fetched again
// by every XCD.
ItemPlan make_items(const std::vector<int64_t>& n, int capacity, int tpp, int elem_bytes,
                    int ngroups, int per_wg) {
    ItemPlan p;
    const int count = (int)n.size();
    p.ngroups = std::max(1, ngroups);
    p.it0.assign(count, 0);
    p.it1.assign(count, 0);
    double total = 0.0;
    for (int64_t v : n) total += (double)v * (double)v * elem_bytes;
    const double target =
        std::min(2.0 * 1024 * 1024,
                 std::max(128.0 * 1024,
                          total / ((double)std::max(1, per_wg) * std::max(1, capacity))));
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    // largest systems first, each to the lightest group so far
    std::vector<std::vector<int>> members(p.ngroups);
    std::vector<double> load(p.ngroups, 0.0);
    for (int s : order) {
        int g = 0;
        for (int q = 1; q < p.ngroups; ++q)
            if (load[q] < load[g]) g = q;
        members[g].push_back(s);
        load[g] += (double)n[s] * (double)n[s];
    }
    const int64_t unit = 16 * (int64_t)tpp;
    p.g_off.push_back(0);
    for (int g = 0; g < p.ngroups; ++g) {
        for (int s : members[g]) {
            p.it0[s] = (int32_t)p.items.size();
            if (n[s] > 0) {
                int64_t rows = (int64_t)std::ceil(target / ((double)n[s] * elem_bytes));
                rows = std::max<int64_t>(unit, (rows + unit - 1) / unit * unit);
                for (int64_t r0 = 0; r0 < n[s]; r0 += rows)
                    p.items.push_back(
                        BJob{s, 0, (int32_t)r0, (int32_t)std::min(n[s], r0 + rows)});
            }
            p.it1[s] = (int32_t)p.items.size();
        }
        p.g_off.push_back((int32_t)p.items.size());
    }
    p.grid = std::min<int64_t>(std::max(1, capacity), (int64_t)p.items.size());
    return p;
}

}  // namespace jac
