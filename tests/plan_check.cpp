// Test driver for the batched workgroup planner (paper_1403_5805_amd/csrc/plan.cpp).
// Reads "capacity tpp unroll bw count n_0 ... n_{count-1}" from stdin and
// prints the plan: "grid G", one "nwg i v" line per system, one
// "wg g sys rank r0 r1" line per fixed job and one "q sys" line per queue
// entry, in queue order.  With a leading "items"
// ("items capacity tpp elem_bytes groups count n_0 ...") it prints the
// lockstep work items instead: "grid G", one "goff q offset" line per group
// boundary, one "range s it0 it1" line per system and one "item j sys r0 r1"
// line per item.  Built with g++;
// no GPU involved.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_1403_5805_amd/csrc/plan.h"

static int items_mode() {
    int capacity, tpp, elem, groups, count;
    if (std::scanf("%d %d %d %d %d", &capacity, &tpp, &elem, &groups, &count) != 5) return 2;
    std::vector<int64_t> n(count);
    for (int i = 0; i < count; ++i) {
        long long v;
        if (std::scanf("%lld", &v) != 1) return 2;
        n[i] = v;
    }
    const jac::ItemPlan p = jac::make_items(n, capacity, tpp, elem, groups);
    std::printf("grid %d\n", p.grid);
    for (size_t g = 0; g < p.g_off.size(); ++g) std::printf("goff %zu %d\n", g, p.g_off[g]);
    for (int i = 0; i < count; ++i) std::printf("range %d %d %d\n", i, p.it0[i], p.it1[i]);
    for (size_t j = 0; j < p.items.size(); ++j)
        std::printf("item %zu %d %d %d\n", j, p.items[j].sys, p.items[j].r0, p.items[j].r1);
    return 0;
}

int main() {
    char head[16] = {0};
    if (std::scanf("%15s", head) != 1) return 2;
    if (!std::strcmp(head, "items")) return items_mode();
    int capacity = std::atoi(head), tpp, unroll, bw, count;
    if (std::scanf("%d %d %d %d", &tpp, &unroll, &bw, &count) != 4) return 2;
    std::vector<int64_t> n(count);
    for (int i = 0; i < count; ++i) {
        long long v;
        if (std::scanf("%lld", &v) != 1) return 2;
        n[i] = v;
    }
    const jac::Plan p = jac::make_plan(n, capacity, tpp, unroll, bw);
    std::printf("grid %d\n", p.grid);
    for (int i = 0; i < count; ++i) std::printf("nwg %d %d\n", i, p.nwg[i]);
    for (int g = 0; g < p.grid; ++g)
        for (int j = p.job_off[g]; j < p.job_off[g + 1]; ++j)
            std::printf("wg %d %d %d %d %d\n", g, p.jobs[j].sys, p.jobs[j].rank, p.jobs[j].r0,
                        p.jobs[j].r1);
    for (int32_t q : p.queue) std::printf("q %d\n", q);
    return 0;
}
