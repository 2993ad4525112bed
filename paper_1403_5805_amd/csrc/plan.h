// Workgroup plan of the persistent batched kernel.  Host code only, free of
// HIP so that its invariants can be checked by a plain C++ build.
#pragma once

#include <stdint.h>

#include <vector>

namespace jac {

// One unit of work for a workgroup: rows [r0, r1) of system sys.
struct BJob {
    int32_t sys;
    int32_t rank;   // index of this workgroup among the system's workgroups
    int32_t r0;
    int32_t r1;
};

// Workgroup plan: fixed jobs of workgroup g are jobs[job_off[g] ..
// job_off[g+1]); afterwards every workgroup takes whole systems from `queue`
// (an atomic head) until it is empty.
struct Plan {
    std::vector<int> nwg;        // workgroups per system
    std::vector<BJob> jobs;
    std::vector<int32_t> job_off;
    std::vector<int32_t> queue;  // systems run whole, largest first
    int grid = 0;
    int max_nwg = 1;
};

// Plan `n.size()` systems (sizes n[i]) onto at most `capacity` co-resident
// workgroups that sweep `tpp` 16-row tiles per pass and cover `bw` columns of
// them per load, `unroll` loads per round trip.  Guarantees: grid <= capacity;
// every system is either split over nwg[i] >= 2 workgroups, one fixed job of
// each rank 0..nwg[i]-1 covering its rows [0, n[i]) exactly once at multiples
// of 16 rows, each on a workgroup with no other fixed job, or listed once in
// the queue (nwg[i] = 1) in order of decreasing modelled cost.  No system is
// split over more than max_split workgroups.
Plan make_plan(const std::vector<int64_t>& n, int capacity, int tpp, int unroll, int bw,
               int max_split = 1 << 30);

// Work items of the lockstep schedule: the rows of every system cut into
// chunks (rows in order); items of system s are items[it0[s] .. it1[s]).
// Systems are shared out among `ngroups` groups (one per XCD: workgroup g
// runs on XCD g % ngroups), balanced by bytes of A; the items of group q are
// items[g_off[q] .. g_off[q + 1]), its systems by decreasing n.
struct ItemPlan {
    std::vector<BJob> items;  // rank = 0
    std::vector<int32_t> it0, it1;
    std::vector<int32_t> g_off;  // ngroups + 1 entries
    int ngroups = 1;
    int grid = 0;             // workgroups to launch: min(capacity, items)
};

// Guarantees: every system with n[s] >= 1 has at least one item; its items
// cover rows [0, n[s]) exactly once, in order, each a multiple of 16 * tpp
// rows long except the system's last; an item holds about
// clamp(total bytes / (capacity * per_wg), 128 KiB, 2 MiB) of A (elem_bytes
// per value) or the whole system when that is smaller.  Systems with n[s] = 0
// get an empty range.  Each system's items lie inside one group; a system
// goes to the group with the fewest bytes so far, largest systems first.
ItemPlan make_items(const std::vector<int64_t>& n, int capacity, int tpp, int elem_bytes,
                    int ngroups = 1, int per_wg = 8);

}  // namespace jac
