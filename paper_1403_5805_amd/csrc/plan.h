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

// Workgroup plan: jobs of workgroup g are jobs[job_off[g] .. job_off[g+1]).
struct Plan {
    std::vector<int> nwg;        // workgroups per system
    std::vector<BJob> jobs;
    std::vector<int32_t> job_off;
    int grid = 0;
    int max_nwg = 1;
};

// Plan `n.size()` systems (sizes n[i]) onto at most `capacity` co-resident
// workgroups that sweep `tpp` 16-row tiles per pass and cover `bw` columns of
// them per load, `unroll` loads per round trip.  Guarantees: grid <= capacity; the jobs of system i cover its
// rows [0, n[i]) exactly once, split at multiples of 16 rows; a system split
// over nwg[i] >= 2 workgroups has one job of each rank 0..nwg[i]-1, and a
// workgroup holding such a job holds nothing else.
Plan make_plan(const std::vector<int64_t>& n, int capacity, int tpp, int unroll, int bw);

}  // namespace jac
