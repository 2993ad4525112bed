// Host side of the batched solver: argument checks, the workgroup plan for the
// persistent MFMA kernel, workspaces, and per-system outcomes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "batch.h"
#include "ctx.h"

namespace jac {

#define HIP_TRY(expr)                                                               \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess) {                                                     \
            set_error("%s failed: %s", #expr, hipGetErrorString(_e));               \
            return _e == hipErrorOutOfMemory ? JACOBI_ERR_OUT_OF_MEMORY             \
                                             : JACOBI_ERR_DEVICE;                   \
        }                                                                           \
    } while (0)

static double bits_to_double(uint64_t b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// Per-system outcomes from the device states after a launch.
static void decode_states(const BState* hst, int32_t count, float ms, float kernel_ms,
                          int32_t kernel, jacobi_info* infos) {
    for (int i = 0; i < count; ++i) {
        jacobi_info& inf = infos[i];
        const BState& T = hst[i];
        inf.device_ms = ms;
        inf.sweep_kernel_ms = kernel_ms;  // the persistent kernel alone
        inf.sweep_kernel_launches = kernel_ms >= 0.f ? 1 : 0;
        inf.kernel = kernel;
        inf.rel_residual = -1.0;
        inf.bad_index = -1;
        if (T.bad_diag != INT64_MAX) {
            inf.bad_index = T.bad_diag / 2;
            inf.status = (T.bad_diag & 1) ? JACOBI_ERR_NONFINITE_INPUT : JACOBI_ERR_ZERO_DIAGONAL;
            inf.iterations = 0;
            inf.final_delta = -1.0;
            continue;
        }
        if (T.bad_rhs != INT64_MAX) {
            inf.bad_index = T.bad_rhs;
            inf.status = JACOBI_ERR_NONFINITE_INPUT;
            inf.iterations = 0;
            inf.final_delta = -1.0;
            continue;
        }
        if (T.error) {
            inf.status = JACOBI_ERR_INTERNAL;
            continue;
        }
        inf.iterations = T.iterations;
        inf.final_delta = T.iterations > 0 ? bits_to_double(T.final_delta) : -1.0;
        if (T.status == STOP_CONVERGED)
            inf.status = JACOBI_OK;
        else if (T.status == STOP_DIVERGED)
            inf.status = JACOBI_DIVERGED;
        else
            inf.status = JACOBI_NOT_CONVERGED;
    }
}

// Run the persistent MFMA kernel on `count` FP32/BF16 systems (k <= 32).
// infos[i] receives each system's outcome.  sched 0: the planned schedule
// (k_batched: split systems meet at per-system barriers, small ones run whole
// from a queue); sched 1: the lockstep schedule (k_rounds: one sweep of every
// system per round, rows dealt out as work items, one grid barrier per round).
// Both give bitwise the same X, counts and maximum-norm distances.
static jacobi_status run_batched_shape(jacobi_ctx* c, int32_t count, const BatchItem* items,
                                       int32_t a_dtype, const jacobi_options& o, int32_t test,
                                       double rel, hipStream_t s, jacobi_info* infos,
                                       const BatchTune& tune) {
    const int variant = tune.shape;
    int sched = tune.sched;
    int kmax = 1;
    int64_t nmax = 1;
    double rows_iter = 0.0;  // bounds the dataflow queue (items x max_iter)
    for (int i = 0; i < count; ++i) {
        kmax = std::max<int>(kmax, (int)items[i].k);
        nmax = std::max(nmax, items[i].n);
        rows_iter += (double)items[i].n * (double)std::max(0, (int)items[i].max_iter);
    }
    // The dataflow queue holds every item a launch may publish: the items of
    // each system times its max_iter, at most 32 Mi entries (256 MiB); a
    // batch that could need more (a huge sweep cap) runs the lockstep
    // schedule.  Every item has at least 16 rows, so rows / 16 bounds the
    // item count before the plan is made.
    if (sched == 2 && (rows_iter / 16.0 > (double)(1ull << 25) || (count == 1 && tune.csplit > 1)))
        sched = 1;
    const int kt = kmax <= 16 ? 16 : 32;
    const bool split = sched == 1 && count == 1 && tune.csplit > 1;
    const int capacity = sched == 2   ? flow_max_grid(a_dtype, kt, variant, c->num_cus)
                         : sched == 1 ? rounds_max_grid(a_dtype, kt, variant, c->num_cus, split)
                                      : batched_max_grid(a_dtype, kt, variant, c->num_cus);
    if (capacity < 1) {
        set_error("batched kernel unavailable for this dtype");
        return JACOBI_ERR_INVALID_ARG;
    }
    std::vector<int64_t> ns(count);
    for (int i = 0; i < count; ++i) ns[i] = items[i].n;
    const int tpp = batched_tiles_per_pass(a_dtype, kt, variant, sched >= 1 && !split);
    Plan plan;
    ItemPlan ip;
    int grid = 0;
    const size_t ea = a_dtype == JACOBI_F64 ? 8 : (a_dtype == JACOBI_F32 ? 4 : 2);
    const size_t ex = a_dtype == JACOBI_F64 ? 8 : 4;  // iterate element
    // Column split (one system, lockstep): chunks of cw columns, a multiple of
    // the workgroup's block span, rows in ranges of 64 (whole passes in both
    // kernel shapes); items range-major, chunk index in `rank`.
    int32_t csplit = 1;
    int64_t cw = 0;
    if (sched == 1 && count == 1 && tune.csplit > 1) {
        const int64_t span = batched_block_cols(a_dtype);
        const int64_t n0 = items[0].n;
        cw = ((n0 + tune.csplit - 1) / tune.csplit + span - 1) / span * span;
        csplit = (int32_t)((n0 + cw - 1) / cw);
    }
    if (csplit > 1) {
        const int64_t n0 = items[0].n;
        ip.ngroups = 1;
        ip.it0.assign(1, 0);
        for (int64_t r0 = 0; r0 < n0; r0 += 64)
            for (int32_t ch = 0; ch < csplit; ++ch)
                ip.items.push_back(BJob{0, ch, (int32_t)r0, (int32_t)std::min<int64_t>(n0, r0 + 64)});
        ip.it1.assign(1, (int32_t)ip.items.size());
        ip.g_off = {0, (int32_t)ip.items.size()};
        ip.grid = std::min<int>(capacity, (int)ip.items.size());
        grid = ip.grid;
    } else if (sched >= 1) {
        ip = make_items(ns, capacity, tpp, (int)ea,
                        sched == 2 ? 1 : std::min(kMaxGroups, std::max(1, tune.groups)),
                        tune.per_wg);
        grid = ip.grid;
    } else {
        int max_split = 1 << 30;
        if (const char* env = getenv("JACOBI_BATCHED_MAXSPLIT")) max_split = atoi(env);
        plan = make_plan(ns, capacity, tpp, batched_unroll(a_dtype),
                         batched_block_cols(a_dtype), max_split);
        grid = plan.grid;
    }
    if (grid > capacity) {
        // the grid barriers need every workgroup resident at once
        set_error("batched plan of %d workgroups exceeds the resident grid %d", grid, capacity);
        return JACOBI_ERR_INTERNAL;
    }

    // workspace: per system buf0, buf1, bT (kt x xld, transposed) and diag (n)
    std::vector<size_t> off(count);
    size_t ws = 0;
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    auto xld_of = [](int64_t n) { return (n + 63) / 64 * 64; };  // a multiple of every block width
    for (int i = 0; i < count; ++i) {
        off[i] = ws;
        ws += 3 * align(ex * xld_of(items[i].n) * kt) + align(ex * items[i].n);
    }
    const size_t part_off = ws;  // split: csplit chunks of partial sums (kt x xld each)
    if (csplit > 1) ws += align(ex * (size_t)csplit * kt * xld_of(items[0].n));
    // device metadata: [sys | st | schedule tables (uploaded) | partial sums]
    //   sched 0 tables: jobs | job_off | queue head (16 bytes) + queue
    //   sched 1 tables: items | group offsets | BCtl
    //   sched 2 tables: items | group offsets | BCtl
    const size_t sys_b = align(sizeof(BSys) * count), st_b = align(sizeof(BState) * count);
    size_t job_b = 0, off_b = 0, q_b = 0, parts_b = 0;
    if (sched >= 1) {
        job_b = align(sizeof(BJob) * std::max<size_t>(1, ip.items.size()));
        // group offsets, then the row-range counters of a split system
        off_b = align(sizeof(int32_t) * ip.g_off.size() +
                      sizeof(uint32_t) * std::max<size_t>(1, ip.items.size()));
        q_b = align(sizeof(BCtl));
        parts_b = align(sizeof(double) * 2 * std::max<size_t>(1, ip.items.size()));
    } else {
        job_b = align(sizeof(BJob) * std::max<size_t>(1, plan.jobs.size()));
        off_b = align(sizeof(int32_t) * plan.job_off.size());
        q_b = align(sizeof(int32_t) * std::max<size_t>(1, plan.queue.size()) + 16);
        parts_b = align(sizeof(double) * 2 * (size_t)count * plan.max_nwg);
    }
    HIP_TRY(c->bws.ensure(ws));
    HIP_TRY(c->bmeta.ensure(sys_b + st_b + job_b + off_b + q_b + parts_b));
    char* meta = (char*)c->bmeta.p;
    BSys* d_sys = (BSys*)meta;
    BState* d_st = (BState*)(meta + sys_b);
    BJob* d_jobs = (BJob*)(meta + sys_b + st_b);
    int32_t* d_off = (int32_t*)(meta + sys_b + st_b + job_b);
    char* d_q = meta + sys_b + st_b + job_b + off_b;  // queue head + queue, or BCtl
    double* d_parts = (double*)(meta + sys_b + st_b + job_b + off_b + q_b);

    std::vector<BSys> hs(count);
    std::vector<BState> hst(count);
    int32_t active0 = 0, max_rounds = 0;
    for (int i = 0; i < count; ++i) {
        const BatchItem& it = items[i];
        char* base = (char*)c->bws.p + off[i];
        BSys& S = hs[i];
        std::memset(&S, 0, sizeof(S));
        S.A = it.A;
        S.lda = it.lda;
        S.B = it.B;
        S.ldb = it.ldb;
        S.X = it.X;
        S.ldx = it.ldx;
        S.X0 = it.X0;
        const size_t xb = align(ex * xld_of(it.n) * kt);
        S.buf0 = base;
        S.buf1 = base + xb;
        S.bT = base + 2 * xb;
        S.xld = xld_of(it.n);
        S.diag = base + 3 * xb;
        S.n = it.n;
        S.k = (int32_t)it.k;
        S.csplit = 1;
        S.first_free = it.first_free;
        if (sched >= 1) {
            S.nwg = 1;
            S.it0 = ip.it0[i];
            S.it1 = ip.it1[i];
            if (csplit > 1) {
                S.csplit = csplit;
                S.cw = cw;
                S.part = (char*)c->bws.p + part_off;
            }
        } else {
            S.nwg = plan.nwg[i];
        }
        S.max_iter = it.max_iter;
        S.test = test;
        S.tol = o.tol;
        S.rel = rel;
        S.norm = o.norm;
        BState& T = hst[i];
        std::memset(&T, 0, sizeof(T));
        T.bad_diag = INT64_MAX;
        T.bad_rhs = INT64_MAX;
        // no sweep (max_iter = 0): X = X0, copied in the first round
        const bool sweeps = it.max_iter > 0 && it.n > 0;
        T.done = sweeps ? 0 : 1;
        if (sweeps) {
            ++active0;
            max_rounds = std::max(max_rounds, it.max_iter);
        }
    }
    // Descriptors, initial states and the schedule tables go up through the
    // pinned stage in one copy kernel; the states come back the same way.
    const size_t up_b = sys_b + st_b + job_b + off_b + q_b;
    HIP_TRY(c->stage.ensure(up_b + st_b + q_b));
    char* h = (char*)c->stage.h;
    std::memcpy(h, hs.data(), sizeof(BSys) * count);
    std::memcpy(h + sys_b, hst.data(), sizeof(BState) * count);
    char* ht = h + sys_b + st_b;
    // Dataflow schedule: queue positions [0, nitems) are the items of every
    // system's first work (sweep 1, or the copy-out of X0 when max_iter = 0);
    // the ring holds every item a launch can publish later: the items of
    // sweeps 2 .. max_iter and of the copy-out, max_iter works per system.
    uint64_t ring_cap = 0;
    if (sched == 2) {
        for (int i = 0; i < count; ++i) {
            BState& T = hst[i];
            T.work = items[i].max_iter > 0 ? 2 : 1;
            ring_cap += (uint64_t)(ip.it1[i] - ip.it0[i]) *
                        (uint64_t)std::max(0, (int)items[i].max_iter);
        }
        ring_cap = std::max<uint64_t>(ring_cap, 1);
        std::memcpy(h + sys_b, hst.data(), sizeof(BState) * count);
        const size_t ring_b = sizeof(uint64_t) * ring_cap;
        if (c->fring.bytes < ring_b) {
            HIP_TRY(c->fring.ensure(ring_b));
            HIP_TRY(hipMemsetAsync(c->fring.p, 0, c->fring.bytes, s));  // no stale tags
            c->flow_gen = 0;
        }
        if (++c->flow_gen == 0) {  // tags wrapped: clear them
            HIP_TRY(hipMemsetAsync(c->fring.p, 0, c->fring.bytes, s));
            c->flow_gen = 1;
        }
    }
    if (sched >= 1) {
        std::memcpy(ht, ip.items.data(), sizeof(BJob) * ip.items.size());
        std::memset(ht + job_b, 0, off_b);
        std::memcpy(ht + job_b, ip.g_off.data(), sizeof(int32_t) * ip.g_off.size());
        BCtl ctl;
        std::memset(&ctl, 0, sizeof(ctl));
        // dataflow: every system with items is active until its copy-out
        int32_t with_items = 0;
        for (int i = 0; i < count; ++i) with_items += ip.it1[i] > ip.it0[i] ? 1 : 0;
        ctl.active = (uint32_t)(sched == 2 ? with_items : active0);
        ctl.ftail = (uint32_t)ip.items.size();
        std::memcpy(ht + job_b + off_b, &ctl, sizeof(ctl));
    } else {
        if (!plan.jobs.empty()) std::memcpy(ht, plan.jobs.data(), sizeof(BJob) * plan.jobs.size());
        std::memcpy(ht + job_b, plan.job_off.data(), sizeof(int32_t) * plan.job_off.size());
        std::memset(ht + job_b + off_b, 0, 16);  // queue head
        if (!plan.queue.empty())
            std::memcpy(ht + job_b + off_b + 16, plan.queue.data(),
                        sizeof(int32_t) * plan.queue.size());
    }
    HIP_TRY(launch_copy16(c->stage.d, meta, up_b, s));
    HIP_TRY(hipEventRecord(c->bev_begin, s));
    HIP_TRY(launch_batched_setup(a_dtype, kt, d_sys, d_st, count, nmax, s));
    HIP_TRY(hipEventRecord(c->bev_kernel, s));
    BatchArgs ba{};
    ba.sys = d_sys;
    ba.st = d_st;
    ba.count = count;
    int rate_khz = 100000;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device) !=
            hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    ba.spin_limit = (int64_t)rate_khz * 1000 * 20;  // 20 s
    if (sched >= 1) {
        ba.items = d_jobs;
        ba.item_parts = d_parts;
        ba.ctl = (BCtl*)d_q;
        ba.group_off = d_off;
        ba.rcnt = (uint32_t*)((char*)d_off + sizeof(int32_t) * ip.g_off.size());
        ba.ngroups = ip.ngroups;
        ba.nitems = (int32_t)ip.items.size();
        ba.active0 = active0;
        ba.max_rounds = max_rounds;
        if (sched == 2) {
            ba.ring = (uint64_t*)c->fring.p;
            ba.ring_cap = (uint32_t)ring_cap;
            ba.gen = c->flow_gen;
            if (grid > 0) HIP_TRY(launch_flow(a_dtype, kt, variant, ba, grid, s));
        } else if (grid > 0) {
            HIP_TRY(launch_rounds(a_dtype, kt, variant, ba, grid, s, csplit > 1));
        }
    } else {
        ba.jobs = d_jobs;
        ba.job_off = d_off;
        ba.parts = d_parts;
        ba.queue_head = (uint32_t*)d_q;
        ba.queue = (const int32_t*)(d_q + 16);
        ba.queue_len = (int32_t)plan.queue.size();
        ba.max_nwg = plan.max_nwg;
        if (grid > 0) HIP_TRY(launch_batched(a_dtype, kt, variant, ba, grid, s));
    }
    HIP_TRY(hipEventRecord(c->bev_end, s));
    HIP_TRY(launch_copy16(d_st, (char*)c->stage.d + up_b, st_b, s));
    if (sched >= 1)
        HIP_TRY(launch_copy16(d_q, (char*)c->stage.d + up_b + st_b, align(sizeof(BCtl)), s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(hst.data(), h + up_b, sizeof(BState) * count);
    if (sched >= 1) {
        BCtl ctl;
        std::memcpy(&ctl, h + up_b + st_b, sizeof(ctl));
        if (ctl.abort)  // a wait timed out: no outcome is trustworthy
            for (int i = 0; i < count; ++i) hst[i].error = 1;
    }
    float ms = 0.f, kms = -1.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->bev_begin, c->bev_end));
    if (grid > 0) HIP_TRY(hipEventElapsedTime(&kms, c->bev_kernel, c->bev_end));
    decode_states(hst.data(), count, ms, kms,
                  (sched == 1 ? 1 : 0) | (variant == 1 ? 2 : 0) | (sched == 2 ? 64 : 0) |
                      (sched == 1 ? (std::min(tune.groups, kMaxGroups) - 1) << 2 : 0) |
                      (sched >= 1 ? tune.per_wg << 8 : 0) | (csplit << 16),
                  infos);
    return JACOBI_OK;
}

// ---------------------------------------------------------------------------
// Tuning.  Every variant of a batched launch -- schedule (planned, lockstep
// or dataflow), kernel shape (wide or deep), XCD grouping and items per
// workgroup of the lockstep schedule -- sums every element in the same order, so all of them
// give bitwise the same X, counts and maximum-norm distances (tested); only
// the time differs.  The first batch of a class (schedule choice, element
// type, output width, and the power-of-two classes of system count, largest
// n and bytes of A) that is worth it is therefore solved several times, once
// per candidate, each run being the solve itself, and the fastest candidate
// is kept: in the context for its life, and in a cache file (one per GPU
// architecture, HIP runtime and library build) that later processes read.
// The search is staged: schedule x shape first, then for the lockstep
// schedule the XCD grouping, and for the lockstep and dataflow schedules the
// items per workgroup, one at a time.
// Environment overrides: JACOBI_BATCHED_SCHED (planned | lockstep | dataflow),
// JACOBI_BATCHED_SHAPE (wide | deep), JACOBI_BATCHED_GROUPS (1..8),
// JACOBI_BATCHED_ITEMS (items per workgroup), JACOBI_TUNE (auto | off |
// always), JACOBI_TUNE_CACHE (file path, or "off").

namespace {

// Build stamp of this library: cached choices of another build are ignored.
const char* const kBuildStamp = __DATE__ " " __TIME__;

std::mutex g_tune_file_mu;

std::string tune_cache_path(int device) {
    const char* env = getenv("JACOBI_TUNE_CACHE");
    if (env && !strcmp(env, "off")) return "";
    if (env && *env) return env;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
    int rt = 0;
    hipRuntimeGetVersion(&rt);
    std::string arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ':' || ch == '/' || ch == ' ') ch = '_';
    const char* home = getenv("HOME");
    const char* xdg = getenv("XDG_CACHE_HOME");
    std::string dir = xdg && *xdg ? std::string(xdg) : (home ? std::string(home) + "/.cache" : "");
    if (dir.empty()) return "";
    return dir + "/libjacobi-tune-" + arch + "-hip" + std::to_string(rt) + ".txt";
}

// Entries of the cache file written by this build:
// "stamp|key shape sched groups per_wg csplit".
void tune_cache_load(jacobi_ctx* c) {
    if (c->tune_loaded) return;
    c->tune_loaded = true;
    c->tune_path = tune_cache_path(c->device);
    if (c->tune_path.empty()) return;
    std::lock_guard<std::mutex> g(g_tune_file_mu);
    FILE* f = fopen(c->tune_path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        if (strcmp(line, kBuildStamp) != 0) continue;
        unsigned long long key = 0;
        BatchTune t;
        if (sscanf(bar + 1, "%llu %d %d %d %d %d", &key, &t.shape, &t.sched, &t.groups,
                   &t.per_wg, &t.csplit) == 6)
            c->batched_tune[(uint64_t)key] = t;
    }
    fclose(f);
}

void tune_cache_store(jacobi_ctx* c, uint64_t key, const BatchTune& t) {
    if (c->tune_path.empty()) return;
    std::lock_guard<std::mutex> g(g_tune_file_mu);
    const size_t slash = c->tune_path.rfind('/');
    if (slash != std::string::npos) mkdir(c->tune_path.substr(0, slash).c_str(), 0755);
    FILE* f = fopen(c->tune_path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s|%llu %d %d %d %d %d\n", kBuildStamp, (unsigned long long)key, t.shape,
            t.sched, t.groups, t.per_wg, t.csplit);
    fclose(f);
}

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

}  // namespace

jacobi_status run_batched(jacobi_ctx* c, int32_t count, const BatchItem* items, int32_t a_dtype,
                          const jacobi_options& o, int32_t test, double rel, hipStream_t s,
                          jacobi_info* infos, bool allow_split) {
    int kmax = 1;
    int64_t nmax = 1;
    double bytes = 0.0;
    bool alias = false;
    for (int i = 0; i < count; ++i) {
        kmax = std::max<int>(kmax, (int)items[i].k);
        nmax = std::max(nmax, items[i].n);
        bytes += (double)items[i].n * (double)items[i].n *
                 (a_dtype == JACOBI_F64 ? 8.0 : (a_dtype == JACOBI_F32 ? 4.0 : 2.0));
        if (items[i].X0 && items[i].X0 == items[i].X) alias = true;
    }
    // The rule of thumb when nothing is measured: lockstep; wide for many
    // systems, deep for few; no grouping; eight items per workgroup.
    BatchTune rule;
    rule.sched = 1;
    rule.shape = count * 4 >= c->num_cus ? 0 : 1;
    rule.groups = 1;
    rule.per_wg = 8;
    // Overrides fix a parameter and keep it out of the search.
    int f_sched = -1, f_shape = -1;
    if (const char* env = getenv("JACOBI_BATCHED_SCHED"))
        f_sched = !strcmp(env, "planned")    ? 0
                  : !strcmp(env, "lockstep") ? 1
                  : !strcmp(env, "dataflow") ? 2
                                             : -1;
    if (const char* env = getenv("JACOBI_BATCHED_SHAPE"))
        f_shape = !strcmp(env, "wide") ? 0 : (!strcmp(env, "deep") ? 1 : -1);
    const int f_groups = env_int("JACOBI_BATCHED_GROUPS", -1);
    const int f_items = env_int("JACOBI_BATCHED_ITEMS", -1);
    // Column split of a single system: chunks of at least 512 FP32 columns
    // (1024 BF16, 256 FP64, i.e. 2 KiB of a row), so that the partial sums
    // (2 x kt values per row and chunk) stay small next to A.
    const int64_t minw = a_dtype == JACOBI_F64 ? 256 : (a_dtype == JACOBI_F32 ? 512 : 1024);
    const bool splittable = allow_split && count == 1 && items[0].n >= 2 * minw;
    int max_split = 1;
    if (splittable)
        while (max_split < 8 && items[0].n / (2 * max_split) >= minw) max_split *= 2;
    const int f_split = splittable ? env_int("JACOBI_BATCHED_SPLIT", -1) : -1;
    if (splittable) {
        // rule: enough 64-row items times chunks to give every CU one
        int cs = 1;
        while (cs < max_split && (items[0].n + 63) / 64 * cs < c->num_cus) cs *= 2;
        rule.csplit = cs;
        rule.sched = 1;
    }
    auto apply = [&](BatchTune t) {
        if (f_sched >= 0) t.sched = f_sched;
        if (f_shape >= 0) t.shape = f_shape;
        if (f_groups >= 1) t.groups = f_groups;
        if (f_items >= 1) t.per_wg = f_items;
        if (f_split >= 1) t.csplit = std::min(f_split, max_split);
        if (!splittable || t.sched != 1) t.csplit = 1;
        return t;
    };
    const char* tenv = getenv("JACOBI_TUNE");
    const int mode = tenv && !strcmp(tenv, "off") ? 0 : (tenv && !strcmp(tenv, "always") ? 2 : 1);
    auto lg = [](double v) {
        int b = 0;
        while (v >= 2.0 && b < 62) {
            v /= 2.0;
            ++b;
        }
        return (uint64_t)b;
    };
    const uint64_t key = ((uint64_t)splittable << 62) | ((uint64_t)(f_sched + 1) << 60) |
                         ((uint64_t)a_dtype << 56) |
                         ((uint64_t)(kmax <= 16 ? 16 : 32) << 48) | (lg(count) << 32) |
                         (lg((double)nmax) << 16) | lg(bytes);
    // Worth a search: at least about 32 MiB of sweeps expected (bytes of A
    // times the sweeps the cap allows, up to 64).
    const double work = bytes * (double)std::min(o.max_iter, 64);
    const bool tune = mode == 2 || (mode == 1 && !alias && o.max_iter >= 2 &&
                                    work >= 32.0 * 1024 * 1024 && count > 0);
    if (mode != 0) tune_cache_load(c);
    auto hit = c->batched_tune.find(key);
    if (mode != 0 && hit != c->batched_tune.end() && mode != 2)
        return run_batched_shape(c, count, items, a_dtype, o, test, rel, s, infos,
                                 apply(hit->second));
    if (!tune)
        return run_batched_shape(c, count, items, a_dtype, o, test, rel, s, infos, apply(rule));
    // Warm-up: an empty launch of each kernel shape takes the one-time cost of
    // a kernel's first launch out of the comparison.
    {
        const int kt = kmax <= 16 ? 16 : 32;
        HIP_TRY(c->warm.ensure(256));
        int32_t zeros[16] = {0};
        HIP_TRY(c->stage.ensure(sizeof(zeros)));
        std::memcpy(c->stage.h, zeros, sizeof(zeros));
        HIP_TRY(launch_copy16(c->stage.d, c->warm.p, sizeof(zeros), s));
        for (int v = 0; v < 2; ++v) {
            BatchArgs wa{};
            wa.ctl = (BCtl*)c->warm.p;  // no item, no system: one empty round
            HIP_TRY(launch_rounds(a_dtype, kt, v, wa, 1, s));
            BatchArgs wb{};
            wb.job_off = (const int32_t*)c->warm.p;  // one workgroup, no fixed job
            wb.queue_head = (uint32_t*)((char*)c->warm.p + 16);
            wb.queue = (const int32_t*)c->warm.p;
            wb.queue_len = 0;  // and an empty queue
            HIP_TRY(launch_batched(a_dtype, kt, v, wb, 1, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }
    const bool trace = getenv("JACOBI_BATCHED_TRACE") != nullptr;
    BatchTune best{}, last{};
    double best_ms = 1e300;
    auto trial = [&](BatchTune t) -> jacobi_status {
        t = apply(t);
        jacobi_status st = run_batched_shape(c, count, items, a_dtype, o, test, rel, s, infos, t);
        if (st != JACOBI_OK) return st;
        last = t;
        const double ms = infos[0].device_ms;
        if (trace)
            std::fprintf(stderr, "jacobi tune: %s %s groups %d items %d split %d: %.3f ms\n",
                         t.sched == 2 ? "dataflow" : (t.sched ? "lockstep" : "planned"),
                         t.shape ? "deep" : "wide", t.groups, t.per_wg, t.csplit, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
        return JACOBI_OK;
    };
    if (splittable) {
        // One system: the column split (lockstep) against the shapes.  The
        // chunk count changes the summation order, so the chosen variant is
        // run last: its output is the call's result, as on every later call.
        for (int cs = 1; cs <= max_split; cs *= 2)
            for (int sh : {0, 1}) {
                if (f_shape >= 0 && sh != f_shape) continue;
                if (f_split >= 1 && cs != std::min(f_split, max_split)) continue;
                BatchTune t = rule;
                t.shape = sh;
                t.csplit = cs;
                jacobi_status st = trial(t);
                if (st != JACOBI_OK) return st;
            }
        if (!(best.shape == last.shape && best.csplit == last.csplit)) {
            jacobi_status st =
                run_batched_shape(c, count, items, a_dtype, o, test, rel, s, infos, best);
            if (st != JACOBI_OK) return st;
        }
        c->batched_tune[key] = best;
        tune_cache_store(c, key, best);
        return JACOBI_OK;
    }
    // stage 1: schedule x shape (the rule's candidate last, so that whatever
    // still favours a later run favours the default)
    std::vector<BatchTune> stage1;
    for (int sc : {0, 1, 2})
        for (int sh : {0, 1}) {
            BatchTune t = rule;
            t.sched = sc;
            t.shape = sh;
            if (!(sc == rule.sched && sh == rule.shape)) stage1.push_back(t);
        }
    stage1.push_back(rule);
    for (const BatchTune& t : stage1) {
        if ((f_sched >= 0 && t.sched != f_sched) || (f_shape >= 0 && t.shape != f_shape))
            continue;
        jacobi_status st = trial(t);
        if (st != JACOBI_OK) return st;
    }
    // stage 2: the lockstep schedule's grouping, and the item size of the
    // lockstep and dataflow schedules
    if (best.sched >= 1) {
        if (f_groups < 1 && best.sched == 1) {
            BatchTune t = best;
            t.groups = kMaxGroups;
            jacobi_status st = trial(t);
            if (st != JACOBI_OK) return st;
        }
        if (f_items < 1)
            for (int m : {4, 16}) {
                BatchTune t = best;
                t.per_wg = m;
                jacobi_status st = trial(t);
                if (st != JACOBI_OK) return st;
            }
    }
    c->batched_tune[key] = best;
    tune_cache_store(c, key, best);
    return JACOBI_OK;
}

}  // namespace jac

using namespace jac;

extern "C" jacobi_status jacobi_solve_batched(jacobi_ctx* ctx, int32_t count,
                                              const jacobi_system* systems, int32_t a_dtype,
                                              const jacobi_options* opt, hipStream_t stream,
                                              jacobi_info* infos) {
    try {
        if (count < 0 || (count > 0 && (!systems || !infos))) {
            set_error("invalid count or null array");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_options o;
        jacobi_options_default(&o);
        if (opt) o = *opt;
        for (int i = 0; i < count; ++i) {
            std::memset(&infos[i], 0, sizeof(jacobi_info));
            infos[i].status = JACOBI_ERR_INVALID_ARG;
            infos[i].bad_index = -1;
            infos[i].final_delta = -1.0;
            infos[i].rel_residual = -1.0;
        }
        if (std::isnan(o.tol) || o.tol < 0.0 || o.max_iter < 0 ||
            (o.norm != JACOBI_NORM_INF && o.norm != JACOBI_NORM_L2) ||
            o.mode != JACOBI_MODE_PLAIN || (a_dtype != JACOBI_F64 && a_dtype != JACOBI_F32 &&
                                            a_dtype != JACOBI_BF16)) {
            set_error("invalid batched options (plain mode, tol >= 0, max_iter >= 0)");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_status st = JACOBI_OK;
        jacobi_ctx* c = ctx ? ctx : default_ctx(&st);
        if (!c) return st;
        std::lock_guard<std::mutex> g(c->mu);
        if (hipSetDevice(c->device) != hipSuccess) return JACOBI_ERR_DEVICE;
        std::vector<BatchItem> items;
        std::vector<int> idx;
        for (int i = 0; i < count; ++i) {
            const jacobi_system& y = systems[i];
            const bool ok = y.n >= 1 && y.k >= 1 && y.lda >= y.n && y.ldb >= y.k &&
                            y.ldx >= y.k && y.A && y.B && y.X && y.n <= (int64_t)INT32_MAX &&
                            y.k <= 32;
            if (!ok) continue;
            BatchItem it{y.n, y.k, y.A, y.lda, y.B, y.ldb, y.X0, y.X, y.ldx, o.max_iter};
            items.push_back(it);
            idx.push_back(i);
        }
        if (items.empty()) return JACOBI_OK;
        std::vector<jacobi_info> out(items.size());
        st = run_batched(c, (int32_t)items.size(), items.data(), a_dtype, o, TEST_ABS, 0.0,
                         stream, out.data());
        if (st != JACOBI_OK) return st;
        for (size_t q = 0; q < items.size(); ++q) infos[idx[q]] = out[q];
        return JACOBI_OK;
    } catch (...) {
        set_error("internal exception");
        return JACOBI_ERR_INTERNAL;
    }
}
