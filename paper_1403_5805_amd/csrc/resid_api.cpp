// Host side of the batched FP64 residual pass: descriptors, job table, one
// launch per right-hand-side width, and the per-system outcomes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

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

static int32_t resid_kt(int64_t k) { return k <= 16 ? 16 : 32; }
static int64_t resid_xld(int64_t n) { return (n + 7) / 8 * 8; }

size_t resid_xT_bytes(int64_t n, int64_t k) {
    return sizeof(double) * (size_t)resid_kt(k) * (size_t)resid_xld(n);
}

jacobi_status run_resid(jacobi_ctx* c, int32_t count, const ResidItem* items, hipStream_t s,
                        RState* out) {
    if (count <= 0) return JACOBI_OK;
    if (count > 65535) {
        set_error("batched residual: at most 65535 systems per call");
        return JACOBI_ERR_INVALID_ARG;
    }
    for (int i = 0; i < count; ++i) {
        const ResidItem& it = items[i];
        if (it.n < 1 || it.k < 1 || it.k > 32 || it.ldx < it.k || it.lda < it.n ||
            it.ldb < it.k || !it.A || !it.B || !it.x || !it.xnew || !it.r64 || !it.rlo || !it.xT ||
            (uintptr_t)it.xT % 16 != 0) {
            set_error("batched residual: invalid system %d", i);
            return JACOBI_ERR_INVALID_ARG;
        }
    }
    // Systems grouped by output width (16 or 32 columns) and rows per job,
    // one launch per group.
    auto key = [&](int i) {
        const int32_t kt = resid_kt(items[i].k);
        return kt * 8 + resid_tiles(kt, items[i].n, c->num_cus);
    };
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<RSys> hs(count);
    std::vector<int32_t> job_sys;
    struct Group {
        int32_t kt, tiles, first, count, job0, jobs;
        int64_t max_xld;
    };
    std::vector<Group> groups;
    for (int o = 0; o < count; ++o) {
        const ResidItem& it = items[order[o]];
        const int32_t kt = resid_kt(it.k);
        const int32_t tiles = resid_tiles(kt, it.n, c->num_cus);
        if (groups.empty() || groups.back().kt != kt || groups.back().tiles != tiles)
            groups.push_back({kt, tiles, o, 0, (int32_t)job_sys.size(), 0, 0});
        Group& g = groups.back();
        const int rows = 16 * tiles;
        const int32_t nj = (int32_t)((it.n + rows - 1) / rows);
        RSys& S = hs[o];
        std::memset(&S, 0, sizeof(S));
        S.A = it.A;
        S.lda = it.lda;
        S.B = it.B;
        S.ldb = it.ldb;
        S.x = it.x;
        S.d = it.d;
        S.xnew = it.xnew;
        S.r64 = it.r64;
        S.rlo = it.rlo;
        S.xT = it.xT;
        S.ldx = it.ldx;
        S.xld = resid_xld(it.n);
        S.n = it.n;
        S.k = (int32_t)it.k;
        S.job0 = (int32_t)job_sys.size() - g.job0;  // group-local job numbering
        S.njobs = nj;
        S.aligned = (((uintptr_t)it.A % 16) == 0 && ((size_t)it.lda * 8) % 16 == 0) ? 1 : 0;
        S.bnorm = it.bnorm;
        S.rel = it.rel;
        for (int32_t j = 0; j < nj; ++j) job_sys.push_back(g.count);  // group-local index
        g.count += 1;
        g.jobs += nj;
        g.max_xld = std::max(g.max_xld, S.xld);
    }
    // Device layout [systems | job table | outcomes | job sums]; the first two
    // are uploaded through the pinned stage, the outcomes come back through it.
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t sys_b = align(sizeof(RSys) * count);
    const size_t job_b = align(sizeof(int32_t) * job_sys.size());
    const size_t st_b = align(sizeof(RState) * count);
    const size_t parts_b = align(sizeof(double) * job_sys.size());
    HIP_TRY(c->rmeta.ensure(sys_b + job_b + st_b + parts_b));
    HIP_TRY(c->stage.ensure(sys_b + job_b + st_b));
    char* meta = (char*)c->rmeta.p;
    RSys* d_sys = (RSys*)meta;
    int32_t* d_job = (int32_t*)(meta + sys_b);
    RState* d_st = (RState*)(meta + sys_b + job_b);
    double* d_parts = (double*)(meta + sys_b + job_b + st_b);
    char* h = (char*)c->stage.h;
    std::memcpy(h, hs.data(), sizeof(RSys) * count);
    std::memcpy(h + sys_b, job_sys.data(), sizeof(int32_t) * job_sys.size());
    HIP_TRY(launch_copy16(c->stage.d, meta, sys_b + job_b, s));
    for (const Group& g : groups) {
        HIP_TRY(launch_resid_prep(g.kt, d_sys + g.first, d_st + g.first, g.count, g.max_xld, s));
        RArgs a{};
        a.sys = d_sys + g.first;
        a.st = d_st + g.first;
        a.job_sys = d_job + g.job0;
        a.parts = d_parts + g.job0;
        HIP_TRY(launch_resid(g.kt, g.tiles, a, g.jobs, s));
    }
    HIP_TRY(launch_copy16(d_st, (char*)c->stage.d + sys_b + job_b, st_b, s));
    HIP_TRY(hipStreamSynchronize(s));
    const RState* hst = (const RState*)(h + sys_b + job_b);
    for (int o = 0; o < count; ++o) out[order[o]] = hst[o];
    return JACOBI_OK;
}

}  // namespace jac
