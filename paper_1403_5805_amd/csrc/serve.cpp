// Serving engine: continuous batching of FP64 solves by iterative refinement.
//
// Two worker threads per server:
//   copy thread     admits queued requests while the HBM budget and the active
//                   slots allow, places their device state in the server's
//                   arena (slabs reserved once, reused as requests retire) and
//                   copies A and B host -> device on its own stream, so
//                   transfers overlap the sweeps of the requests already on
//                   the device;
//   compute thread  turns arrived requests into active ones (A_lo = round(A)
//                   on the device, x = 0) and steps the whole active set: one
//                   batched FP64 residual launch for every request (x += d
//                   fused in, stop test per request, one read-back of every
//                   outcome), retirement of finished requests (result copied
//                   back, memory freed at once), then one persistent batched
//                   launch that runs every remaining request's inner Jacobi
//                   solve A_lo d = r (per system relative stop).
// Each request's arithmetic depends only on its own data, so its result is
// the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "batch.h"
#include "ctx.h"

namespace jac {

namespace {

using Clock = std::chrono::steady_clock;

double now_s() {
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

int kpad_of(int64_t k) {
    int kt = 1;
    while (kt < k) kt <<= 1;
    return kt;
}

struct Req {
    uint64_t id = 0;
    jacobi_request r{};
    int32_t status = JACOBI_PENDING;
    jacobi_info info{};
    double t_submit = 0, t_ready = 0, t_done = 0;
    double bnorm = 0;
    int kp = 1;
    int64_t ld_lo = 0;
    size_t bytes = 0;
    // device state (one allocation)
    char* base = nullptr;
    double* dA = nullptr;
    void* dAlo = nullptr;
    double* dB = nullptr;
    double* xcur = nullptr;
    double* xnext = nullptr;
    double* r64 = nullptr;
    float* rlo = nullptr;
    float* d = nullptr;
    double* xT = nullptr;  // residual workspace (transposed x + d)
    int outer = 0;
    int inner = 0;
    double rel = -1.0;
    bool has_d = false;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Arena slabs: 4 GiB (two of the largest requests of the size mix) unless a
// request needs more; reserved with hipMalloc on the server's device.
constexpr size_t kSlabBytes = (size_t)4 << 30;

void* arena_slab_alloc(size_t bytes, void*) {
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void arena_slab_free(void* p, void*) { hipFree(p); }

size_t footprint(int64_t n, int64_t k, int32_t lo, int64_t* ld_lo_out) {
    const int kp = kpad_of(k);
    const int64_t ld_lo = (n + 7) / 8 * 8;
    if (ld_lo_out) *ld_lo_out = ld_lo;
    const size_t elo = lo == JACOBI_F32 ? 4 : 2;
    size_t b = align256(8 * (size_t)n * n) + align256(elo * (size_t)n * ld_lo) +
               align256(8 * (size_t)n * k) + 3 * align256(8 * (size_t)n * kp) +
               2 * align256(4 * (size_t)n * kp) + align256(resid_xT_bytes(n, k));
    return b;
}

}  // namespace

}  // namespace jac

using namespace jac;

struct jacobi_server {
    jacobi_serve_config cfg{};
    jacobi_ctx* ctx = nullptr;
    hipStream_t s_copy = nullptr, s_comp = nullptr;
    std::mutex mu;
    std::condition_variable cv_copy, cv_comp, cv_done;
    std::deque<Req*> queued;
    std::vector<Req*> arrived;
    uint64_t n_active = 0;   // requests owned by the compute thread
    std::unordered_map<uint64_t, Req*> all;
    uint64_t next_id = 1;
    uint64_t hbm_in_use = 0, hbm_peak = 0;
    int admitted_slots = 0;
    bool stopping = false;
    std::thread t_copy, t_comp;
    // stats
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, steps = 0;
    double t_first = -1.0, t_last = 0.0;
    std::vector<double> lat_e2e, lat_dev;
    bool copy_failed = false;
    jac::Arena* arena = nullptr;  // device memory of the requests (guarded by mu)
    uint64_t releases = 0;        // retirements so far (wakes an arena wait)
};

namespace {

void finish_locked(jacobi_server* s, Req* q, int32_t status) {
    q->status = status;
    q->info.status = status;
    q->t_done = now_s();
    if (status == JACOBI_OK || status == JACOBI_NOT_CONVERGED || status == JACOBI_DIVERGED) {
        s->completed += 1;
        s->lat_e2e.push_back((q->t_done - q->t_submit) * 1e3);
        s->lat_dev.push_back((q->t_done - q->t_ready) * 1e3);
        q->info.device_ms = (q->t_done - q->t_ready) * 1e3;
        s->t_last = q->t_done;
    } else if (status != JACOBI_CANCELLED) {
        s->failed += 1;
    }
    s->cv_done.notify_all();
}

void copy_loop(jacobi_server* s) {
    hipSetDevice(s->cfg.device);
    const bool trace = getenv("JACOBI_SERVE_TRACE") != nullptr;  // per-copy timing to stderr
    for (;;) {
        Req* q = nullptr;
        void* p = nullptr;
        double t_copy0 = 0.0;
        {
            std::unique_lock<std::mutex> g(s->mu);
            for (;;) {
                s->cv_copy.wait(g, [&] {
                    if (s->stopping) return true;
                    if (s->queued.empty()) return false;
                    Req* h = s->queued.front();
                    return s->admitted_slots < s->cfg.max_active &&
                           s->hbm_in_use + h->bytes <= s->cfg.hbm_budget_bytes;
                });
                if (s->stopping) return;
                t_copy0 = now_s();
                p = s->arena->alloc(s->queued.front()->bytes);
                if (p) break;
                if (s->arena->in_use() == 0) break;  // cannot be placed at all
                // the free space is fragmented: wait for a retirement
                const uint64_t gen = s->releases;
                s->cv_copy.wait(g, [&] { return s->stopping || s->releases != gen; });
            }
            q = s->queued.front();
            s->queued.pop_front();
            if (!p) {
                set_error("request of %zu bytes does not fit the device arena", q->bytes);
                finish_locked(s, q, JACOBI_ERR_OUT_OF_MEMORY);
                continue;
            }
            s->admitted_slots += 1;
            s->hbm_in_use += q->bytes;
            s->hbm_peak = std::max(s->hbm_peak, s->hbm_in_use);
        }
        hipError_t e = hipSuccess;
        const int64_t n = q->r.n, k = q->r.k;
        if (e == hipSuccess) {
            char* b = (char*)p;
            const size_t elo = q->r.sweep_dtype == JACOBI_F32 ? 4 : 2;
            q->base = b;
            q->dA = (double*)b;
            b += align256(8 * (size_t)n * n);
            q->dAlo = b;
            b += align256(elo * (size_t)n * q->ld_lo);
            q->dB = (double*)b;
            b += align256(8 * (size_t)n * k);
            q->xcur = (double*)b;
            b += align256(8 * (size_t)n * q->kp);
            q->xnext = (double*)b;
            b += align256(8 * (size_t)n * q->kp);
            q->r64 = (double*)b;
            b += align256(8 * (size_t)n * q->kp);
            q->rlo = (float*)b;
            b += align256(4 * (size_t)n * q->kp);
            q->d = (float*)b;
            b += align256(4 * (size_t)n * q->kp);
            q->xT = (double*)b;
            // contiguous rows go as one linear copy (the fast DMA path)
            if (q->r.lda == n)
                e = hipMemcpyAsync(q->dA, q->r.A, 8 * (size_t)n * n, hipMemcpyHostToDevice,
                                   s->s_copy);
            else
                e = hipMemcpy2DAsync(q->dA, 8 * n, q->r.A, 8 * q->r.lda, 8 * n, n,
                                     hipMemcpyHostToDevice, s->s_copy);
            if (e == hipSuccess) {
                if (q->r.ldb == k)
                    e = hipMemcpyAsync(q->dB, q->r.B, 8 * (size_t)n * k, hipMemcpyHostToDevice,
                                       s->s_copy);
                else
                    e = hipMemcpy2DAsync(q->dB, 8 * k, q->r.B, 8 * q->r.ldb, 8 * k, n,
                                         hipMemcpyHostToDevice, s->s_copy);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s->s_copy);
        }
        if (trace) {
            const double dt = now_s() - t_copy0;
            const double gb = 8.0 * (double)n * (double)(n + k) / 1e9;
            fprintf(stderr, "[serve] copy n=%lld k=%lld %.2f ms %.2f GB/s\n", (long long)n,
                    (long long)k, dt * 1e3, gb / dt);
        }
        if (e != hipSuccess) hipStreamSynchronize(s->s_copy);  // nothing in flight before the free
        std::lock_guard<std::mutex> g(s->mu);
        if (e != hipSuccess) {
            s->arena->free(q->base, q->bytes);
            q->base = nullptr;
            s->hbm_in_use -= q->bytes;
            s->admitted_slots -= 1;
            s->releases += 1;
            finish_locked(s, q, JACOBI_ERR_DEVICE);
            continue;
        }
        q->t_ready = now_s();
        s->arrived.push_back(q);
        s->cv_comp.notify_all();
    }
}

// Result to the caller's host X: pack x (leading dim kp) into n x k rows on
// the device (the r64 buffer is free by now), then one linear copy when the
// host rows are contiguous.  A pitched copy of narrow rows would issue one
// transfer per row.
void copy_out(jacobi_server* s, Req* q) {
    const int64_t n = q->r.n, k = q->r.k;
    launch_copy_rows(8, q->xcur, q->kp, q->r64, k, n, (int)k, s->s_comp);
    if (q->r.ldx == k)
        hipMemcpyAsync(q->r.X, q->r64, 8 * (size_t)n * k, hipMemcpyDeviceToHost, s->s_comp);
    else
        hipMemcpy2DAsync(q->r.X, 8 * q->r.ldx, q->r64, 8 * k, 8 * k, n, hipMemcpyDeviceToHost,
                         s->s_comp);
}

// Release a request's device memory.  The compute stream has finished every
// use of it (the step ends with a stream synchronisation).
void release_locked(jacobi_server* s, Req* q) {
    s->arena->free(q->base, q->bytes);
    q->base = nullptr;
    s->hbm_in_use -= q->bytes;
    s->admitted_slots -= 1;
    s->releases += 1;
    s->cv_copy.notify_all();
}

void compute_loop(jacobi_server* s) {
    hipSetDevice(s->cfg.device);
    std::vector<Req*> act;  // active requests, owned by this thread
    const bool trace = getenv("JACOBI_SERVE_TRACE") != nullptr;  // per-step timing to stderr
    for (;;) {
        std::vector<Req*> fresh;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_comp.wait(g, [&] { return s->stopping || !s->arrived.empty() || !act.empty(); });
            if (s->stopping) return;
            fresh.swap(s->arrived);
            s->n_active += fresh.size();
        }
        // Arrived requests: A_lo = round(A), x = 0.
        for (Req* q : fresh) {
            launch_convert(q->dA, q->r.n, q->r.n, q->r.sweep_dtype, q->dAlo, q->ld_lo, s->s_comp);
            launch_zero_rows(8, q->xcur, q->kp, q->r.n, q->kp, s->s_comp);
            launch_zero_rows(8, q->xnext, q->kp, q->r.n, q->kp, s->s_comp);
            act.push_back(q);
        }
        if (act.empty()) continue;
        const double t_step0 = now_s();
        // 1. One batched FP64 residual pass over every active request.
        std::vector<ResidItem> ritems(act.size());
        std::vector<RState> rst(act.size());
        for (size_t i = 0; i < act.size(); ++i) {
            Req* q = act[i];
            ResidItem& it = ritems[i];
            it.n = q->r.n;
            it.k = q->r.k;
            it.ldx = q->kp;
            it.A = q->dA;
            it.lda = q->r.n;
            it.B = q->dB;
            it.ldb = q->r.k;
            it.x = q->xcur;
            it.d = q->has_d ? q->d : nullptr;
            it.xnew = q->xnext;
            it.r64 = q->r64;
            it.rlo = q->rlo;
            it.xT = q->xT;
            it.bnorm = q->bnorm;
            it.rel = q->r.rel_tol;
        }
        const jacobi_status rs_st =
            run_resid(s->ctx, (int32_t)act.size(), ritems.data(), s->s_comp, rst.data());
        const double t_resid = now_s();
        // 2. Decide: retire finished requests, keep the rest.
        std::vector<Req*> keep, done;
        std::vector<int32_t> done_status;
        for (size_t i = 0; i < act.size(); ++i) {
            Req* q = act[i];
            int32_t st = JACOBI_PENDING;
            if (rs_st != JACOBI_OK) {
                // the residual launch failed: fail the whole active set
                done.push_back(q);
                done_status.push_back(rs_st);
                continue;
            }
            std::swap(q->xcur, q->xnext);
            q->outer += 1;
            double rel;
            std::memcpy(&rel, &rst[i].rel_bits, sizeof(rel));
            q->rel = rel;
            if (rst[i].stop == STOP_CONVERGED)
                st = JACOBI_OK;
            else if (rst[i].stop == STOP_DIVERGED)
                st = JACOBI_DIVERGED;
            else if (q->outer > (q->r.max_outer > 0 ? q->r.max_outer : s->cfg.max_outer))
                st = JACOBI_NOT_CONVERGED;
            if (st == JACOBI_PENDING) {
                keep.push_back(q);
            } else {
                copy_out(s, q);
                done.push_back(q);
                done_status.push_back(st);
            }
        }
        // 3. One batched launch for every remaining inner solve, per sweep dtype.
        // Each starts from d = 0, whose first sweep is d = r / a_ii: the setup
        // kernel writes it (no pass over A_lo) and the sweeps go on from there
        // (that sweep cannot meet the relative stop test when rel < 1).
        const bool first_free = s->cfg.inner_rel_tol < 1.0 && s->cfg.inner_max >= 2;
        const int32_t cap = first_free ? s->cfg.inner_max - 1 : s->cfg.inner_max;
        int64_t inner_sweeps = 0, inner_sys = 0;
        double inner_bytes = 0.0;
        for (int32_t lo : {JACOBI_F32, JACOBI_BF16}) {
            std::vector<BatchItem> items;
            std::vector<Req*> owners;
            for (Req* q : keep) {
                if (q->r.sweep_dtype != lo) continue;
                BatchItem it{q->r.n, q->r.k, q->dAlo, q->ld_lo, q->rlo, q->kp, nullptr,
                             q->d, q->kp, cap};
                it.first_free = first_free ? 1 : 0;
                items.push_back(it);
                owners.push_back(q);
            }
            if (items.empty()) continue;
            std::vector<jacobi_info> infos(items.size());
            jacobi_options o;
            jacobi_options_default(&o);
            o.tol = 0.0;
            o.max_iter = cap;
            jacobi_status st = run_batched(s->ctx, (int32_t)items.size(), items.data(), lo, o,
                                           TEST_REL, s->cfg.inner_rel_tol, s->s_comp, infos.data());
            for (size_t i = 0; i < owners.size(); ++i) {
                Req* q = owners[i];
                q->has_d = true;
                if (st != JACOBI_OK || infos[i].status < 0) {
                    // a failed inner solve fails the request
                    auto it = std::find(keep.begin(), keep.end(), q);
                    if (it != keep.end()) keep.erase(it);
                    done.push_back(q);
                    done_status.push_back(st != JACOBI_OK ? st : infos[i].status);
                    continue;
                }
                q->inner += infos[i].iterations + (first_free ? 1 : 0);
                inner_sweeps += infos[i].iterations + (first_free ? 1 : 0);
                inner_sys += 1;
                inner_bytes += (double)infos[i].iterations * (double)q->r.n * (double)q->r.n *
                               (lo == JACOBI_F32 ? 4.0 : 2.0);
                if (infos[i].status == JACOBI_DIVERGED) {
                    auto it = std::find(keep.begin(), keep.end(), q);
                    if (it != keep.end()) keep.erase(it);
                    copy_out(s, q);
                    done.push_back(q);
                    done_status.push_back(JACOBI_DIVERGED);
                }
            }
        }
        hipStreamSynchronize(s->s_comp);
        if (trace) {
            double rbytes = 0.0;
            for (Req* q : act) rbytes += 8.0 * (double)q->r.n * (double)q->r.n;
            const double t_end = now_s();
            fprintf(stderr,
                    "[serve] step %llu active=%zu retired=%zu resid %.2f ms (%.2f GB) inner %.2f "
                    "ms (%lld systems, %lld sweeps, %.2f GB)\n",
                    (unsigned long long)s->steps, act.size(), done.size(),
                    (t_resid - t_step0) * 1e3, rbytes / 1e9, (t_end - t_resid) * 1e3,
                    (long long)inner_sys, (long long)inner_sweeps, inner_bytes / 1e9);
        }
        std::lock_guard<std::mutex> g(s->mu);
        s->steps += 1;
        for (size_t i = 0; i < done.size(); ++i) {
            Req* q = done[i];
            q->info.iterations = q->inner;
            q->info.outer_iterations = q->outer;
            q->info.rel_residual = q->rel;
            q->info.bad_index = -1;
            release_locked(s, q);
            finish_locked(s, q, done_status[i]);
        }
        s->n_active -= done.size();
        act.swap(keep);
    }
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t r = (size_t)std::ceil(p * v.size());  // nearest rank
    if (r < 1) r = 1;
    if (r > v.size()) r = v.size();
    return v[r - 1];
}

}  // namespace

extern "C" {

void jacobi_serve_config_default(jacobi_serve_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->device = 0;
    c->max_active = 64;
    c->hbm_budget_bytes = 0;
    c->inner_max = 64;
    c->max_outer = 50;
    c->inner_rel_tol = 1e-3;
}

jacobi_status jacobi_serve_create(const jacobi_serve_config* cfg, jacobi_server** out) {
    try {
        if (!out) return JACOBI_ERR_INVALID_ARG;
        *out = nullptr;
        jacobi_serve_config c;
        jacobi_serve_config_default(&c);
        if (cfg) c = *cfg;
        if (c.max_active < 1 || c.inner_max < 1 || c.max_outer < 0 || !(c.inner_rel_tol >= 0.0)) {
            set_error("invalid serve config");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_ctx* ctx = nullptr;
        jacobi_status st = jacobi_ctx_create(c.device, &ctx);
        if (st != JACOBI_OK) return st;
        hipSetDevice(c.device);
        if (c.hbm_budget_bytes == 0) {
            size_t fr = 0, tot = 0;
            hipMemGetInfo(&fr, &tot);
            c.hbm_budget_bytes = (uint64_t)(0.8 * (double)fr);
        }
        jacobi_server* s = new jacobi_server();
        s->cfg = c;
        s->ctx = ctx;
        s->arena = new Arena(arena_slab_alloc, arena_slab_free, nullptr, kSlabBytes,
                             (size_t)c.hbm_budget_bytes);
        if (hipStreamCreateWithFlags(&s->s_copy, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking) != hipSuccess) {
            jacobi_ctx_destroy(ctx);
            delete s->arena;
            delete s;
            return JACOBI_ERR_DEVICE;
        }
        s->t_copy = std::thread(copy_loop, s);
        s->t_comp = std::thread(compute_loop, s);
        *out = s;
        return JACOBI_OK;
    } catch (...) {
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_serve_submit(jacobi_server* s, const jacobi_request* r, uint64_t* ticket) {
    try {
        if (!s || !r || !ticket) return JACOBI_ERR_INVALID_ARG;
        *ticket = 0;
        Req* q = new Req();
        q->r = *r;
        q->t_submit = now_s();
        q->info.bad_index = -1;
        q->info.final_delta = -1.0;
        q->info.rel_residual = -1.0;
        const int64_t n = r->n, k = r->k;
        int32_t st = JACOBI_PENDING;
        if (n < 1 || k < 1 || k > 32 || r->lda < n || r->ldb < k || r->ldx < k || !r->A ||
            !r->B || !r->X || (r->sweep_dtype != JACOBI_F32 && r->sweep_dtype != JACOBI_BF16) ||
            !(r->rel_tol >= 0.0) || r->max_outer < 0 || n > (int64_t)INT32_MAX) {
            st = JACOBI_ERR_INVALID_ARG;
            set_error("invalid request");
        }
        if (st == JACOBI_PENDING) {
            // Input check on the host copy (sec. 2: the method fails when
            // alpha_ii = 0): first bad diagonal, then non-finite B.
            for (int64_t i = 0; i < n && st == JACOBI_PENDING; ++i) {
                const double d = r->A[i * r->lda + i];
                if (d == 0.0) {
                    st = JACOBI_ERR_ZERO_DIAGONAL;
                    q->info.bad_index = i;
                } else if (!std::isfinite(d)) {
                    st = JACOBI_ERR_NONFINITE_INPUT;
                    q->info.bad_index = i;
                }
            }
            double bb = 0.0;
            for (int64_t i = 0; i < n && st == JACOBI_PENDING; ++i)
                for (int64_t c = 0; c < k; ++c) {
                    const double v = r->B[i * r->ldb + c];
                    if (!std::isfinite(v)) {
                        st = JACOBI_ERR_NONFINITE_INPUT;
                        q->info.bad_index = i;
                        break;
                    }
                    bb += v * v;
                }
            q->bnorm = std::sqrt(bb);
        }
        q->kp = kpad_of(k);
        if (st == JACOBI_PENDING) q->bytes = footprint(n, k, r->sweep_dtype, &q->ld_lo);
        std::lock_guard<std::mutex> g(s->mu);
        q->id = s->next_id++;
        s->all[q->id] = q;
        *ticket = q->id;
        s->submitted += 1;
        if (s->t_first < 0) s->t_first = q->t_submit;
        if (st == JACOBI_PENDING && q->bytes > s->cfg.hbm_budget_bytes) {
            st = JACOBI_ERR_REJECTED;
            set_error("request footprint %zu B exceeds the HBM budget", q->bytes);
        }
        if (st != JACOBI_PENDING) {
            q->status = st;
            q->info.status = st;
            if (st == JACOBI_ERR_REJECTED) s->rejected += 1;
            else s->failed += 1;
            s->cv_done.notify_all();
            return (jacobi_status)st;
        }
        s->queued.push_back(q);
        s->cv_copy.notify_all();
        return JACOBI_OK;
    } catch (...) {
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_serve_poll(jacobi_server* s, uint64_t ticket, jacobi_info* info) {
    if (!s) return JACOBI_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return JACOBI_ERR_INVALID_ARG;
    if (info) *info = it->second->info;
    if (info) info->status = it->second->status;
    return (jacobi_status)it->second->status;
}

jacobi_status jacobi_serve_wait(jacobi_server* s, uint64_t ticket, int64_t timeout_us,
                                jacobi_info* info) {
    if (!s) return JACOBI_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return JACOBI_ERR_INVALID_ARG;
    Req* q = it->second;
    auto ready = [&] { return q->status != JACOBI_PENDING; };
    if (timeout_us < 0)
        s->cv_done.wait(g, ready);
    else
        s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), ready);
    if (info) {
        *info = q->info;
        info->status = q->status;
    }
    return (jacobi_status)q->status;
}

jacobi_status jacobi_serve_stats_get(jacobi_server* s, jacobi_serve_stats* out) {
    if (!s || !out) return JACOBI_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->failed = s->failed;
    out->active = s->n_active + s->arrived.size();
    out->queued = s->queued.size();
    out->hbm_in_use = s->hbm_in_use;
    out->hbm_peak = s->hbm_peak;
    out->steps = s->steps;
    const double el = (s->t_first >= 0 && s->t_last > s->t_first) ? s->t_last - s->t_first : 0.0;
    out->elapsed_s = el;
    out->solves_per_s = el > 0 ? (double)s->completed / el : 0.0;
    out->p50_ms = percentile(s->lat_e2e, 0.50);
    out->p99_ms = percentile(s->lat_e2e, 0.99);
    out->p50_device_ms = percentile(s->lat_dev, 0.50);
    out->p99_device_ms = percentile(s->lat_dev, 0.99);
    return JACOBI_OK;
}

jacobi_status jacobi_serve_destroy(jacobi_server* s) {
    if (!s) return JACOBI_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        s->cv_copy.notify_all();
        s->cv_comp.notify_all();
    }
    if (s->t_copy.joinable()) s->t_copy.join();
    if (s->t_comp.joinable()) s->t_comp.join();
    hipSetDevice(s->cfg.device);
    hipStreamSynchronize(s->s_copy);
    hipStreamSynchronize(s->s_comp);
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (auto& kv : s->all) {
            Req* q = kv.second;
            if (q->base) {
                s->arena->free(q->base, q->bytes);
                q->base = nullptr;
            }
            if (q->status == JACOBI_PENDING) finish_locked(s, q, JACOBI_CANCELLED);
        }
    }
    delete s->arena;  // both streams are idle: the slabs go back to the device
    s->arena = nullptr;
    for (auto& kv : s->all) delete kv.second;
    s->all.clear();
    hipStreamDestroy(s->s_copy);
    hipStreamDestroy(s->s_comp);
    jacobi_ctx_destroy(s->ctx);
    delete s;
    return JACOBI_OK;
}

}  // extern "C"
