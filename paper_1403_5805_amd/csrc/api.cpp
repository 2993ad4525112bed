// Host runtime and C ABI of libjacobi: argument checks, device workspaces,
// the sweep loop with its device stop flag, and iterative refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/jacobi.h"
#include "batch.h"
#include "ctx.h"
#include "internal.h"

using namespace jac;

namespace jac {

thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

hipError_t DevBuf::ensure(size_t b) {
    if (b <= bytes) return hipSuccess;
    if (p) {
        hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    size_t want = std::max(b, (size_t)256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    bytes = want;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
}

hipError_t HostStage::ensure(size_t b) {
    if (b <= bytes) return hipSuccess;
    release();
    const size_t want = std::max<size_t>(b, 64 * 1024);
    hipError_t e = hipHostMalloc(&h, want, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) {
        h = nullptr;
        return e;
    }
    e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
        hipHostFree(h);
        h = d = nullptr;
        return e;
    }
    bytes = want;
    return hipSuccess;
}

void HostStage::release() {
    if (h) hipHostFree(h);
    h = d = nullptr;
    bytes = 0;
}

jacobi_status ctx_init(jacobi_ctx* c, int device) {
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return JACOBI_ERR_DEVICE;
    c->num_cus = prop.multiProcessorCount;
    if (hipSetDevice(device) != hipSuccess) return JACOBI_ERR_DEVICE;
    if (hipMalloc(&c->ctl, sizeof(Ctl)) != hipSuccess) return JACOBI_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&c->slots, 3 * sizeof(Slot)) != hipSuccess) return JACOBI_ERR_OUT_OF_MEMORY;
    if (hipMalloc(&c->parts, 3 * sizeof(double) * kMaxParts) != hipSuccess)
        return JACOBI_ERR_OUT_OF_MEMORY;
    if (hipHostMalloc(&c->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
        return JACOBI_ERR_OUT_OF_MEMORY;
    // the small-system kernel writes its outcome here directly when the
    // mirror is mapped into the device's address space
    if (hipHostGetDevicePointer((void**)&c->h_ctl_dev, c->h_ctl, 0) != hipSuccess) {
        (void)hipGetLastError();
        c->h_ctl_dev = nullptr;
    }
    if (hipEventCreate(&c->ev_begin) != hipSuccess) return JACOBI_ERR_DEVICE;
    if (hipEventCreate(&c->ev_end) != hipSuccess) return JACOBI_ERR_DEVICE;
    if (hipEventCreate(&c->bev_begin) != hipSuccess) return JACOBI_ERR_DEVICE;
    if (hipEventCreate(&c->bev_end) != hipSuccess) return JACOBI_ERR_DEVICE;
    if (hipEventCreate(&c->bev_kernel) != hipSuccess) return JACOBI_ERR_DEVICE;
    return JACOBI_OK;
}

void ctx_release(jacobi_ctx* c) {
    hipSetDevice(c->device);
    for (DevBuf* b : {&c->diag, &c->w0, &c->w1, &c->alo, &c->diag_lo, &c->xa, &c->xb, &c->r64,
                      &c->rlo, &c->d0, &c->d1, &c->scal, &c->bws, &c->bmeta, &c->rmeta,
                      &c->xT, &c->warm, &c->fring})
        b->release();
    c->stage.release();
    if (c->bev_begin) hipEventDestroy(c->bev_begin);
    if (c->bev_end) hipEventDestroy(c->bev_end);
    if (c->bev_kernel) hipEventDestroy(c->bev_kernel);
    if (c->ctl) hipFree(c->ctl);
    if (c->slots) hipFree(c->slots);
    if (c->parts) hipFree(c->parts);
    if (c->h_ctl) hipHostFree(c->h_ctl);
    if (c->ev_begin) hipEventDestroy(c->ev_begin);
    if (c->ev_end) hipEventDestroy(c->ev_end);
    for (auto& e : c->prof_ev) hipEventDestroy(e);
    c->prof_ev.clear();
}

std::mutex g_default_mu;
std::vector<jacobi_ctx*> g_default_ctx;

jacobi_ctx* default_ctx(jacobi_status* st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *st = JACOBI_ERR_DEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> g(g_default_mu);
    if ((int)g_default_ctx.size() <= dev) g_default_ctx.resize(dev + 1, nullptr);
    if (!g_default_ctx[dev]) {
        jacobi_ctx* c = new (std::nothrow) jacobi_ctx();
        if (!c) {
            *st = JACOBI_ERR_OUT_OF_MEMORY;
            return nullptr;
        }
        jacobi_status s = ctx_init(c, dev);
        if (s != JACOBI_OK) {
            ctx_release(c);
            delete c;
            *st = s;
            return nullptr;
        }
        g_default_ctx[dev] = c;
    }
    *st = JACOBI_OK;
    return g_default_ctx[dev];
}

int mfma_min_cols(int32_t) { return 3; }

int kpad_for(int64_t k) {
    if (k <= 32) {
        int kt = 1;
        while (kt < k) kt <<= 1;
        return kt;
    }
    return (int)((k + 31) / 32 * 32);
}

static size_t dtype_bytes(int32_t d) { return d == JACOBI_F64 ? 8 : (d == JACOBI_F32 ? 4 : 2); }

#define HIP_TRY(expr)                                                               \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess) {                                                     \
            set_error("%s failed: %s", #expr, hipGetErrorString(_e));               \
            return _e == hipErrorOutOfMemory ? JACOBI_ERR_OUT_OF_MEMORY             \
                                             : JACOBI_ERR_DEVICE;                   \
        }                                                                           \
    } while (0)

jacobi_status check_common(int64_t n, int64_t k, int32_t a_dtype, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* X, int64_t ldx,
                           const jacobi_options& o) {
    if (n < 1 || k < 1 || lda < n || ldb < k || ldx < k || !A || !B || !X) {
        set_error("invalid sizes or null pointer (n=%lld k=%lld lda=%lld ldb=%lld ldx=%lld)",
                  (long long)n, (long long)k, (long long)lda, (long long)ldb, (long long)ldx);
        return JACOBI_ERR_INVALID_ARG;
    }
    if (a_dtype < JACOBI_F64 || a_dtype > JACOBI_BF16) {
        set_error("unknown a_dtype %d", a_dtype);
        return JACOBI_ERR_INVALID_ARG;
    }
    if (std::isnan(o.tol) || o.tol < 0.0 || o.max_iter < 0 ||
        (o.norm != JACOBI_NORM_INF && o.norm != JACOBI_NORM_L2) ||
        (o.mode != JACOBI_MODE_PLAIN && o.mode != JACOBI_MODE_REFINE) || o.sync_every < 0) {
        set_error("invalid options (tol, max_iter, norm, mode or sync_every)");
        return JACOBI_ERR_INVALID_ARG;
    }
    if (n > (int64_t)INT32_MAX || k > 4096) {
        set_error("size out of supported range");
        return JACOBI_ERR_INVALID_ARG;
    }
    return JACOBI_OK;
}

static jacobi_status validation_status(const Ctl& h, int64_t* bad) {
    const int64_t bz = h.bad_zero, bn = h.bad_nonfinite, br = h.bad_rhs;
    if (bz != INT64_MAX || bn != INT64_MAX) {
        if (bz < bn) {
            *bad = bz;
            return JACOBI_ERR_ZERO_DIAGONAL;
        }
        *bad = bn;
        return JACOBI_ERR_NONFINITE_INPUT;
    }
    *bad = br;
    return JACOBI_ERR_NONFINITE_INPUT;
}

static double bits_to_double(uint64_t b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// Run Jacobi sweeps on the prepared buffers until the device stop flag is set
// or `cap` sweeps ran.  bufs[0] holds x^(0); sweep s reads bufs[(s-1)&1] and
// writes bufs[s&1].  Returns the stop code and the number of sweeps whose
// result is final (K); the final iterate lives in bufs[K & 1].
jacobi_status run_sweeps(const SweepCtl& sc, int32_t a_dtype, SweepArgs args,
                         const LaunchCfg& cfg, void* bufs[2], int32_t cap, int32_t sync_every,
                         int profile, hipStream_t s, uint32_t* stop_out, int32_t* k_out,
                         double* delta_out, double* xmax_out, double* kernel_ms,
                         int64_t* launches) {
    int32_t done = 0;
    // Launches queued after the device decided to stop return at once (a few
    // microseconds each), so a small system, whose sweeps cost about as much
    // as a launch, starts with a longer group and saves host round trips.
    const double sweep_bytes =
        (double)args.n * (double)args.lda * (a_dtype == JACOBI_F64 ? 8 : 4);
    int32_t chunk = sync_every > 0 ? sync_every : (sweep_bytes <= 64.0 * 1024 * 1024 ? 16 : 4);
    *stop_out = STOP_RUNNING;
    if (profile && !sc.prof_ev) {
        set_error("per-sweep profiling is not available here");
        return JACOBI_ERR_INVALID_ARG;
    }
    if (profile && (int)sc.prof_ev->size() < 2 * 512) {
        while ((int)sc.prof_ev->size() < 2 * 512) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            sc.prof_ev->push_back(e);
        }
    }
    Ctl* const h_ctl = sc.h_ctl;
    const int32_t max_chunk = profile ? 512 : 256;
    while (done < cap) {
        int32_t S = std::min(chunk, cap - done);
        if (profile) S = std::min(S, max_chunk);
        for (int32_t q = 1; q <= S; ++q) {
            const int32_t sw = done + q;
            args.sweep = sw;
            args.seq = sw;
            args.xin = bufs[(sw - 1) & 1];
            args.xout = bufs[sw & 1];
            if (profile) HIP_TRY(hipEventRecord((*sc.prof_ev)[2 * (q - 1)], s));
            HIP_TRY(launch_sweep(a_dtype, args, cfg, s));
            if (profile) HIP_TRY(hipEventRecord((*sc.prof_ev)[2 * (q - 1) + 1], s));
        }
        // each launch decides its predecessor; the group's last one is decided
        // here (a no-op when the phase has already stopped)
        HIP_TRY(launch_decide(args, cfg.grid * ((args.k + 31) / 32), s));
        HIP_TRY(hipMemcpyAsync(h_ctl, sc.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const Ctl& h = *h_ctl;
        if (profile) {
            const int32_t ran = h.stop != STOP_RUNNING ? std::max(0, h.stop_sweep - done) : S;
            for (int32_t q = 1; q <= ran; ++q) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, (*sc.prof_ev)[2 * (q - 1)], (*sc.prof_ev)[2 * (q - 1) + 1]));
                *kernel_ms += ms;
                *launches += 1;
            }
        }
        if (h.stop != STOP_RUNNING) {
            *stop_out = h.stop;
            *k_out = h.stop == STOP_INVALID ? 0 : h.stop_sweep;
            *delta_out = bits_to_double(h.last_delta_bits);
            *xmax_out = bits_to_double(h.last_xmax_bits);
            return JACOBI_OK;
        }
        done += S;
        if (sync_every == 0) chunk = std::min(chunk * 2, 256);
    }
    if (cap == 0) {
        HIP_TRY(hipMemcpyAsync(h_ctl, sc.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h_ctl->stop == STOP_INVALID) *stop_out = STOP_INVALID;
        *delta_out = -1.0;
    } else {
        *delta_out = bits_to_double(h_ctl->last_delta_bits);
        *xmax_out = bits_to_double(h_ctl->last_xmax_bits);
    }
    *k_out = cap;
    return JACOBI_OK;
}

jacobi_status solve_plain_locked(jacobi_ctx* c, int64_t n, int64_t k, int32_t a_dtype,
                                 const void* A, int64_t lda, const void* B, int64_t ldb,
                                 const void* X0, void* X, int64_t ldx, const jacobi_options& o,
                                 hipStream_t s, jacobi_info* info) {
    // Several right-hand sides: the sweep is a real dense contraction, run
    // on MFMA tiles (FP32 for FP32/BF16 A, FP64 for FP64 A) by the
    // persistent kernel.  The vector kernel keeps one or two columns, where
    // it streams faster (n = 16384, TB/s, vector / MFMA: FP64 k = 1 6.8 / 4.9,
    // k = 2 5.9 / 4.9; FP32 k = 2 5.9 / 4.4; BF16 k = 2 3.6 / 3.4); from three
    // columns its per-column reductions fall behind (k = 3: FP64 2.5, FP32
    // 3.0, BF16 1.4 against 4.9, 4.3 and 3.4 on the tiles).
    if (k >= mfma_min_cols(a_dtype) && k <= 32 && o.profile == 0) {
        BatchItem it{n, k, A, lda, B, ldb, X0, X, ldx, o.max_iter};
        jacobi_status st = run_batched(c, 1, &it, a_dtype, o, TEST_ABS, 0.0, s, info, true);
        if (st != JACOBI_OK) return st;
        if (info->status < 0 && info->status != JACOBI_ERR_INTERNAL)
            set_error("input validation failed at row %lld", (long long)info->bad_index);
        return (jacobi_status)info->status;
    }
    const int kp = kpad_for(k);
    const size_t sx = a_dtype == JACOBI_F64 ? 8 : 4;
    HIP_TRY(c->diag.ensure(sx * n));
    HIP_TRY(c->w0.ensure(sx * n * kp));
    HIP_TRY(c->w1.ensure(sx * n * kp));
    PlainWs w{sweep_ctl(c), c->slots, c->parts, c->diag.p, c->w0.p, c->w1.p,
              c->ev_begin, c->ev_end, c->num_cus, c->h_ctl_dev, &c->small_chain};
    return solve_plain_vec(w, n, k, a_dtype, A, lda, B, ldb, X0, X, ldx, o, s, info);
}

// Small systems: every sweep in one persistent launch instead of one launch
// per sweep, whose launch cost exceeds such a sweep.  The register-resident
// variant (k_small_reg: each wave loads its rows of A once, then one memory
// round trip per sweep) runs whenever every wave's rows fit its registers
// with at most one workgroup per CU; otherwise the LDS variant (k_small: A
// re-read every sweep) runs while A holds at most 12 MiB and the iterate
// fits its LDS.  Measured per solve (us; register / LDS / per-sweep vector
// kernel): FP64 n = 512: 99 / 118 / 154, n = 2048: 182 / 283 / 206; FP32
// n = 2048: 141 / 167 / 171, n = 3072 (no register fit): - / 227 / 173;
// BF16 n = 4096: 142 / 254 / 187.  JACOBI_SMALL_MAX (rows) overrides the
// bound, 0 turns both off; JACOBI_SMALL_REG=0 keeps the LDS variant;
// JACOBI_SMALL_ROWS sets the rows per workgroup.
constexpr double kSmallMaxBytes = 12.0 * 1024 * 1024;

// Fewest workgroups with which every wave's rows of an n-row system fit the
// register variant's registers, or 0 when they do not fit in max_grid.
// Eight waves per workgroup (four rows each, half the workgroups at the grid
// barrier) for FP32 and BF16 A where that variant exists and fits, four for
// FP64 (per solve, us, four / eight waves: FP64 n = 512 81 / 83; FP32 n =
// 1024 74 / 65; BF16 n = 2048 96 / 83); JACOBI_SMALL_WAVES=4|8 overrides.
static int64_t small_reg_min_grid(int32_t a_dtype, int64_t n, int kp, int64_t max_grid,
                                  int* np_out, int* rpw_out, int* waves_out) {
    const char* renv = getenv("JACOBI_SMALL_REG");
    if (renv && atoi(renv) == 0) return 0;
    const int np = small_reg_np(a_dtype, n);
    if (np == 0) return 0;
    const char* wenv = getenv("JACOBI_SMALL_WAVES");
    const int pref = wenv ? (atoi(wenv) == 8 ? 8 : 4) : (a_dtype == JACOBI_F64 ? 4 : 8);
    for (const int waves : {pref, 4}) {
        const int rpw = small_reg_rows_per_wave(a_dtype, kp, np, waves);
        if (rpw <= 0) continue;
        const int64_t per = (int64_t)waves * rpw;
        const int64_t need = std::max<int64_t>(1, (n + per - 1) / per);
        if (need > max_grid) continue;
        if (np_out) *np_out = np;
        if (rpw_out) *rpw_out = rpw;
        if (waves_out) *waves_out = waves;
        return need;
    }
    return 0;
}

static bool small_eligible(int32_t a_dtype, int64_t n, int kp, int num_cus) {
    const char* env = getenv("JACOBI_SMALL_MAX");
    if (env && n > atoll(env)) return false;
    if (small_reg_min_grid(a_dtype, n, kp, std::min<int64_t>(num_cus, kMaxParts), nullptr,
                           nullptr, nullptr) > 0)
        return true;
    if (n > small_max_rows(a_dtype, kp)) return false;
    return env || (double)n * (double)n * (double)dtype_bytes(a_dtype) <= kSmallMaxBytes;
}

// Launches the small-system kernel.  Unless sa.fused, also copies the control
// block back, waits, and returns the outcome; a fused launch (register
// variant only) writes its outcome to the host mirror and X itself, and the
// caller waits.
static jacobi_status run_small(const PlainWs& w, int32_t a_dtype, SmallArgs sa, int kp,
                               bool aligned, hipStream_t s, uint32_t* stop_out, int32_t* k_out,
                               double* delta_out, double* xmax_out, bool* reg_out,
                               int* grid_out) {
    const int64_t max_grid = std::min<int64_t>(w.num_cus, kMaxParts);
    int np = 0, rpw = 0, waves = 4;
    const int64_t reg_grid = small_reg_min_grid(a_dtype, sa.n, kp, max_grid, &np, &rpw, &waves);
    const bool reg = reg_grid > 0;
    // rows per workgroup: 4 per wave for the register variant, 8 (2 per wave)
    // for the LDS one, measured best at n = 512
    int64_t rows = reg ? 4 * waves : 8;
    if (const char* env = getenv("JACOBI_SMALL_ROWS")) rows = std::max<int64_t>(1, atoll(env));
    int grid = (int)std::max<int64_t>(1, std::min<int64_t>(max_grid, (sa.n + rows - 1) / rows));
    if (reg) grid = (int)std::max<int64_t>(grid, reg_grid);
    int rate_khz = 100000;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    sa.spin_limit = (int64_t)rate_khz * 1000 * 20;  // 20 s
    sa.aligned = aligned ? 1 : 0;
    if (sa.fused && !reg) return JACOBI_ERR_INTERNAL;  // the caller checked the fit
    *grid_out = grid;
    if (sa.fused) w.sc.h_ctl->timeout = 0;  // host write, before the launch
    if (reg)
        HIP_TRY(launch_small_reg(a_dtype, sa, kp, np, waves, grid, s));
    else
        HIP_TRY(launch_small(a_dtype, sa, kp, aligned, grid, s));
    *reg_out = reg;
    if (sa.fused) return JACOBI_OK;
    HIP_TRY(hipMemcpyAsync(w.sc.h_ctl, w.sc.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const Ctl& h = *w.sc.h_ctl;
    if (h.stop == STOP_TIMEOUT) {
        set_error("a grid barrier wait of the small-system kernel timed out");
        return JACOBI_ERR_INTERNAL;
    }
    *stop_out = h.stop;
    *k_out = h.stop == STOP_INVALID ? 0 : (h.stop != STOP_RUNNING ? h.stop_sweep : sa.cap);
    *delta_out = sa.cap > 0 ? bits_to_double(h.last_delta_bits) : -1.0;
    *xmax_out = bits_to_double(h.last_xmax_bits);
    return JACOBI_OK;
}

jacobi_status solve_plain_vec(const PlainWs& w, int64_t n, int64_t k, int32_t a_dtype,
                              const void* A, int64_t lda, const void* B, int64_t ldb,
                              const void* X0, void* X, int64_t ldx, const jacobi_options& o,
                              hipStream_t s, jacobi_info* info) {
    const int kp = kpad_for(k);
    const size_t sx = a_dtype == JACOBI_F64 ? 8 : 4;
    const LaunchCfg cfg = default_cfg(a_dtype, n, (int)k, w.num_cus);
    if (cfg.grid * ((k + 31) / 32) > kMaxParts) {
        set_error("grid too large");
        return JACOBI_ERR_INVALID_ARG;
    }
    Ctl* const ctl = w.sc.ctl;
    const bool small =
        o.profile == 0 && o.sync_every == 0 && small_eligible(a_dtype, n, kp, w.num_cus);
    // Fused small solve: the register variant also takes the set-up's place
    // and the copy-out, and leaves its outcome in the mapped host mirror:
    // k_init_ctl and that launch, then one wait.  JACOBI_SMALL_FUSED=0 keeps
    // the separate set-up, read-back and copy-out.
    const char* fenv = getenv("JACOBI_SMALL_FUSED");
    const bool x0_packed =
        X0 == nullptr || (ldx == kp && (uintptr_t)X0 % 16 == 0);
    const bool fused = small && o.max_iter >= 1 && w.h_ctl_dev != nullptr && x0_packed &&
                       !(fenv && atoi(fenv) == 0) &&
                       small_reg_min_grid(a_dtype, n, kp, std::min<int64_t>(w.num_cus, kMaxParts),
                                          nullptr, nullptr, nullptr) > 0;
    // A fused launch after a fused launch on the same control block skips
    // k_init_ctl (the kernel continues the barrier count and the slot
    // rotation the previous one left); any other use of the block, a timeout
    // or invalid input makes the next one initialise it.
    SmallChain* const chain = w.chain;
    const bool chained = fused && chain != nullptr && chain->ready;
    if (chain) chain->ready = false;
    if (w.ev_begin) HIP_TRY(hipEventRecord(w.ev_begin, s));
    if (!chained) {
        HIP_TRY(launch_init_ctl(ctl, w.slots, 1, s));
        if (chain) {
            chain->bar_base = 0;
            chain->slot_base = 0;
        }
    }
    if (!fused)
        HIP_TRY(launch_setup(a_dtype, A, lda, B, ldb, X0, ldx, n, (int)k, kp, w.diag, w.w0,
                             w.w1, ctl, s));
    SweepArgs a{};
    a.A = A;
    a.lda = lda;
    a.B = B;
    a.ldb = ldb;
    a.diag = w.diag;
    a.n = n;
    a.k = (int)k;
    a.kpad = kp;
    a.ldin = kp;
    a.ldout = kp;
    a.ctl = ctl;
    a.slots = w.slots;
    a.parts = w.parts;
    a.tol = o.tol;
    a.test = TEST_ABS;
    a.norm = o.norm;
    const size_t ea = dtype_bytes(a_dtype);
    a.aligned = (((uintptr_t)A % 16) == 0 && ((size_t)lda * ea) % 16 == 0) ? 1 : 0;
    void* bufs[2] = {w.w0, w.w1};
    uint32_t stop = 0;
    int32_t K = 0;
    double delta = -1.0, xmax = 0.0, kms = 0.0;
    int64_t launches = 0;
    jacobi_status st;
    bool reg = false;
    if (small) {
        SmallArgs sa{};
        sa.A = A;
        sa.lda = lda;
        sa.B = B;
        sa.ldb = ldb;
        sa.diag = w.diag;
        sa.n = n;
        sa.k = (int32_t)k;
        sa.cap = o.max_iter;
        sa.buf0 = w.w0;
        sa.buf1 = w.w1;
        sa.ctl = ctl;
        sa.slots = w.slots;
        sa.parts = w.parts;
        sa.tol = o.tol;
        sa.norm = o.norm;
        // JACOBI_SMALL_ATOMIC_GRID overrides the largest grid that gathers
        // the distance's maximum with atomics (tuning and diagnosis)
        sa.atomic_max_grid = kSmallAtomicMaxGrid;
        if (const char* env = getenv("JACOBI_SMALL_ATOMIC_GRID")) sa.atomic_max_grid = atoi(env);
        if (fused) {
            sa.fused = 1;
            sa.X0 = X0;
            sa.ldx0 = ldx;
            sa.X = X;
            sa.ldx = ldx;
            sa.hctl = w.h_ctl_dev;
            sa.bar_base = chain ? chain->bar_base : 0u;
            sa.slot_base = chain ? chain->slot_base : 0;
        }
        int grid = 0;
        st = run_small(w, a_dtype, sa, kp, a.aligned != 0, s, &stop, &K, &delta, &xmax, &reg,
                       &grid);
        if (st == JACOBI_OK && fused) {
            if (w.ev_begin && w.ev_end) {
                HIP_TRY(hipEventRecord(w.ev_end, s));
                HIP_TRY(hipEventSynchronize(w.ev_end));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, w.ev_begin, w.ev_end));
                info->device_ms = ms;
            } else {
                HIP_TRY(hipStreamSynchronize(s));
                info->device_ms = -1.0;
            }
            const Ctl& h = *w.sc.h_ctl;
            if (h.timeout != 0) {
                set_error("a grid barrier wait of the small-system kernel timed out");
                return JACOBI_ERR_INTERNAL;
            }
            info->bad_index = -1;
            if (h.stop == STOP_INVALID) {
                jacobi_status vs = validation_status(h, &info->bad_index);
                info->status = vs;
                info->iterations = 0;
                info->final_delta = -1.0;
                set_error("input validation failed at row %lld", (long long)info->bad_index);
                return vs;
            }
            if (chain) {
                // every workgroup arrived at barriers 1 .. sweeps_done; after
                // a launch that used the slots, the one after the last
                // computed sweep's is clear (a larger grid leaves them as
                // they were)
                chain->bar_base += (uint32_t)grid * (uint32_t)h.sweeps_done;
                if (grid <= sa.atomic_max_grid)
                    chain->slot_base = (chain->slot_base + h.sweeps_done) % 3;
                chain->ready = true;
            }
            K = h.stop != STOP_RUNNING ? h.stop_sweep : o.max_iter;
            info->iterations = K;
            info->final_delta = bits_to_double(h.last_delta_bits);
            info->sweep_kernel_ms = 0.0;
            info->sweep_kernel_launches = 0;
            info->kernel = 129;
            jacobi_status res = JACOBI_NOT_CONVERGED;
            if (h.stop == STOP_CONVERGED) res = JACOBI_OK;
            if (h.stop == STOP_DIVERGED) res = JACOBI_DIVERGED;
            info->status = res;
            return res;
        }
    } else {
        st = run_sweeps(w.sc, a_dtype, a, cfg, bufs, o.max_iter, o.sync_every, o.profile, s,
                        &stop, &K, &delta, &xmax, &kms, &launches);
    }
    if (st != JACOBI_OK) return st;
    info->bad_index = -1;
    if (stop == STOP_INVALID) {
        jacobi_status vs = validation_status(*w.sc.h_ctl, &info->bad_index);
        info->status = vs;
        info->iterations = 0;
        info->final_delta = -1.0;
        HIP_TRY(hipStreamSynchronize(s));
        set_error("input validation failed at row %lld", (long long)info->bad_index);
        return vs;
    }
    HIP_TRY(launch_copy_rows((int)sx, bufs[K & 1], kp, X, ldx, n, (int)k, s));
    if (w.ev_begin && w.ev_end) {
        HIP_TRY(hipEventRecord(w.ev_end, s));
        HIP_TRY(hipEventSynchronize(w.ev_end));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, w.ev_begin, w.ev_end));
        info->device_ms = ms;
    } else {
        HIP_TRY(hipStreamSynchronize(s));
        info->device_ms = -1.0;
    }
    info->iterations = K;
    info->final_delta = K > 0 ? delta : -1.0;
    info->sweep_kernel_ms = kms;
    info->sweep_kernel_launches = launches;
    info->kernel = small ? (reg ? 129 : 128) : 0;
    jacobi_status res = JACOBI_NOT_CONVERGED;
    if (stop == STOP_CONVERGED) res = JACOBI_OK;
    if (stop == STOP_DIVERGED) res = JACOBI_DIVERGED;
    info->status = res;
    return res;
}

}  // namespace jac

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void jacobi_options_default(jacobi_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_iter = 10000;
    o->norm = JACOBI_NORM_INF;
    o->mode = JACOBI_MODE_PLAIN;
    o->sweep_dtype = JACOBI_BF16;
    o->inner_rel_tol = 1e-3;
    o->max_inner = 200;
    o->max_outer = 50;
    o->refine_tol = 1e-12;
    o->sync_every = 0;
    o->profile = 0;
}

jacobi_status jacobi_ctx_create(int32_t device, jacobi_ctx** out) {
    try {
        if (!out) return JACOBI_ERR_INVALID_ARG;
        *out = nullptr;
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess) {
            set_error("hipGetDeviceCount failed");
            return JACOBI_ERR_DEVICE;
        }
        if (device < 0 || device >= count) {
            set_error("device %d out of range (%d devices)", device, count);
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_ctx* c = new (std::nothrow) jacobi_ctx();
        if (!c) return JACOBI_ERR_OUT_OF_MEMORY;
        jacobi_status s = ctx_init(c, device);
        if (s != JACOBI_OK) {
            ctx_release(c);
            delete c;
            return s;
        }
        *out = c;
        return JACOBI_OK;
    } catch (...) {
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_ctx_destroy(jacobi_ctx* c) {
    try {
        if (!c) return JACOBI_ERR_INVALID_ARG;
        {
            std::lock_guard<std::mutex> g(c->mu);
            ctx_release(c);
        }
        delete c;
        return JACOBI_OK;
    } catch (...) {
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_solve(jacobi_ctx* ctx, int64_t n, int64_t k, int32_t a_dtype, const void* A,
                           int64_t lda, const void* B, int64_t ldb, const void* X0, void* X,
                           int64_t ldx, const jacobi_options* opt, hipStream_t stream,
                           jacobi_info* info) {
    try {
        jacobi_info local;
        if (!info) info = &local;
        std::memset(info, 0, sizeof(*info));
        info->status = JACOBI_ERR_INVALID_ARG;
        info->bad_index = -1;
        info->final_delta = -1.0;
        info->rel_residual = -1.0;
        jacobi_options o;
        jacobi_options_default(&o);
        if (opt) o = *opt;
        jacobi_status st = check_common(n, k, a_dtype, A, lda, B, ldb, X, ldx, o);
        if (st != JACOBI_OK) return (jacobi_status)(info->status = st);
        if (o.mode == JACOBI_MODE_REFINE && a_dtype != JACOBI_F64) {
            set_error("REFINE mode needs an FP64 system");
            return (jacobi_status)(info->status = JACOBI_ERR_INVALID_ARG);
        }
        jacobi_ctx* c = ctx;
        if (!c) {
            c = default_ctx(&st);
            if (!c) return (jacobi_status)(info->status = st);
        }
        std::lock_guard<std::mutex> g(c->mu);
        if (hipSetDevice(c->device) != hipSuccess) {
            set_error("hipSetDevice(%d) failed", c->device);
            return (jacobi_status)(info->status = JACOBI_ERR_DEVICE);
        }
        if (o.mode == JACOBI_MODE_REFINE)
            st = solve_refine(c, n, k, A, lda, B, ldb, X0, X, ldx, o, stream, info);
        else
            st = solve_plain_locked(c, n, k, a_dtype, A, lda, B, ldb, X0, X, ldx, o, stream, info);
        info->status = st;
        return st;
    } catch (...) {
        set_error("internal exception");
        if (info) info->status = JACOBI_ERR_INTERNAL;
        return JACOBI_ERR_INTERNAL;
    }
}

const char* jacobi_status_string(int32_t s) {
    switch (s) {
        case JACOBI_OK: return "OK";
        case JACOBI_NOT_CONVERGED: return "NOT_CONVERGED";
        case JACOBI_DIVERGED: return "DIVERGED";
        case JACOBI_PENDING: return "PENDING";
        case JACOBI_CANCELLED: return "CANCELLED";
        case JACOBI_ERR_INVALID_ARG: return "ERR_INVALID_ARG";
        case JACOBI_ERR_ZERO_DIAGONAL: return "ERR_ZERO_DIAGONAL";
        case JACOBI_ERR_NONFINITE_INPUT: return "ERR_NONFINITE_INPUT";
        case JACOBI_ERR_OUT_OF_MEMORY: return "ERR_OUT_OF_MEMORY";
        case JACOBI_ERR_DEVICE: return "ERR_DEVICE";
        case JACOBI_ERR_REJECTED: return "ERR_REJECTED";
        case JACOBI_ERR_INTERNAL: return "ERR_INTERNAL";
    }
    return "UNKNOWN";
}

const char* jacobi_last_error(void) { return jac::g_last_error.c_str(); }

jacobi_status jacobi_shutdown(void) {
    try {
        std::vector<jacobi_ctx*> all;
        {
            std::lock_guard<std::mutex> g(jac::g_default_mu);
            all.swap(jac::g_default_ctx);
        }
        for (jacobi_ctx* c : all) {
            if (!c) continue;
            {
                std::lock_guard<std::mutex> g(c->mu);
                hipSetDevice(c->device);
                hipDeviceSynchronize();
                ctx_release(c);
            }
            delete c;
        }
        return JACOBI_OK;
    } catch (...) {
        return JACOBI_ERR_INTERNAL;
    }
}

}  // extern "C"
