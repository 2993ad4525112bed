// Mixed-precision iterative refinement around the Jacobi sweep.
//
// The system of record is FP64 (A, B, X).  A reduced-precision copy A_lo
// (FP32 or BF16, round to nearest even) is built on the device once per call.
// Outer loop:   r = B - A x            (FP64 residual pass over FP64 A)
//               stop if ||r||_2 < refine_tol * ||B||_2
//               solve A_lo d = r       (Jacobi sweeps, FP32 accumulation,
//                                       d^0 = 0, relative stop)
//               x = x + d              (FP64, fused into the next residual pass)
// The residual and the update are the only FP64 steps on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <cmath>

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

static int kpad_of(int64_t k) {
    if (k <= 32) {
        int kt = 1;
        while (kt < k) kt <<= 1;
        return kt;
    }
    return (int)((k + 31) / 32 * 32);
}

static double bits_to_double(uint64_t b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

jacobi_status solve_refine(jacobi_ctx* c, int64_t n, int64_t k, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* X0, void* X, int64_t ldx,
                           const jacobi_options& o, hipStream_t s, jacobi_info* info,
                           const PreparedLo* pre) {
    c->small_chain.ready = false;  // this path re-initialises ctl and its slots
    const int32_t lo = o.sweep_dtype;
    if ((lo != JACOBI_F32 && lo != JACOBI_BF16) || !(o.inner_rel_tol >= 0.0) ||
        !(o.refine_tol >= 0.0) || o.max_inner < 1 || o.max_outer < 0) {
        set_error("invalid refinement options");
        return JACOBI_ERR_INVALID_ARG;
    }
    if (pre && pre->lo_dtype != lo) {
        set_error("the matrix was prepared for another sweep dtype");
        return JACOBI_ERR_INVALID_ARG;
    }
    const int kp = kpad_of(k);
    const size_t elo = lo == JACOBI_F32 ? 4 : 2;
    // 16-byte aligned rows for both FP32 and BF16 (or the prepared copy's)
    const int64_t ld_lo = pre ? pre->ld_lo : (n + 7) / 8 * 8;
    HIP_TRY(c->diag.ensure(8 * n));
    HIP_TRY(c->xa.ensure(8 * n * kp));
    HIP_TRY(c->xb.ensure(8 * n * kp));
    HIP_TRY(c->r64.ensure(8 * n * kp));
    HIP_TRY(c->rlo.ensure(4 * n * kp));
    HIP_TRY(c->d0.ensure(4 * n * kp));
    HIP_TRY(c->d1.ensure(4 * n * kp));
    HIP_TRY(c->scal.ensure(64));
    if (!pre) {
        HIP_TRY(c->diag_lo.ensure(4 * n));
        HIP_TRY(c->alo.ensure(elo * (size_t)n * ld_lo));
    }
    void* const alo = pre ? const_cast<void*>(pre->alo) : c->alo.p;
    float* const diag_lo = pre ? const_cast<float*>(pre->diag) : (float*)c->diag_lo.p;
    // Several right-hand sides: the residual runs on FP64 MFMA tiles and (from
    // 3 columns, as in the plain solve) the inner solve on the FP32 MFMA
    // kernel; one column streams through the vector kernels.
    // (k = 1 measured 20% slower on the MFMA residual: the FP64 tiles pad one
    // column to sixteen, and the vector kernel streams a single column well.)
    const bool mfma_resid = k >= 2 && k <= 32;
    const bool mfma_inner = k >= mfma_min_cols(lo) && k <= 32;
    if (mfma_resid) HIP_TRY(c->xT.ensure(resid_xT_bytes(n, k)));

    HIP_TRY(hipEventRecord(c->ev_begin, s));
    // Validation of the FP64 system and x^(0) into xa.
    HIP_TRY(launch_init_ctl(c->ctl, c->slots, 1, s));
    HIP_TRY(launch_setup(JACOBI_F64, A, lda, B, ldb, X0, ldx, n, (int)k, kp, c->diag.p, c->xa.p,
                         c->xb.p, c->ctl, s));
    HIP_TRY(launch_bnorm((const double*)B, ldb, n, (int)k, (double*)c->scal.p, s));
    HIP_TRY(hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    double bnorm = 0.0;
    HIP_TRY(hipMemcpyAsync(&bnorm, c->scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->h_ctl->stop == STOP_INVALID) {
        const Ctl& h = *c->h_ctl;
        jacobi_status vs;
        if (h.bad_zero != INT64_MAX || h.bad_nonfinite != INT64_MAX) {
            vs = h.bad_zero < h.bad_nonfinite ? JACOBI_ERR_ZERO_DIAGONAL
                                              : JACOBI_ERR_NONFINITE_INPUT;
            info->bad_index = std::min(h.bad_zero, h.bad_nonfinite);
        } else {
            vs = JACOBI_ERR_NONFINITE_INPUT;
            info->bad_index = h.bad_rhs;
        }
        set_error("input validation failed at row %lld", (long long)info->bad_index);
        return vs;
    }
    // A_lo = round(A) and its diagonal.  From x0 = 0 the first residual is B
    // itself and reads no A.  Otherwise, with one column, the first residual
    // pass writes A_lo while it streams A (one read of the FP64 matrix
    // instead of two); the MFMA residual leaves it to the conversion kernel.
    const bool zero_start = X0 == nullptr;
    bool fuse_convert = !pre && !mfma_resid && !zero_start;
    if (const char* env = getenv("JACOBI_REFINE_FUSED_CONVERT"))
        fuse_convert = fuse_convert && strcmp(env, "0") != 0;
    if (!pre && !fuse_convert) {
        HIP_TRY(launch_convert((const double*)A, lda, n, lo, alo, ld_lo, s));
        HIP_TRY(launch_gather_diag(lo, alo, ld_lo, n, diag_lo, s));
    }
    const LaunchCfg rcfg = residual_cfg(n, (int)k, c->num_cus);
    const LaunchCfg icfg = default_cfg(lo, n, (int)k, c->num_cus);

    void* xcur = c->xa.p;
    void* xnext = c->xb.p;
    const float* dlt = nullptr;  // correction to add in the next residual pass
    int32_t inner_total = 0, outer = 0;
    double rel = -1.0, last_delta = -1.0, kms = 0.0;
    int64_t launches = 0;
    jacobi_status result = JACOBI_NOT_CONVERGED;
    // One residual pass: x <- x + d, r = B - A x, ||r||_2 / ||B||_2.  Leaves
    // the outcome (STOP_*) in *stop and the relative residual in rel.
    auto residual_pass = [&](uint32_t* stop) -> jacobi_status {
        if (zero_start && outer == 0) {
            // r = B - A 0 = B exactly; x stays 0; ||r|| / ||B|| = 1 (or 0 for B = 0,
            // where x = 0 solves the system)
            HIP_TRY(launch_rhs_residual((const double*)B, ldb, n, (int)k, kp,
                                        (double*)c->r64.p, (float*)c->rlo.p, s));
            HIP_TRY(launch_copy_rows(8, xcur, kp, xnext, kp, n, (int)k, s));
            *stop = bnorm == 0.0 ? STOP_CONVERGED : STOP_RUNNING;
            rel = bnorm == 0.0 ? 0.0 : 1.0;
            return JACOBI_OK;
        }
        if (mfma_resid) {
            ResidItem it{};
            it.n = n;
            it.k = k;
            it.ldx = kp;
            it.A = (const double*)A;
            it.lda = lda;
            it.B = (const double*)B;
            it.ldb = ldb;
            it.x = (const double*)xcur;
            it.d = dlt;
            it.xnew = (double*)xnext;
            it.r64 = (double*)c->r64.p;
            it.rlo = (float*)c->rlo.p;
            it.xT = (double*)c->xT.p;
            it.bnorm = bnorm;
            it.rel = o.refine_tol;
            RState rs{};
            jacobi_status st = run_resid(c, 1, &it, s, &rs);
            if (st != JACOBI_OK) return st;
            *stop = rs.stop;
            rel = bits_to_double(rs.rel_bits);
            return JACOBI_OK;
        }
        HIP_TRY(launch_init_ctl(c->ctl, c->slots, 0, s));
        SweepArgs ra{};
        ra.A = A;
        ra.lda = lda;
        ra.B = B;
        ra.ldb = ldb;
        ra.xin = xcur;
        ra.xout = xnext;
        ra.ldin = kp;
        ra.ldout = kp;
        ra.n = n;
        ra.k = (int)k;
        ra.kpad = kp;
        ra.sweep = outer + 1;
        ra.seq = 1;
        ra.ctl = c->ctl;
        ra.slots = c->slots;
        ra.parts = c->parts;
        ra.test = TEST_RESID;
        ra.rel = o.refine_tol;
        ra.bnorm = bnorm;
        ra.aligned = (((uintptr_t)A % 16) == 0 && ((size_t)lda * 8) % 16 == 0) ? 1 : 0;
        ra.dlt = dlt;
        ra.r64 = (double*)c->r64.p;
        ra.rlo = (float*)c->rlo.p;
        const bool write_lo = fuse_convert && outer == 0;
        if (write_lo) {
            ra.alo = alo;
            ra.ld_lo = ld_lo;
            ra.lo_dtype = lo;
        }
        HIP_TRY(launch_residual(ra, rcfg, s));
        HIP_TRY(launch_decide(ra, rcfg.grid * (int)((k + 31) / 32), s));
        if (write_lo) HIP_TRY(launch_gather_diag(lo, alo, ld_lo, n, diag_lo, s));
        HIP_TRY(hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *stop = c->h_ctl->stop;
        rel = bits_to_double(c->h_ctl->last_delta_bits);
        return JACOBI_OK;
    };
    // Inner solve A_lo d = r from d = 0 (relative stop); d is left in *dout.
    // Sweep 1 from d = 0 multiplies every off-diagonal entry by zero: d^(1) =
    // r / a_ii, written by one elementwise kernel instead of a pass over A_lo
    // (the same FP32 division, so the same values); it cannot meet the
    // relative test (|d1 - 0| <= rel |d1| needs rel >= 1), and the sweeps go
    // on from d^(1) and count it.
    const bool first_free = o.inner_rel_tol < 1.0 && o.max_inner >= 2;
    auto inner_solve = [&](const float** dout, uint32_t* stop) -> jacobi_status {
        const int32_t cap = first_free ? o.max_inner - 1 : o.max_inner;
        if (mfma_inner) {
            BatchItem it{n, k, alo, ld_lo, c->rlo.p, kp, nullptr, c->d0.p, kp, cap};
            it.first_free = first_free ? 1 : 0;  // the setup kernel writes d^(1)
            jacobi_options io;
            jacobi_options_default(&io);
            io.tol = 0.0;
            io.max_iter = cap;
            jacobi_info ii{};
            jacobi_status st =
                run_batched(c, 1, &it, lo, io, TEST_REL, o.inner_rel_tol, s, &ii, true);
            if (st != JACOBI_OK) return st;
            if (ii.status < 0) return (jacobi_status)ii.status;
            inner_total += ii.iterations + (first_free ? 1 : 0);
            last_delta = ii.final_delta;
            *stop = ii.status == JACOBI_DIVERGED ? STOP_DIVERGED : STOP_RUNNING;
            *dout = (const float*)c->d0.p;
            return JACOBI_OK;
        }
        HIP_TRY(launch_init_ctl(c->ctl, c->slots, 0, s));
        HIP_TRY(launch_zero_rows(4, c->d0.p, kp, n, kp, s));
        if (first_free)
            HIP_TRY(launch_first_sweep((const float*)c->rlo.p, diag_lo, n,
                                       (int)k, kp, (float*)c->d1.p, s));
        else
            HIP_TRY(launch_zero_rows(4, c->d1.p, kp, n, kp, s));
        SweepArgs ia{};
        ia.A = alo;
        ia.lda = ld_lo;
        ia.B = c->rlo.p;
        ia.ldb = kp;
        ia.diag = diag_lo;
        ia.n = n;
        ia.k = (int)k;
        ia.kpad = kp;
        ia.ldin = kp;
        ia.ldout = kp;
        ia.ctl = c->ctl;
        ia.slots = c->slots;
        ia.parts = c->parts;
        ia.test = TEST_REL;
        ia.rel = o.inner_rel_tol;
        ia.norm = JACOBI_NORM_INF;
        ia.aligned = 1;
        // the sweeps start from d^(1) in d1 (or from zero in d0)
        void* dbufs[2] = {first_free ? c->d1.p : c->d0.p, first_free ? c->d0.p : c->d1.p};
        int32_t K = 0;
        double xmax = 0.0;
        jacobi_status st = run_sweeps(sweep_ctl(c), lo, ia, icfg, dbufs, cap, o.sync_every,
                                      o.profile, s, stop, &K, &last_delta, &xmax, &kms,
                                      &launches);
        if (st != JACOBI_OK) return st;
        inner_total += K + (first_free ? 1 : 0);
        *dout = (const float*)dbufs[K & 1];
        return JACOBI_OK;
    };
    for (;;) {
        uint32_t stop = STOP_RUNNING;
        jacobi_status st = residual_pass(&stop);
        if (st != JACOBI_OK) return st;
        std::swap(xcur, xnext);
        outer += 1;
        if (stop == STOP_CONVERGED) {
            result = JACOBI_OK;
            break;
        }
        if (stop == STOP_DIVERGED) {
            result = JACOBI_DIVERGED;
            break;
        }
        if (outer > o.max_outer) {
            result = JACOBI_NOT_CONVERGED;
            break;
        }
        st = inner_solve(&dlt, &stop);
        if (st != JACOBI_OK) return st;
        if (stop == STOP_DIVERGED) {
            result = JACOBI_DIVERGED;
            break;
        }
    }
    HIP_TRY(launch_copy_rows(8, xcur, kp, X, ldx, n, (int)k, s));
    HIP_TRY(hipEventRecord(c->ev_end, s));
    HIP_TRY(hipEventSynchronize(c->ev_end));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_begin, c->ev_end));
    info->device_ms = ms;
    info->iterations = inner_total;
    info->outer_iterations = outer;
    info->rel_residual = rel;
    info->final_delta = last_delta;
    info->sweep_kernel_ms = kms;
    info->sweep_kernel_launches = launches;
    info->bad_index = -1;
    return result;
}

}  // namespace jac
