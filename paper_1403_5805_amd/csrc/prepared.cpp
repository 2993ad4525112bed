// Prepared matrices: an A kept for repeated solves with new right-hand sides.
// For refinement the reduced-precision copy A_lo = RNE(A) and its diagonal are
// built once, in the handle's own device memory, instead of once per solve.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "batch.h"
#include "ctx.h"

struct jacobi_matrix {
    jacobi_ctx* ctx = nullptr;  // the context the solves run in (null: the default one)
    int device = 0;
    int64_t n = 0;
    int32_t a_dtype = 0;
    const void* A = nullptr;    // the caller's matrix (not copied)
    int64_t lda = 0;
    int32_t lo_dtype = -1;      // JACOBI_F32 / JACOBI_BF16: A_lo built; -1: none
    int64_t ld_lo = 0;
    jac::DevBuf alo, diag_lo;
};

using namespace jac;

extern "C" {

jacobi_status jacobi_matrix_create(jacobi_ctx* ctx, int64_t n, int32_t a_dtype, const void* A,
                                   int64_t lda, int32_t lo_dtype, hipStream_t stream,
                                   jacobi_matrix** out) {
    try {
        if (!out) {
            set_error("null output handle");
            return JACOBI_ERR_INVALID_ARG;
        }
        *out = nullptr;
        if (n < 1 || lda < n || !A ||
            (a_dtype != JACOBI_F64 && a_dtype != JACOBI_F32 && a_dtype != JACOBI_BF16) ||
            (lo_dtype != -1 && lo_dtype != JACOBI_F32 && lo_dtype != JACOBI_BF16) ||
            (lo_dtype != -1 && a_dtype != JACOBI_F64) || n > (int64_t)INT32_MAX) {
            set_error("invalid matrix (n >= 1, lda >= n, A, dtype; a reduced copy needs FP64 A)");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_status st = JACOBI_OK;
        jacobi_ctx* c = ctx ? ctx : default_ctx(&st);
        if (!c) return st;
        auto* m = new jacobi_matrix();
        m->ctx = ctx;
        m->device = c->device;
        m->n = n;
        m->a_dtype = a_dtype;
        m->A = A;
        m->lda = lda;
        m->lo_dtype = lo_dtype;
        if (lo_dtype != -1) {
            if (hipSetDevice(c->device) != hipSuccess) {
                delete m;
                set_error("hipSetDevice(%d) failed", c->device);
                return JACOBI_ERR_DEVICE;
            }
            const size_t elo = lo_dtype == JACOBI_F32 ? 4 : 2;
            m->ld_lo = (n + 7) / 8 * 8;  // 16-byte aligned rows
            hipError_t e = m->alo.ensure(elo * (size_t)n * (size_t)m->ld_lo);
            if (e == hipSuccess) e = m->diag_lo.ensure(4 * (size_t)n);
            if (e == hipSuccess)
                e = launch_convert((const double*)A, lda, n, lo_dtype, m->alo.p, m->ld_lo, stream);
            if (e == hipSuccess)
                e = launch_gather_diag(lo_dtype, m->alo.p, m->ld_lo, n, m->diag_lo.p, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                m->alo.release();
                m->diag_lo.release();
                delete m;
                set_error("building the reduced copy failed: %s", hipGetErrorString(e));
                return e == hipErrorOutOfMemory ? JACOBI_ERR_OUT_OF_MEMORY : JACOBI_ERR_DEVICE;
            }
        }
        *out = m;
        return JACOBI_OK;
    } catch (...) {
        set_error("internal exception");
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_solve_prepared(jacobi_matrix* m, int64_t k, const void* B, int64_t ldb,
                                    const void* X0, void* X, int64_t ldx,
                                    const jacobi_options* opt, hipStream_t stream,
                                    jacobi_info* info) {
    try {
        if (!m) {
            set_error("null matrix");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_options o;
        jacobi_options_default(&o);
        if (opt) o = *opt;
        if (o.mode != JACOBI_MODE_REFINE)  // the plain solve of the kept A
            return jacobi_solve(m->ctx, m->n, k, m->a_dtype, m->A, m->lda, B, ldb, X0, X, ldx,
                                &o, stream, info);
        jacobi_info local;
        if (!info) info = &local;
        std::memset(info, 0, sizeof(*info));
        info->status = JACOBI_ERR_INVALID_ARG;
        info->bad_index = -1;
        info->final_delta = -1.0;
        info->rel_residual = -1.0;
        if (m->lo_dtype == -1 || m->lo_dtype != o.sweep_dtype) {
            set_error("REFINE with a prepared matrix needs its reduced copy in the sweep dtype");
            return JACOBI_ERR_INVALID_ARG;
        }
        jacobi_status st =
            check_common(m->n, k, m->a_dtype, m->A, m->lda, B, ldb, X, ldx, o);
        if (st != JACOBI_OK) return (jacobi_status)(info->status = st);
        jacobi_ctx* c = m->ctx ? m->ctx : default_ctx(&st);
        if (!c) return (jacobi_status)(info->status = st);
        std::lock_guard<std::mutex> g(c->mu);
        if (hipSetDevice(c->device) != hipSuccess) {
            set_error("hipSetDevice(%d) failed", c->device);
            return (jacobi_status)(info->status = JACOBI_ERR_DEVICE);
        }
        const PreparedLo pre{m->alo.p, m->ld_lo, (const float*)m->diag_lo.p, m->lo_dtype};
        st = solve_refine(c, m->n, k, m->A, m->lda, B, ldb, X0, X, ldx, o, stream, info, &pre);
        info->status = st;
        return st;
    } catch (...) {
        set_error("internal exception");
        if (info) info->status = JACOBI_ERR_INTERNAL;
        return JACOBI_ERR_INTERNAL;
    }
}

jacobi_status jacobi_matrix_destroy(jacobi_matrix* m) {
    if (!m) return JACOBI_OK;
    if (m->alo.p || m->diag_lo.p) {
        hipSetDevice(m->device);
        m->alo.release();
        m->diag_lo.release();
    }
    delete m;
    return JACOBI_OK;
}

}  // extern "C"
