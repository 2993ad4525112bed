// Host-side declarations of the batched (persistent MFMA) solver.
#pragma once

#include <vector>

#include "ctx.h"
#include "plan.h"

namespace jac {

// One system handed to the persistent kernel (device pointers, FP32 B/X).
struct BatchItem {
    int64_t n, k;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    const void* X0;
    void* X;
    int64_t ldx;
    int32_t max_iter;
    // 1: start from x^(1) = B / a_ii, the first sweep from x^(0) = 0 (which
    // multiplies every off-diagonal entry by zero), computed by the setup
    // kernel without a pass over A; X0 is ignored, max_iter counts the
    // sweeps after it and the reported count excludes it.  For relative stop
    // tests with rel < 1, which that first sweep can never meet.
    int32_t first_free = 0;
};

// allow_split: a single system may have its columns split over workgroups
// (its arithmetic then depends on the chunk count the tuner picks, so the
// batched and served paths, whose results must not depend on the batch,
// leave it off).
jacobi_status run_batched(jacobi_ctx* c, int32_t count, const BatchItem* items, int32_t a_dtype,
                          const jacobi_options& o, int32_t test, double rel, hipStream_t s,
                          jacobi_info* infos, bool allow_split = false);

jacobi_status solve_plain_locked(jacobi_ctx* c, int64_t n, int64_t k, int32_t a_dtype,
                                 const void* A, int64_t lda, const void* B, int64_t ldb,
                                 const void* X0, void* X, int64_t ldx, const jacobi_options& o,
                                 hipStream_t s, jacobi_info* info);

}  // namespace jac
