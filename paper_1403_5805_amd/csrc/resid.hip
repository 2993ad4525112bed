// Batched FP64 residual pass of the mixed-precision refinement (gfx950).
//
// For every system s of a batch, in one launch:
//     x_new = x + d                      (FP64 update with the inner correction)
//     r     = B - A x_new                (FP64 A, FP64 accumulation)
//     ||r||_2 and the outer stop test    ||r||_2 < rel * ||B||_2  or  r == 0
// These are the only FP64 steps of the refinement; the inner Jacobi solve of
// A_lo d = r runs in FP32/BF16 elsewhere.
//
// The contraction A x_new (n x n by n x k, k <= 32) runs on
// v_mfma_f64_16x16x4f64:
//   * a workgroup owns one job: 16 * TPW consecutive rows of one system (TPW
//     depends only on the system's size, so a system is cut the same way in
//     any batch); each of its W waves walks every W-th block of 8 columns for
//     all TPW 16-row tiles, and the W partial tiles are added in wave order
//     through LDS;
//   * lane l loads 16 bytes (2 doubles) of row (l % 16) at columns
//     8b + 2(l / 16) + {0, 1}: one load feeds two MFMA k-steps, the k-index
//     l / 16 of step s standing for column 8b + 2(l / 16) + s;
//   * the B operand is (x + d) kept transposed in a small workspace (row c of
//     the workspace is column c of x_new, zero padded to a multiple of 8), so
//     the matching operand of both k-steps is one 16-byte load that hits the
//     L2 (every job of the system reads it);
//   * the output tile of v_mfma_f64_16x16x4f64 puts element (i, j) in lane
//     16 * (i % 4) + j, register i / 4.
// Each job publishes its sum of r^2; the last job of the system (atomic
// ticket) adds the sums in job order, so ||r||_2 depends only on the system
// and is the same alone and in any batch.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "internal.h"

namespace jac {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ uint64_t wmax(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = __shfl_xor(v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}

template <int KT>
constexpr int max_tiles_per_wave() {
    return KT <= 16 ? 4 : 2;
}

constexpr int kRW = 4;  // waves per workgroup
constexpr int kRU = 2;  // column blocks per pipeline stage

}  // namespace

// x_new = x + d (row-major, ld ldx) and its transposed, zero-padded copy xT;
// clears the per-system outcome.  grid = (row blocks, systems).
template <int KT>
__global__ void k_resid_prep(const RSys* __restrict__ sys, RState* __restrict__ st) {
    const RSys S = sys[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        RState* T = &st[blockIdx.y];
        T->stop = STOP_RUNNING;
        T->ticket = 0u;
        T->rel_bits = 0u;
        T->rmax_bits = 0u;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < S.xld; j += stride) {
#pragma unroll 4
        for (int c = 0; c < KT; ++c) {
            double v = 0.0;
            if (j < S.n && c < S.k) {
                v = S.x[j * S.ldx + c];
                if (S.d) v += (double)S.d[j * S.ldx + c];
            }
            S.xT[(int64_t)c * S.xld + j] = v;
            if (j < S.n && c < S.ldx) S.xnew[j * S.ldx + c] = v;
        }
    }
}

template <int KT, int W, int TPW, int U>
__global__ __launch_bounds__(W * 64) void k_resid(RArgs p) {
    constexpr int NT = KT / 16;      // 16-column output tiles
    constexpr int ROWS = 16 * TPW;   // rows of one job
    constexpr int BW = 8;            // columns of one block
    __shared__ double red[W * TPW * NT * 256];
    __shared__ double red_q[W];
    __shared__ uint64_t red_m[W];
    __shared__ uint32_t s_last;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, li = lane & 15;
    const int job = blockIdx.x;
    const int si = p.job_sys[job];
    const RSys S = p.sys[si];
    const int64_t n = S.n;
    const int64_t r0 = (int64_t)(job - S.job0) * ROWS;

    const double* arow[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int64_t ri = r0 + 16 * q + li;
        if (ri >= n) ri = n - 1;  // rows past n: load a valid row, discard the result
        arow[q] = S.A + ri * S.lda + 2 * grp;
    }
    const double* xrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) xrow[t] = S.xT + (int64_t)(t * 16 + li) * S.xld + 2 * grp;

    f64x4 acc[TPW][NT];
#pragma unroll
    for (int q = 0; q < TPW; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = (f64x4){0.0, 0.0, 0.0, 0.0};

    const int64_t nb = (n + BW - 1) / BW;  // column blocks per row
    const int64_t nbf = n / BW;            // blocks entirely inside the row
    // this wave's full blocks: b = wave + W * t, t < ntw
    const int64_t ntw = nbf > wave ? (nbf - wave + W - 1) / W : 0;
    const int64_t nfull = (ntw / U) * U;
    // The main loop, compiled once for 16-byte row loads (rows 16-byte
    // aligned) and once for pairs of 8-byte loads.
    auto run = [&](auto vec_tag) {
        constexpr bool VEC16 = decltype(vec_tag)::value;
        auto load_a = [&](f64x2 (&a)[TPW], int64_t b) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const double* src = arow[q] + b * BW;
                // ordinary loads: each 128-byte line of a row is shared by
                // the blocks of two waves, and non-temporal loads could fetch
                // it twice
                if constexpr (VEC16) {
                    a[q] = *reinterpret_cast<const f64x2*>(src);
                } else {
                    a[q].x = src[0];
                    a[q].y = src[1];
                }
            }
        };
        auto load_b = [&](f64x2 (&x)[NT], int64_t b) {
#pragma unroll
            for (int t = 0; t < NT; ++t) x[t] = *reinterpret_cast<const f64x2*>(xrow[t] + b * BW);
        };
        auto mma = [&](const f64x2 (&a)[TPW], const f64x2 (&x)[NT]) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int q = 0; q < TPW; ++q)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s], x[t][s],
                                                                         acc[q][t], 0, 0, 0);
        };
        // Full blocks: two pipeline stages of U blocks, the loads of one stage
        // in flight while the MFMAs of the other run; the scheduling barriers
        // keep the compiler from sinking the loads below those MFMAs.
        if (nfull > 0) {
            f64x2 a0[U][TPW], x0[U][NT], a1[U][TPW], x1[U][NT];
            auto issue = [&](f64x2 (&a)[U][TPW], f64x2 (&x)[U][NT], int64_t t0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t b = wave + W * (t0 + u);
                    load_a(a[u], b);
                    load_b(x[u], b);
                }
            };
            auto consume = [&](f64x2 (&a)[U][TPW], f64x2 (&x)[U][NT]) {
#pragma unroll
                for (int u = 0; u < U; ++u) mma(a[u], x[u]);
            };
            issue(a0, x0, 0);
            int64_t t = 0;
            for (; t + 3 * U <= nfull; t += 2 * U) {
                issue(a1, x1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(a0, x0);
                __builtin_amdgcn_sched_barrier(0);
                issue(a0, x0, t + 2 * U);
                __builtin_amdgcn_sched_barrier(0);
                consume(a1, x1);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (t + 2 * U <= nfull) {
                issue(a1, x1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(a0, x0);
                __builtin_amdgcn_sched_barrier(0);
                consume(a1, x1);
            } else {
                consume(a0, x0);
            }
        }
        // Remaining full blocks of this wave and the ragged last block.
        for (int64_t b = wave + W * nfull; b < nb; b += W) {
            f64x2 a[TPW], x[NT];
            if (b < nbf) {
                load_a(a, b);
            } else {
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    const int64_t col = b * BW + 2 * grp;
                    a[q].x = col < n ? arow[q][b * BW] : 0.0;
                    a[q].y = col + 1 < n ? arow[q][b * BW + 1] : 0.0;
                }
            }
            load_b(x, b);  // zero padded past n
            mma(a, x);
        }
    };
    if (S.aligned)
        run(std::true_type{});
    else
        run(std::false_type{});

    // Add the W partial tiles in wave order; epilogue r = B - A x_new.
#pragma unroll
    for (int q = 0; q < TPW; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[(((wave * TPW + q) * NT + t) * 4 + v) * 64 + lane] = acc[q][t][v];
    __syncthreads();
    double Q = 0.0;
    uint64_t M = 0;
    for (int e = tid; e < TPW * NT * 256; e += W * 64) {
        const int l = e & 63, v = (e >> 6) & 3, qt = e >> 8;
        const int q = qt / NT, t = qt - q * NT;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) s += red[(((w * TPW + q) * NT + t) * 4 + v) * 64 + l];
        const int64_t i = r0 + 16 * q + (l >> 4) + 4 * v;
        const int c = t * 16 + (l & 15);
        if (i < n && c < S.ldx) {
            double r = 0.0;
            if (c < S.k) {
                r = S.B[i * S.ldb + c] - s;
                Q += r * r;
                const uint64_t mb = dbits(fabs(r));
                M = mb > M ? mb : M;
            }
            S.r64[i * S.ldx + c] = r;
            S.rlo[i * S.ldx + c] = (float)r;
        }
    }
    Q = wsum(Q);
    M = wmax(M);
    if (lane == 0) {
        red_q[wave] = Q;
        red_m[wave] = M;
    }
    __syncthreads();
    RState* T = &p.st[si];
    if (tid == 0) {
        double q = 0.0;
        uint64_t m = 0;
        for (int w = 0; w < W; ++w) {
            q += red_q[w];
            m = red_m[w] > m ? red_m[w] : m;
        }
        __hip_atomic_store(&p.parts[job], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&T->rmax_bits, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t tk =
            __hip_atomic_fetch_add(&T->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (tk == (uint32_t)(S.njobs - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    // Last job of the system: add the job sums in job order and decide.
    __threadfence();
    double sum = 0.0;
    for (int j = tid; j < S.njobs; j += W * 64)
        sum += __hip_atomic_load(&p.parts[S.job0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sum = wsum(sum);
    __syncthreads();
    if (lane == 0) red_q[wave] = sum;
    __syncthreads();
    if (tid == 0) {
        double q = 0.0;
        for (int w = 0; w < W; ++w) q += red_q[w];
        const double rn = sqrt(q);
        const double rel = S.bnorm > 0.0 ? rn / S.bnorm : rn;
        uint32_t stop = STOP_RUNNING;
        if (!isfinite(rel))
            stop = STOP_DIVERGED;
        else if (q == 0.0 || rel < S.rel)
            stop = STOP_CONVERGED;
        __hip_atomic_store(&T->rel_bits, dbits(rel), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&T->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// 16-row tiles per wave for a system of n rows: the most that still gives
// every compute unit a job (more tiles per job share each B operand load).
int resid_tiles(int32_t kt, int64_t n, int num_cus) {
    int t = kt <= 16 ? max_tiles_per_wave<16>() : max_tiles_per_wave<32>();
    while (t > 1 && (n + 16 * t - 1) / (16 * t) < num_cus) t /= 2;
    return t;
}

hipError_t launch_resid_prep(int32_t kt, const RSys* sys, RState* st, int32_t count,
                             int64_t max_xld, hipStream_t s) {
    int64_t bx = (max_xld + 255) / 256;
    if (bx > 64) bx = 64;
    if (bx < 1) bx = 1;
    if (kt == 16)
        hipLaunchKernelGGL((k_resid_prep<16>), dim3((unsigned)bx, count), dim3(256), 0, s, sys, st);
    else if (kt == 32)
        hipLaunchKernelGGL((k_resid_prep<32>), dim3((unsigned)bx, count), dim3(256), 0, s, sys, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// 16-byte word copy between any two device-visible buffers (descriptor
// uploads from and outcome read-backs to pinned host memory).
__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
        return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)(bytes / 16);
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 64) blocks = 64;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src,
                       (uint4*)dst, n16);
    return hipGetLastError();
}

template <int KT, int TPW>
static hipError_t launch_resid_t(const RArgs& a, int32_t jobs, hipStream_t s) {
    hipLaunchKernelGGL((k_resid<KT, kRW, TPW, kRU>), dim3(jobs), dim3(kRW * 64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_resid(int32_t kt, int32_t tiles, const RArgs& a, int32_t jobs, hipStream_t s) {
    if (jobs < 1) return hipSuccess;
    if (kt == 16) {
        if (tiles == 4) return launch_resid_t<16, 4>(a, jobs, s);
        if (tiles == 2) return launch_resid_t<16, 2>(a, jobs, s);
        if (tiles == 1) return launch_resid_t<16, 1>(a, jobs, s);
    } else if (kt == 32) {
        if (tiles == 2) return launch_resid_t<32, 2>(a, jobs, s);
        if (tiles == 1) return launch_resid_t<32, 1>(a, jobs, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace jac
