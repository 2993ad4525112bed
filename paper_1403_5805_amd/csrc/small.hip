// Small systems in one launch (gfx950).
//
// The plain path runs one kernel launch per sweep, which for a system of a
// few MiB costs more than the sweep itself.  This kernel runs every sweep of
// one system (k <= 2 right-hand sides, iterate small enough for LDS) in a
// single launch of G co-resident workgroups, G <= the CU count:
//   * each sweep stages x^(r-1) (n x kp values, row-major) in LDS;
//   * wave w of workgroup g takes rows w + 4 g, w + 4 g + 4 G, ...; the 64
//     lanes split a row's columns in 16-byte pieces (one vector load when the
//     rows are 16-byte aligned), skip the diagonal, multiply with the staged
//     iterate and add the lanes' sums in a fixed butterfly order; lane c < k
//     applies the component update of sec. 2, x_new = (b - s) / a_ii, and
//     folds |x_new - x_old| into the workgroup's distance statistics;
//   * the statistics go to the same three rotating slots as the vector
//     kernel's (atomic maxima on the bit patterns, and one partial sum of
//     squares per workgroup, added in workgroup order for the Euclidean
//     distance, so the decision is deterministic);
//   * one grid barrier per sweep (one release arrival, one acquire), after
//     which every workgroup takes the same stop decision from the slot:
//     NaN/Inf distance -> diverged, distance < tol -> converged, or the sweep
//     cap; workgroup 0 records it in the control block the host reads.
// Validation (k_setup, before this launch) leaves Ctl::stop = STOP_INVALID on
// bad input; the kernel then runs no sweep.  Every barrier wait has a
// wall-clock bound: a wait that cannot end sets STOP_TIMEOUT, which the host
// reports as an internal error.
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace jac {

namespace {

typedef uint16_t bf16_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

template <typename T>
__device__ __forceinline__ T lane_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint64_t lane_max(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t w = (uint64_t)__shfl_xor((long long)v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// A values of one 16-byte piece, widened to the accumulation type.
template <typename TA, typename TX>
struct Piece;
template <>
struct Piece<double, double> {
    static constexpr int V = 2;
    __device__ static void load(const double* p, bool vec, int64_t c0, int64_t n, double* a) {
        if (vec) {
            const u32x4 u = *(const u32x4*)p;
            a[0] = __hiloint2double((int)u.y, (int)u.x);
            a[1] = __hiloint2double((int)u.w, (int)u.z);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) a[e] = c0 + e < n ? p[e] : 0.0;
        }
    }
};
template <>
struct Piece<float, float> {
    static constexpr int V = 4;
    __device__ static void load(const float* p, bool vec, int64_t c0, int64_t n, float* a) {
        if (vec) {
            const u32x4 u = *(const u32x4*)p;
            a[0] = __uint_as_float(u.x);
            a[1] = __uint_as_float(u.y);
            a[2] = __uint_as_float(u.z);
            a[3] = __uint_as_float(u.w);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) a[e] = c0 + e < n ? p[e] : 0.0f;
        }
    }
};
template <>
struct Piece<bf16_t, float> {
    static constexpr int V = 8;
    __device__ static void load(const bf16_t* p, bool vec, int64_t c0, int64_t n, float* a) {
        if (vec) {
            const u32x4 u = *(const u32x4*)p;
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[2 * e] = __uint_as_float(w[e] << 16);
                a[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e)
                a[e] = c0 + e < n ? __uint_as_float((uint32_t)p[e] << 16) : 0.0f;
        }
    }
};

}  // namespace

// LDS for the staged iterate: 32 KiB.
constexpr int kSmallLdsBytes = 32 * 1024;

template <typename TA, typename TX, int KP, bool ALIGNED>
__global__ __launch_bounds__(256) void k_small(SmallArgs a) {
    constexpr int W = 4;
    constexpr int V = Piece<TA, TX>::V;
    __shared__ TX xs[kSmallLdsBytes / sizeof(TX)];
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ uint32_t s_go;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = (int)gridDim.x;
    const int64_t n = a.n;
    const int k = a.k;
    const TA* A = (const TA*)a.A;
    const TX* B = (const TX*)a.B;
    const TX* diag = (const TX*)a.diag;
    Ctl* ctl = a.ctl;
    if (tid == 0)
        s_go = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               STOP_RUNNING;
    __syncthreads();
    if (!s_go) return;  // invalid input: no sweep
    for (int r = 1; r <= a.cap; ++r) {
        const TX* xin = (const TX*)((r & 1) ? a.buf0 : a.buf1);
        TX* xout = (TX*)((r & 1) ? a.buf1 : a.buf0);
        for (int64_t e = tid; e < n * KP; e += W * 64) xs[e] = xin[e];
        __syncthreads();
        uint64_t dmax = 0, xmax = 0;
        double sq = 0.0;
        for (int64_t i = wave + (int64_t)W * blockIdx.x; i < n; i += (int64_t)W * G) {
            TX s[KP];
#pragma unroll
            for (int c = 0; c < KP; ++c) s[c] = TX(0);
            const TA* row = A + i * a.lda;
            for (int64_t c0 = (int64_t)lane * V; c0 < n; c0 += 64 * V) {
                TX v[V];
                Piece<TA, TX>::load(row + c0, ALIGNED && c0 + V <= n, c0, n, v);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int64_t j = c0 + e;
                    const TX av = j == i ? TX(0) : v[e];  // the diagonal term is skipped
                    if (j < n) {
#pragma unroll
                        for (int c = 0; c < KP; ++c) s[c] += av * xs[j * KP + c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < KP; ++c) s[c] = lane_sum(s[c]);
            if (lane < k) {
                TX sc = s[0];
#pragma unroll
                for (int c = 1; c < KP; ++c) sc = lane == c ? s[c] : sc;
                const TX xo = xs[i * KP + lane];
                const TX xn = (B[i * a.ldb + lane] - sc) / diag[i];
                xout[i * KP + lane] = xn;
                const double dd = fabs((double)xn - (double)xo);
                const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                dmax = db > dmax ? db : dmax;
                xmax = mb > xmax ? mb : xmax;
                sq += dd * dd;
            }
        }
        dmax = lane_max(dmax);
        xmax = lane_max(xmax);
        sq = lane_sum(sq);
        if (lane == 0) {
            red_d[wave] = dmax;
            red_m[wave] = xmax;
            red_s[wave] = sq;
        }
        __syncthreads();
        Slot* sl = &a.slots[r % 3];
        if (tid == 0) {
            uint64_t D = 0, M = 0;
            double Q = 0.0;
            for (int w = 0; w < W; ++w) {
                D = red_d[w] > D ? red_d[w] : D;
                M = red_m[w] > M ? red_m[w] : M;
                Q += red_s[w];
            }
            __hip_atomic_fetch_max(&sl->dmax_bits, D, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&sl->xmax_bits, M, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.parts[(size_t)(r % 3) * kMaxParts + blockIdx.x], Q,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (blockIdx.x == 0) {
                // slot (r + 1) % 3 was last read in the decision of sweep
                // r - 2, which every workgroup took before barrier r - 1
                Slot* nx = &a.slots[(r + 1) % 3];
                __hip_atomic_store(&nx->dmax_bits, (uint64_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&nx->xmax_bits, (uint64_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            // grid barrier r: every workgroup's statistics and rows of x^(r)
            // precede its arrival (release); the waits end with an acquire
            __hip_atomic_fetch_add(&ctl->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = (uint32_t)G * (uint32_t)r;
            const uint64_t t0 = wall_clock64();
            bool ok = true;
            while (__hip_atomic_load(&ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                   target) {
                __builtin_amdgcn_s_sleep(1);
                if ((int64_t)(wall_clock64() - t0) > a.spin_limit) {
                    ok = false;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            uint32_t st = STOP_RUNNING;
            const double dm = bitsd(__hip_atomic_load(&sl->dmax_bits, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
            const double xm = bitsd(__hip_atomic_load(&sl->xmax_bits, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
            double delta = dm;
            if (a.norm == 1) {
                double S = 0.0;  // workgroup order
                for (int g = 0; g < G; ++g)
                    S += __hip_atomic_load(&a.parts[(size_t)(r % 3) * kMaxParts + g],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                delta = sqrt(S);
            }
            if (!isfinite(delta))
                st = STOP_DIVERGED;
            else if (delta < a.tol)
                st = STOP_CONVERGED;
            if (!ok) st = STOP_TIMEOUT;
            if (blockIdx.x == 0) {
                __hip_atomic_store(&ctl->last_delta_bits, dbits(delta), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->last_xmax_bits, dbits(xm), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->sweeps_done, r, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            if (st != STOP_RUNNING && (blockIdx.x == 0 || st == STOP_TIMEOUT)) {
                __hip_atomic_store(&ctl->stop_sweep, r, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->stop, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_go = st == STOP_RUNNING;
        }
        __syncthreads();
        if (!s_go) break;
    }
}

template <typename TA, typename TX, int KP>
static const void* small_fn(bool aligned) {
    return aligned ? (const void*)k_small<TA, TX, KP, true> : (const void*)k_small<TA, TX, KP, false>;
}

int64_t small_max_rows(int32_t a_dtype, int32_t kp) {
    const int64_t sx = a_dtype == 0 ? 8 : 4;
    return kSmallLdsBytes / (sx * kp);
}

hipError_t launch_small(int32_t a_dtype, const SmallArgs& a, int kp, bool aligned, int grid,
                        hipStream_t s) {
    const void* fn = nullptr;
    if (a_dtype == 0)
        fn = kp == 1 ? small_fn<double, double, 1>(aligned) : small_fn<double, double, 2>(aligned);
    else if (a_dtype == 1)
        fn = kp == 1 ? small_fn<float, float, 1>(aligned) : small_fn<float, float, 2>(aligned);
    else if (a_dtype == 2)
        fn = kp == 1 ? small_fn<bf16_t, float, 1>(aligned) : small_fn<bf16_t, float, 2>(aligned);
    if (!fn || (kp != 1 && kp != 2) || a.n > small_max_rows(a_dtype, kp) || grid < 1 ||
        grid > kMaxParts)
        return hipErrorInvalidValue;
    SmallArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

}  // namespace jac
