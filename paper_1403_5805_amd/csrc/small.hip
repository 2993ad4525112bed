// Small systems in one launch (gfx950).
//
// The plain path runs one kernel launch per sweep, which for a system of a
// few MiB costs more than the sweep itself.  Two kernels here run every
// sweep of one system (k <= 2 right-hand sides) in a single launch of G
// co-resident workgroups, G <= the CU count: k_small_reg (further below),
// which holds each wave's rows of A in registers and can also take the
// set-up's and the copy-out's place, and k_small, its fallback for rows too
// long for the registers, described here (iterate small enough for LDS):
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

// Exchange of a value between lanes for step S of the wave reductions:
// S = 0, 1 swap within groups of four lanes (DPP quad_perm, lane ^ 1 and
// lane ^ 2), S = 2 the other group of four of a half row (DPP
// row_half_mirror), S = 3 the other half of a row of 16 (DPP row_mirror),
// S = 4, 5 lane ^ 16 and lane ^ 32 (lane permutes).  After steps 0 and 1
// every lane of a group of four holds the same value (and after step 2 every
// lane of a half row), so the mirrors pair the same partial results as
// lane ^ 4 and lane ^ 8 would; the DPP steps are register moves instead of
// the LDS-routed permutes.
template <int S>
__device__ __forceinline__ uint32_t xchg32(uint32_t v) {
    // DPP controls: quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E,
    // row_half_mirror = 0x141, row_mirror = 0x140
    constexpr int kCtrl[4] = {0xB1, 0x4E, 0x141, 0x140};
    if constexpr (S < 4)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl[S], 0xf, 0xf, false);
    else
        return (uint32_t)__shfl_xor((int)v, S == 4 ? 16 : 32, 64);
}
template <int S>
__device__ __forceinline__ float xchg(float v) {
    return __uint_as_float(xchg32<S>(__float_as_uint(v)));
}
template <int S>
__device__ __forceinline__ double xchg(double v) {
    const uint32_t lo = xchg32<S>((uint32_t)__double2loint(v));
    const uint32_t hi = xchg32<S>((uint32_t)__double2hiint(v));
    return __hiloint2double((int)hi, (int)lo);
}
template <int S>
__device__ __forceinline__ uint64_t xchg(uint64_t v) {
    const uint32_t lo = xchg32<S>((uint32_t)v);
    const uint32_t hi = xchg32<S>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Sum over the wave in the fixed step order above: every lane ends with the
// same bits (each step adds two equal-by-symmetry partners, a + b = b + a).
template <typename T>
__device__ __forceinline__ T lane_sum(T v) {
    v += xchg<0>(v);
    v += xchg<1>(v);
    v += xchg<2>(v);
    v += xchg<3>(v);
    v += xchg<4>(v);
    v += xchg<5>(v);
    return v;
}
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t lane_max(uint64_t v) {
    v = umax64(v, xchg<0>(v));
    v = umax64(v, xchg<1>(v));
    v = umax64(v, xchg<2>(v));
    v = umax64(v, xchg<3>(v));
    v = umax64(v, xchg<4>(v));
    v = umax64(v, xchg<5>(v));
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

// ---------------------------------------------------------------------------
// Register-resident variant.  A does not change between sweeps and wave w of
// workgroup g always owns the same rows (w + W g + W G t, W waves per
// workgroup), so the wave loads its rows once, before the first sweep, into
// registers: one 16-byte piece of a row per lane and step of 64 pieces (NP
// steps cover the row), the diagonal entry stored as zero, and b_i, a_ii
// beside them.  Every sweep then reads only the iterate, straight into
// registers (a lane needs the same NP pieces of x for every row it holds),
// all loads issued before the first use: one memory round trip per sweep
// instead of one per piece.  The products, their order, the lane sums, the
// update and the distance the stop test uses are those of k_small, so both
// kernels give the same bits (only the statistics no decision needs are
// left out).

// Rows per wave that the register budget holds beside the iterate's pieces,
// 0 if not one row fits: 192 32-bit registers per lane and at most 8 rows
// with W = 4 waves per workgroup (one wave per SIMD, up to 512 registers),
// 96 and at most 4 rows with W = 8 (two waves per SIMD, up to 256 each).
template <typename TA, typename TX, int KP, int NP, int W>
constexpr int small_reg_rpw() {
    constexpr int V = Piece<TA, TX>::V;
    constexpr int xv = NP * V * KP * (int)sizeof(TX) / 4;
    constexpr int r = ((W == 4 ? 192 : 96) - xv) / (4 * NP);
    constexpr int cap = W == 4 ? 8 : 4;
    return r < 1 ? 0 : (r > cap ? cap : r);
}

template <typename TA, typename TX>
__device__ __forceinline__ u32x4 pack_piece(const TX* v);
template <>
__device__ __forceinline__ u32x4 pack_piece<double, double>(const double* v) {
    u32x4 u;
    u.x = (uint32_t)__double2loint(v[0]);
    u.y = (uint32_t)__double2hiint(v[0]);
    u.z = (uint32_t)__double2loint(v[1]);
    u.w = (uint32_t)__double2hiint(v[1]);
    return u;
}
template <>
__device__ __forceinline__ u32x4 pack_piece<float, float>(const float* v) {
    u32x4 u;
    u.x = __float_as_uint(v[0]);
    u.y = __float_as_uint(v[1]);
    u.z = __float_as_uint(v[2]);
    u.w = __float_as_uint(v[3]);
    return u;
}
template <>
__device__ __forceinline__ u32x4 pack_piece<bf16_t, float>(const float* v) {
    // every value came from a BF16 (low 16 bits zero): the pair packs exactly
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        w[e] = (__float_as_uint(v[2 * e]) >> 16) | (__float_as_uint(v[2 * e + 1]) & 0xffff0000u);
    u32x4 u;
    u.x = w[0];
    u.y = w[1];
    u.z = w[2];
    u.w = w[3];
    return u;
}

// The inverse of pack_piece: the V values of a held piece, widened.
template <typename TA, typename TX>
__device__ __forceinline__ void unpack_piece(const u32x4 u, TX* v);
template <>
__device__ __forceinline__ void unpack_piece<double, double>(const u32x4 u, double* v) {
    v[0] = __hiloint2double((int)u.y, (int)u.x);
    v[1] = __hiloint2double((int)u.w, (int)u.z);
}
template <>
__device__ __forceinline__ void unpack_piece<float, float>(const u32x4 u, float* v) {
    v[0] = __uint_as_float(u.x);
    v[1] = __uint_as_float(u.y);
    v[2] = __uint_as_float(u.z);
    v[3] = __uint_as_float(u.w);
}
template <>
__device__ __forceinline__ void unpack_piece<bf16_t, float>(const u32x4 u, float* v) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[2 * e] = __uint_as_float(w[e] << 16);
        v[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
    }
}

template <typename TA, typename TX, int KP, int NP, int W>
__global__ __launch_bounds__(W * 64) void k_small_reg(SmallArgs a) {
    constexpr int V = Piece<TA, TX>::V;
    constexpr int RPW = small_reg_rpw<TA, TX, KP, NP, W>();
    __shared__ uint64_t red_d[W];
    __shared__ double red_s[W];
    __shared__ uint32_t s_go, s_stop;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = (int)gridDim.x;
    const int64_t n = a.n;
    const int k = a.k;
    const TA* A = (const TA*)a.A;
    const TX* B = (const TX*)a.B;
    const TX* diag = (const TX*)a.diag;
    Ctl* ctl = a.ctl;
    // a separate set-up kernel may have found invalid input (fused: the
    // checks are this launch's, and the stop word is left as it was)
    if (!a.fused) {
        if (tid == 0)
            s_go = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                   STOP_RUNNING;
        __syncthreads();
        if (!s_go) return;  // invalid input: no sweep
    }
    // Fused launches may follow one another on the same control block without
    // a k_init_ctl in between: the barrier count then starts at bar_base and
    // sweep r uses slot (slot_base + r) % 3, which the host sets so that the
    // first sweep's slot is one the previous launch left clear.
    const int sb = a.slot_base;
    // one atomic word gathers the distance's maximum on small grids; larger
    // ones, where those atomics queue, store one word per workgroup
    const bool atomic_max = G <= a.atomic_max_grid;
    const int64_t i0 = wave + (int64_t)W * blockIdx.x;
    const int64_t di = (int64_t)W * G;
    // rows t < nr of this wave; the host guarantees nr <= RPW
    const int nr = i0 < n ? (int)((n - i0 + di - 1) / di) : 0;
    u32x4 ar[RPW][NP];
    TX br[RPW], dr[RPW];
    // every 16-byte piece of the wave's rows in flight at once
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
        const int64_t i = i0 + di * t;
        br[t] = TX(0);
        dr[t] = TX(1);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int64_t c0 = ((int64_t)lane + 64 * p) * V;
            ar[t][p] = u32x4{0u, 0u, 0u, 0u};
            if (t < nr && a.aligned != 0 && c0 + V <= n)
                ar[t][p] = *(const u32x4*)(A + i * a.lda + c0);
        }
        if (t < nr && lane < k) {
            br[t] = B[i * a.ldb + lane];
            if (a.fused) {
                TX v1[V];  // a_ii, widened as the set-up kernel does
                Piece<TA, TX>::load(A + i * a.lda + i, false, 0, 1, v1);
                dr[t] = v1[0];
            } else {
                dr[t] = diag[i];
            }
        }
    }
    // the piece that ends a row, and every piece of rows that are not
    // 16-byte aligned, element by element
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
        const int64_t i = i0 + di * t;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int64_t c0 = ((int64_t)lane + 64 * p) * V;
            if (t < nr && c0 < n && !(a.aligned != 0 && c0 + V <= n)) {
                TX v[V];
                Piece<TA, TX>::load(A + i * a.lda + c0, false, c0, n, v);
                ar[t][p] = pack_piece<TA, TX>(v);
            }
        }
    }
    // the diagonal term is skipped: held as zero (one lane and piece per row)
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
        const int64_t i = i0 + di * t;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int64_t c0 = ((int64_t)lane + 64 * p) * V;
            if (t < nr && c0 <= i && i < c0 + V) {
                TX v[V];
                unpack_piece<TA, TX>(ar[t][p], v);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (c0 + e == i) v[e] = TX(0);
                ar[t][p] = pack_piece<TA, TX>(v);
            }
        }
    }
    // Iteration r loads x^(r-1), then takes the stop decision of sweep r - 1
    // (its statistics were final at barrier r - 1, whose acquire thread 0
    // has taken), so that their two loads overlap; iteration cap + 1 only
    // decides.  A stop discards the loads of x.  Fused (set-up and copy-out
    // in this launch): sweep 1 reads x^(0) from X0 (or takes zero) and checks
    // the rows' a_ii, b and x^(0) as the set-up kernel does; the decision of
    // sweep 1 sees the outcome of every workgroup's checks (they precede
    // barrier 1) and stops with STOP_INVALID before anything is written to X;
    // the final decision has each wave write its rows of X from registers.
    TX xl[RPW];  // the rows' components of the wave's last sweep (lanes c < k)
#pragma unroll
    for (int t = 0; t < RPW; ++t) xl[t] = TX(0);
    int64_t bad_z = INT64_MAX, bad_n = INT64_MAX, bad_r = INT64_MAX;  // thread 0
    for (int r = 1;; ++r) {
        const bool sweep = r <= a.cap;
        // fused sweep 1 reads x^(0) from X0 (n x k, packed), null for zero
        const TX* xin = (a.fused && r == 1) ? (const TX*)a.X0
                                            : (const TX*)((r & 1) ? a.buf0 : a.buf1);
        TX* xout = (TX*)((r & 1) ? a.buf1 : a.buf0);
        // the lane's pieces of x^(r-1) (columns (lane + 64 p) V ...) and, for
        // lanes c < k, the old value of its rows' component c
        TX xv[NP][V * KP];
        TX xo[RPW];
        if (sweep && xin == nullptr) {
            // fused, x^(0) = 0
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int e = 0; e < V * KP; ++e) xv[p][e] = TX(0);
#pragma unroll
            for (int t = 0; t < RPW; ++t) xo[t] = TX(0);
        } else if (sweep) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int64_t c0 = ((int64_t)lane + 64 * p) * V;
                if (c0 + V <= n) {
#pragma unroll
                    for (int q = 0; q < V * KP * (int)sizeof(TX) / 16; ++q) {
                        const u32x4 u = *(const u32x4*)(xin + c0 * KP + q * (16 / sizeof(TX)));
                        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
                        if constexpr (sizeof(TX) == 8) {
                            xv[p][2 * q] = __hiloint2double((int)w[1], (int)w[0]);
                            xv[p][2 * q + 1] = __hiloint2double((int)w[3], (int)w[2]);
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) xv[p][4 * q + e] = __uint_as_float(w[e]);
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < V * KP; ++e)
                        xv[p][e] = c0 + e / KP < n ? xin[c0 * KP + e] : TX(0);
                }
            }
#pragma unroll
            for (int t = 0; t < RPW; ++t)
                xo[t] = (t < nr && lane < k) ? xin[(i0 + di * t) * KP + lane] : TX(0);
        }
        if (r > 1 && wave == 0) {
            // the distance's maximum over the workgroups for sweep r - 1:
            // the slot every workgroup folded its own into with an atomic
            // maximum (grids of at most a.atomic_max_grid), else the
            // workgroups' own stored maxima (each stored before barrier
            // r - 1), four loads per lane in flight
            const uint64_t* dp =
                (const uint64_t*)(a.parts + (size_t)((sb + r - 1) % 3) * kMaxParts + kMaxParts / 2);
            uint64_t pd = 0;
            if (atomic_max && lane == 0)
                pd = __hip_atomic_load(&a.slots[(sb + r - 1) % 3].dmax_bits, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            for (int g0 = 0; !atomic_max && g0 < G; g0 += 256) {
                uint64_t v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int g = g0 + lane + 64 * j;
                    v[j] = g < G ? __hip_atomic_load(&dp[g], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : 0;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) pd = v[j] > pd ? v[j] : pd;
            }
            pd = lane_max(pd);
            if (lane == 0) {
                const int q = r - 1;
                uint32_t st = STOP_RUNNING;
                double delta = bitsd(pd);
                if (a.norm == 1) {
                    double S = 0.0;  // workgroup order
                    for (int g = 0; g < G; ++g)
                        S += __hip_atomic_load(&a.parts[(size_t)((sb + q) % 3) * kMaxParts + g],
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    delta = sqrt(S);
                }
                if (!isfinite(delta))
                    st = STOP_DIVERGED;
                else if (delta < a.tol)
                    st = STOP_CONVERGED;
                if (a.fused && q == 1) {
                    bad_z = __hip_atomic_load(&ctl->bad_zero, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    bad_n = __hip_atomic_load(&ctl->bad_nonfinite, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    bad_r = __hip_atomic_load(&ctl->bad_rhs, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    if (bad_z != INT64_MAX || bad_n != INT64_MAX || bad_r != INT64_MAX)
                        st = STOP_INVALID;
                }
                if (blockIdx.x == 0) {
                    __hip_atomic_store(&ctl->last_delta_bits, dbits(delta), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&ctl->sweeps_done, q, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    if (st != STOP_RUNNING) {
                        __hip_atomic_store(&ctl->stop_sweep, q, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&ctl->stop, st, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                    Ctl* h = a.hctl;
                    if (h != nullptr && (st != STOP_RUNNING || !sweep)) {
                        // the final control block, straight to the host
                        __hip_atomic_store(&h->stop, st, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->stop_sweep, st != STOP_RUNNING ? q : 0,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->sweeps_done, q, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->last_delta_bits, dbits(delta), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->bad_zero, bad_z, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->bad_nonfinite, bad_n, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&h->bad_rhs, bad_r, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                }
                s_go = st == STOP_RUNNING;
                s_stop = st;
            }
        }
        if (r > 1) {
            __syncthreads();
            if (!s_go || !sweep) {
                const uint32_t st = s_stop;
                if (a.fused && st != STOP_INVALID && st != STOP_TIMEOUT && lane < k) {
                    TX* X = (TX*)a.X;
#pragma unroll
                    for (int t = 0; t < RPW; ++t)
                        if (t < nr) X[(i0 + di * t) * a.ldx + lane] = xl[t];
                }
                break;
            }
        }
        if (!sweep) break;
        // the distance's statistics (max|x_new| is not needed on this path:
        // the plain solve reports no iterate size; the sum of squares only
        // for the Euclidean distance)
        uint64_t dmax = 0;
        double sq = 0.0;
        // Rows in chunks of up to four, all rows of a chunk at once (rows
        // t >= nr hold zeros): their products, lane sums and divisions
        // overlap; each row's own order of operations is unchanged.
        constexpr int CH = RPW < 4 ? RPW : 4;
#pragma unroll
        for (int t0 = 0; t0 < RPW; t0 += CH) {
            if (t0 >= nr) break;
            TX s[CH][KP];
#pragma unroll
            for (int j = 0; j < CH; ++j)
#pragma unroll
                for (int c = 0; c < KP; ++c) s[j][c] = TX(0);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int64_t c0 = ((int64_t)lane + 64 * p) * V;
                if (c0 < n) {
#pragma unroll
                    for (int j = 0; j < CH; ++j) {
                        if (t0 + j >= RPW) break;
                        TX v[V];
                        u32x4 u = ar[t0 + j][p];
                        // BF16: unpack in every sweep; hoisted out of the
                        // loop, the widened values would take twice the
                        // registers
                        if constexpr (sizeof(TA) == 2) asm volatile("" : "+v"(u));
                        unpack_piece<TA, TX>(u, v);
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            if (c0 + e < n) {
#pragma unroll
                                for (int c = 0; c < KP; ++c)
                                    s[j][c] += v[e] * xv[p][e * KP + c];
                            }
                        }
                    }
                }
            }
            // the steps of lane_sum, interleaved over the chunk's rows
#define JAC_SUM_STEP(S_)                                        \
    _Pragma("unroll") for (int j = 0; j < CH; ++j)              \
        _Pragma("unroll") for (int c = 0; c < KP; ++c) s[j][c] += xchg<S_>(s[j][c]);
            JAC_SUM_STEP(0)
            JAC_SUM_STEP(1)
            JAC_SUM_STEP(2)
            JAC_SUM_STEP(3)
            JAC_SUM_STEP(4)
            JAC_SUM_STEP(5)
#undef JAC_SUM_STEP
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int t = t0 + j;
                if (t >= RPW) break;
                const int64_t i = i0 + di * t;
                const bool live = t < nr && lane < k;
                TX sc = s[j][0];
#pragma unroll
                for (int c = 1; c < KP; ++c) sc = lane == c ? s[j][c] : sc;
                const TX xn = (br[t] - sc) / dr[t];
                xl[t] = xn;
                if (live) {
                    xout[i * KP + lane] = xn;
                    if (a.fused && r == 1) {
                        // the set-up kernel's checks of this row
                        if (lane == 0 && dr[t] == TX(0))
                            __hip_atomic_fetch_min(&ctl->bad_zero, i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        else if (lane == 0 && !isfinite(dr[t]))
                            __hip_atomic_fetch_min(&ctl->bad_nonfinite, i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        if (!isfinite(br[t]) || !isfinite(xo[t]))
                            __hip_atomic_fetch_min(&ctl->bad_rhs, i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                const double dd = fabs((double)xn - (double)xo[t]);
                const uint64_t db = live ? dbits(dd) : 0;
                dmax = db > dmax ? db : dmax;
                sq += live ? dd * dd : 0.0;  // + 0.0 leaves the sum's bits as they are
            }
        }
        dmax = lane_max(dmax);
        if (a.norm == 1) sq = lane_sum(sq);
        if (lane == 0) {
            red_d[wave] = dmax;
            red_s[wave] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            uint64_t D = 0;
            double Q = 0.0;
            for (int w = 0; w < W; ++w) {
                D = red_d[w] > D ? red_d[w] : D;
                Q += red_s[w];
            }
            // this workgroup's maximum and partial sum of sweep r: an atomic
            // maximum into slot (sb + r) % 3 on small grids (workgroup 0
            // clears the slot after next, last read in the decision of sweep
            // r - 2, which every workgroup took at the start of sweep r - 1,
            // before barrier r - 1), else a plain store of its own, like the
            // partial sum, in its words of parts slot (sb + r) % 3 (read after
            // barrier r, overwritten in sweep r + 3, after barrier r + 2)
            double* pr = a.parts + (size_t)((sb + r) % 3) * kMaxParts;
            if (atomic_max) {
                __hip_atomic_fetch_max(&a.slots[(sb + r) % 3].dmax_bits, D, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                if (blockIdx.x == 0)
                    __hip_atomic_store(&a.slots[(sb + r + 1) % 3].dmax_bits, (uint64_t)0,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store((uint64_t*)(pr + kMaxParts / 2) + blockIdx.x, D,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (a.norm == 1)
                __hip_atomic_store(pr + blockIdx.x, Q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // grid barrier r: every workgroup's statistics and rows of x^(r)
            // precede its arrival (release); the wait ends with an acquire
            __hip_atomic_fetch_add(&ctl->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = a.bar_base + (uint32_t)G * (uint32_t)r;
            const uint64_t t0 = wall_clock64();
            bool ok = true;
            while ((int32_t)(__hip_atomic_load(&ctl->bar, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) -
                             target) < 0) {
                __builtin_amdgcn_s_sleep(1);
                if ((int64_t)(wall_clock64() - t0) > a.spin_limit) {
                    ok = false;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (!ok) {
                __hip_atomic_store(&ctl->stop_sweep, r, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->stop, (uint32_t)STOP_TIMEOUT, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                if (a.hctl != nullptr)
                    __hip_atomic_store(&a.hctl->timeout, 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
            }
            s_go = ok;
        }
        __syncthreads();
        if (!s_go) break;
    }
}

template <typename TA, typename TX, int KP, int NP, int W>
static const void* small_reg_one(int* rpw) {
    constexpr int r = small_reg_rpw<TA, TX, KP, NP, W>();
    if constexpr (r == 0) {
        return nullptr;
    } else {
        *rpw = r;
        return (const void*)k_small_reg<TA, TX, KP, NP, W>;
    }
}

// Eight waves per workgroup only where a row takes at most eight pieces per
// lane (n <= 1024 FP64, 2048 FP32, 4096 BF16; where the 96-register budget
// holds too few rows for the grid, the host falls back to four waves).
template <typename TA, typename TX, int KP>
static const void* small_reg_fn(int np, int waves, int* rpw) {
    if (waves == 8) {
        switch (np) {
            case 1: return small_reg_one<TA, TX, KP, 1, 8>(rpw);
            case 2: return small_reg_one<TA, TX, KP, 2, 8>(rpw);
            case 4: return small_reg_one<TA, TX, KP, 4, 8>(rpw);
            case 8: return small_reg_one<TA, TX, KP, 8, 8>(rpw);
            default: return nullptr;
        }
    }
    if (waves != 4) return nullptr;
    switch (np) {
        case 1: return small_reg_one<TA, TX, KP, 1, 4>(rpw);
        case 2: return small_reg_one<TA, TX, KP, 2, 4>(rpw);
        case 4: return small_reg_one<TA, TX, KP, 4, 4>(rpw);
        case 8: return small_reg_one<TA, TX, KP, 8, 4>(rpw);
        case 12: return small_reg_one<TA, TX, KP, 12, 4>(rpw);
        case 16: return small_reg_one<TA, TX, KP, 16, 4>(rpw);
        default: return nullptr;
    }
}

static const void* small_reg_pick(int32_t a_dtype, int kp, int np, int waves, int* rpw) {
    if (a_dtype == 0)
        return kp == 1 ? small_reg_fn<double, double, 1>(np, waves, rpw)
                       : small_reg_fn<double, double, 2>(np, waves, rpw);
    if (a_dtype == 1)
        return kp == 1 ? small_reg_fn<float, float, 1>(np, waves, rpw)
                       : small_reg_fn<float, float, 2>(np, waves, rpw);
    if (a_dtype == 2)
        return kp == 1 ? small_reg_fn<bf16_t, float, 1>(np, waves, rpw)
                       : small_reg_fn<bf16_t, float, 2>(np, waves, rpw);
    return nullptr;
}

int small_reg_np(int32_t a_dtype, int64_t n) {
    // pieces per lane and row: 1, 2, 4, 8, 12 or 16 (12: rows of 9 to 12
    // steps fit the registers where 16 would not, e.g. FP32 n = 3072)
    const int64_t v = a_dtype == 0 ? 2 : (a_dtype == 1 ? 4 : 8);
    const int64_t need = (n + 64 * v - 1) / (64 * v);
    for (const int np : {1, 2, 4, 8, 12, 16})
        if (np >= need) return np;
    return 0;
}

int small_reg_rows_per_wave(int32_t a_dtype, int kp, int np, int waves) {
    int rpw = 0;
    return (kp == 1 || kp == 2) && small_reg_pick(a_dtype, kp, np, waves, &rpw) ? rpw : 0;
}

hipError_t launch_small_reg(int32_t a_dtype, const SmallArgs& a, int kp, int np, int waves,
                            int grid, hipStream_t s) {
    int rpw = 0;
    const void* fn =
        (kp == 1 || kp == 2) ? small_reg_pick(a_dtype, kp, np, waves, &rpw) : nullptr;
    const int64_t per = (int64_t)waves * grid;
    if (!fn || grid < 1 || grid > kMaxParts || small_reg_np(a_dtype, a.n) > np ||
        (a.n + per - 1) / per > rpw)
        return hipErrorInvalidValue;
    SmallArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * waves), args, 0, s);
}

template <typename TA, typename TX, int KP>
static const void* small_fn(bool aligned) {
    return aligned ? (const void*)k_small<TA, TX, KP, true>
                   : (const void*)k_small<TA, TX, KP, false>;
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
