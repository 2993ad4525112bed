// Dense Jacobi sweep kernels for gfx950 (CDNA4, wave64).
//
// One launch performs one sweep of the component equation of sec. 2 of the
// paper,  x_i^(k) = (beta_i - sum_{j != i} alpha_ij x_j^(k-1)) / alpha_ii,
// for every row i and right-hand side c, fused with the distance
// max|x^(k) - x^(k-1)| (or its Euclidean form, sec. 3.1) and the stop test of
// the serial pseudocode (sec. 2, step (b)).
//
// Design (HBM-bound streaming, 0.5 flop/byte for one right-hand side in FP32):
//   * A is streamed once per sweep with 16-byte non-temporal loads; every wave
//     owns R consecutive rows and its 64 lanes cover 64*VEC consecutive columns
//     per load, so each row segment is a contiguous 1 KiB read.
//   * x^(k-1) is staged in LDS (the whole vector when it fits, else column
//     chunks) and read back with 16-byte LDS loads; the R rows of a wave share
//     each x read.
//   * Each lane keeps R*K accumulators; a butterfly shuffle reduces them across
//     the wave in a fixed order (results do not depend on timing).
//   * The epilogue divides by alpha_ii (IEEE division), writes x^(k) into the
//     other ping-pong buffer and folds |x^(k) - x^(k-1)| into a per-workgroup
//     maximum, reduced across the grid with one atomic max per workgroup on
//     the bit pattern of the non-negative double (a NaN compares above +Inf,
//     so a NaN distance is never lost).
//   * Stop decision without a grid-wide wait: sweep launch `seq` publishes its
//     distance atomics into reduction slot seq % 3 and ends.  Every workgroup
//     of the next launch reads that slot as it starts and takes the same stop
//     decision (workgroup 0 records it, with the device stop flag, and clears
//     slot (seq + 1) % 3 for the launch after); the last launch of a host group
//     is decided by a one-workgroup decide kernel.  Launches queued after a
//     stop return at once, so the host only reads the flag every few sweeps.
//   * The same kernel, in residual mode, computes r = b - A x in FP64 (no
//     diagonal mask, no division) for iterative refinement, with the update
//     x += d fused into the staging of x.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "internal.h"
#include "round.h"

namespace jac {

typedef uint16_t bf16_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Elem;
template <>
struct Elem<double> {
    static constexpr int vec = 2;
};
template <>
struct Elem<float> {
    static constexpr int vec = 4;
};
template <>
struct Elem<bf16_t> {
    static constexpr int vec = 8;
};

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

template <typename TA, typename TX>
__device__ __forceinline__ TX widen(TA a);
template <>
__device__ __forceinline__ double widen<double, double>(double a) {
    return a;
}
template <>
__device__ __forceinline__ float widen<float, float>(float a) {
    return a;
}
template <>
__device__ __forceinline__ float widen<bf16_t, float>(bf16_t a) {
    return bf16_bits_to_f32(a);
}

// Unpack one 16-byte vector of TA into VEC values of TX.
template <typename TA, typename TX>
__device__ __forceinline__ void unpack16(const u32x4& v, TX* out);
template <>
__device__ __forceinline__ void unpack16<double, double>(const u32x4& v, double* out) {
    out[0] = __hiloint2double((int)v.y, (int)v.x);
    out[1] = __hiloint2double((int)v.w, (int)v.z);
}
template <>
__device__ __forceinline__ void unpack16<float, float>(const u32x4& v, float* out) {
    out[0] = __uint_as_float(v.x);
    out[1] = __uint_as_float(v.y);
    out[2] = __uint_as_float(v.z);
    out[3] = __uint_as_float(v.w);
}
template <>
__device__ __forceinline__ void unpack16<bf16_t, float>(const u32x4& v, float* out) {
    out[0] = bf16_bits_to_f32(v.x & 0xffffu);
    out[1] = bf16_bits_to_f32(v.x >> 16);
    out[2] = bf16_bits_to_f32(v.y & 0xffffu);
    out[3] = bf16_bits_to_f32(v.y >> 16);
    out[4] = bf16_bits_to_f32(v.z & 0xffffu);
    out[5] = bf16_bits_to_f32(v.z >> 16);
    out[6] = bf16_bits_to_f32(v.w & 0xffffu);
    out[7] = bf16_bits_to_f32(v.w >> 16);
}

__device__ __forceinline__ double tx_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tx_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        uint64_t o = __shfl_xor(v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t ld_stop(const Ctl* c) {
    return __hip_atomic_load(&c->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Control-block initialisation.  full = 1 also clears the validation fields.
__global__ void k_init_ctl(Ctl* ctl, Slot* slots, int full) {
    if (threadIdx.x == 0) {
        ctl->stop = STOP_RUNNING;
        ctl->stop_sweep = 0;
        ctl->sweeps_done = 0;
        ctl->last_delta_bits = dbits(-1.0);
        ctl->last_xmax_bits = 0;
        ctl->bar = 0;
        if (full) {
            ctl->bad_zero = INT64_MAX;
            ctl->bad_nonfinite = INT64_MAX;
            ctl->bad_rhs = INT64_MAX;
            ctl->setup_ticket = 0;
        }
        for (int s = 0; s < 3; ++s) {
            slots[s].dmax_bits = 0;
            slots[s].xmax_bits = 0;
            slots[s].ticket = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Setup (validation + initial iterate).  Gathers alpha_ii into diag, records
// the first row with a zero or non-finite diagonal (sec. 2: the method fails
// when alpha_ii = 0) and the first row with a non-finite B or X0 entry, copies
// X0 (or zeros) into the iterate buffer w0 (leading dim kpad, padding columns
// zero) and clears w1.  The last workgroup raises STOP_INVALID if anything was
// wrong, so no sweep runs and X is never written.
template <typename TA, typename TX>
__global__ void k_setup(const TA* __restrict__ A, int64_t lda, const TX* __restrict__ B,
                        int64_t ldb, const TX* __restrict__ X0, int64_t ldx0, int64_t n, int k,
                        int kpad, TX* __restrict__ diag, TX* __restrict__ w0, TX* __restrict__ w1,
                        Ctl* ctl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const TX d = widen<TA, TX>(A[i * lda + i]);
        diag[i] = d;
        if (d == (TX)0)
            __hip_atomic_fetch_min(&ctl->bad_zero, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!isfinite(d))
            __hip_atomic_fetch_min(&ctl->bad_nonfinite, i, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        bool bad = false;
        for (int c = 0; c < kpad; ++c) {
            TX x0 = (TX)0;
            if (c < k) {
                if (X0) x0 = X0[i * ldx0 + c];
                const TX b = B[i * ldb + c];
                if (!isfinite(b) || !isfinite(x0)) bad = true;
            }
            w0[i * kpad + c] = x0;
            w1[i * kpad + c] = (TX)0;
        }
        if (bad)
            __hip_atomic_fetch_min(&ctl->bad_rhs, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&ctl->setup_ticket, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (t == gridDim.x - 1) {
            __threadfence();
            const int64_t bz = __hip_atomic_load(&ctl->bad_zero, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const int64_t bn = __hip_atomic_load(&ctl->bad_nonfinite, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const int64_t br = __hip_atomic_load(&ctl->bad_rhs, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (bz != INT64_MAX || bn != INT64_MAX || br != INT64_MAX)
                __hip_atomic_store(&ctl->stop, (uint32_t)STOP_INVALID, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Stage columns [c0, c0 + cl) of the iterate (leading dim KT, contiguous rows)
// into LDS.  In residual mode (dlt != null) the staged value is x + d, the
// refinement update, formed in FP64.
template <typename TX, int KT, int NT>
__device__ __forceinline__ void stage_x(TX* __restrict__ xs, const TX* __restrict__ xin,
                                        const float* __restrict__ dlt, int64_t c0, int64_t cl) {
    const int tid = threadIdx.x;
    const int64_t elems = cl * KT;
    const TX* src = xin + c0 * KT;
    if (dlt == nullptr) {
        const int64_t nvec = (elems * (int64_t)sizeof(TX)) / 16;
        const u32x4* s16 = reinterpret_cast<const u32x4*>(src);
        u32x4* d16 = reinterpret_cast<u32x4*>(xs);
        for (int64_t base = 0; base < nvec; base += (int64_t)NT * 8) {
            u32x4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t idx = base + (int64_t)u * NT + tid;
                if (idx < nvec) v[u] = s16[idx];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t idx = base + (int64_t)u * NT + tid;
                if (idx < nvec) d16[idx] = v[u];
            }
        }
        for (int64_t e = nvec * 16 / (int64_t)sizeof(TX) + tid; e < elems; e += NT) xs[e] = src[e];
    } else {
        const float* ds = dlt + c0 * KT;
        for (int64_t base = 0; base < elems; base += (int64_t)NT * 4) {
            TX v[4];
            float w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t idx = base + (int64_t)u * NT + tid;
                if (idx < elems) {
                    v[u] = src[idx];
                    w[u] = ds[idx];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t idx = base + (int64_t)u * NT + tid;
                if (idx < elems) xs[idx] = v[u] + (TX)w[u];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Accumulate sum_j alpha_ij x_j over columns [c0, c0 + cl) for the R rows
// g..g+R-1 (the same rows for every wave of the workgroup).  The columns are
// cut into span blocks of 64*VEC; wave w takes blocks w, w+W, w+2W, ... so the
// W waves together read W consecutive 1 KiB pieces of each row per load.
// MODE 0 skips j == i (sec. 2: the sum runs over j != i); MODE 1 (residual)
// keeps every term.
//
// MODE 1 with lo_dtype != 0 also stores every A value it loads, rounded to
// FP32 (lo_dtype 1) or BF16 (2), at the same place of alo (leading dimension
// ld_lo): a pass reads each value once, so the copy is written exactly once.
template <typename TA, typename TX, int KT, int R, int U, int W, int MODE>
__device__ __forceinline__ void accumulate(TX (&acc)[R][KT], const TA* __restrict__ A, int64_t lda,
                                           int64_t n, int64_t g, int64_t c0, int64_t cl,
                                           const TX* __restrict__ xs, int lane, int wave,
                                           bool aligned, void* alo = nullptr, int64_t ld_lo = 0,
                                           int lo_dtype = 0) {
    constexpr int VEC = Elem<TA>::vec;
    constexpr int SPAN = 64 * VEC;
    constexpr int NV = (VEC * KT * (int)sizeof(TX)) / 16;  // LDS 16-byte reads per load
    static_assert(NV >= 1, "x slice must be at least 16 bytes");
    const TA* rowp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = (g + r < n) ? (g + r) : (n - 1);
        rowp[r] = A + i * lda + c0 + lane * VEC;
    }
    const int64_t nsb = aligned ? (cl / SPAN) : 0;           // full span blocks
    const int64_t nj = nsb > wave ? (nsb - wave + W - 1) / W : 0;  // blocks of this wave
    const int64_t dlo = g - c0;  // diagonal of row g+r sits at relative column dlo+r

    auto consume = [&](const u32x4 (&v)[R], int64_t sb) {
        const int64_t cbase = sb * SPAN;
        TX xv[VEC * KT];
        {
            u32x4 t[NV];
            const u32x4* src = reinterpret_cast<const u32x4*>(xs + (cbase + (int64_t)lane * VEC) * KT);
#pragma unroll
            for (int q = 0; q < NV; ++q) t[q] = src[q];
            __builtin_memcpy(xv, t, sizeof(xv));
        }
        TX a[R][VEC];
#pragma unroll
        for (int r = 0; r < R; ++r) unpack16<TA, TX>(v[r], a[r]);
        if constexpr (MODE == 1 && sizeof(TA) == 8 && VEC == 2) {
            if (lo_dtype != 0) {
                const int64_t col = c0 + cbase + (int64_t)lane * VEC;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (g + r >= n) continue;
                    const double d0 = __longlong_as_double(
                        (long long)(((uint64_t)v[r].y << 32) | v[r].x));
                    const double d1 = __longlong_as_double(
                        (long long)(((uint64_t)v[r].w << 32) | v[r].z));
                    if (lo_dtype == 2) {
                        const uint32_t w = (uint32_t)f64_to_bf16_rne(d0) |
                                           ((uint32_t)f64_to_bf16_rne(d1) << 16);
                        *reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(alo) +
                                                     (g + r) * ld_lo + col) = w;
                    } else {
                        *reinterpret_cast<float2*>(static_cast<float*>(alo) + (g + r) * ld_lo +
                                                   col) = make_float2((float)d0, (float)d1);
                    }
                }
            }
        }
        if (MODE == 0 && cbase < dlo + R && dlo < cbase + SPAN) {
            const int64_t col = cbase + (int64_t)lane * VEC;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (col + e == dlo + r) a[r][e] = (TX)0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int c = 0; c < KT; ++c) acc[r][c] = tx_fma(a[r][e], xv[e * KT + c], acc[r][c]);
    };

    int64_t j = 0;
    for (; j + U <= nj; j += U) {
        u32x4 v[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t sb = wave + (j + u) * W;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[u][r] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rowp[r] + sb * SPAN));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) consume(v[u], wave + (j + u) * W);
    }
    for (; j < nj; ++j) {
        u32x4 v[R];
        const int64_t sb = wave + j * W;
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rowp[r] + sb * SPAN));
        consume(v, sb);
    }
    // Ragged tail (and whole rows when they are not 16-byte aligned).
    for (int64_t col = nsb * SPAN + wave * 64 + lane; col < cl; col += W * 64) {
        TX xv[KT];
#pragma unroll
        for (int c = 0; c < KT; ++c) xv[c] = xs[col * KT + c];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const TA raw = rowp[r][col - lane * VEC];
            if constexpr (MODE == 1 && sizeof(TA) == 8) {
                if (lo_dtype != 0 && g + r < n) {
                    const double d = (double)raw;
                    if (lo_dtype == 2)
                        static_cast<uint16_t*>(alo)[(g + r) * ld_lo + c0 + col] =
                            f64_to_bf16_rne(d);
                    else
                        static_cast<float*>(alo)[(g + r) * ld_lo + c0 + col] = (float)d;
                }
            }
            TX a = widen<TA, TX>(raw);
            if (MODE == 0 && col == dlo + r) a = (TX)0;
#pragma unroll
            for (int c = 0; c < KT; ++c) acc[r][c] = tx_fma(a, xv[c], acc[r][c]);
        }
    }
}

// ---------------------------------------------------------------------------
// Distance statistics and the stop decision.
//
// A launch only publishes: each workgroup folds its lanes' maxima (and sum
// of squares) and adds them to the launch's slot with relaxed atomics
// (slot = launch number % 3), nothing waits for a reply.  The decision for a
// launch is taken by every workgroup of the next launch of the phase as it
// starts (the launch boundary orders it after all of the previous launch's
// atomics), or, after the last launch of a group, by k_decide.  All
// workgroups read the same values and decide alike; workgroup 0 records the
// outcome in the control block.  All threads of the workgroup must call.
template <int W>
__device__ __forceinline__ void finish_launch(const SweepArgs& p, uint64_t dmax, uint64_t xmax,
                                              double sq) {
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool need_sum = (p.norm == 1) || (p.test == TEST_RESID);
    dmax = wave_max_u64(dmax);
    xmax = wave_max_u64(xmax);
    sq = wave_sum(sq);
    if (lane == 0) {
        red_d[wave] = dmax;
        red_m[wave] = xmax;
        red_s[wave] = sq;
    }
    __syncthreads();
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    Slot* sl = &p.slots[p.seq % 3];
    double* parts = p.parts + (size_t)(p.seq % 3) * kMaxParts;
    if (tid == 0) {
        uint64_t D = 0, M = 0;
        double S = 0.0;
        for (int w = 0; w < W; ++w) {
            D = red_d[w] > D ? red_d[w] : D;
            M = red_m[w] > M ? red_m[w] : M;
            S += red_s[w];
        }
        if (need_sum)
            __hip_atomic_store(&parts[bid], S, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&sl->dmax_bits, D, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&sl->xmax_bits, M, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The stop decision for launch `seq` of the phase (logical sweep `sweep`),
// whose `total` workgroups have all finished.  Returns STOP_* (the same in
// every thread); when `record`, thread 0 writes the outcome into the control
// block.  All threads of the workgroup must call.
//
// The control block's stop flag is read with the slot: when the phase has
// already stopped, that flag is returned and nothing is recorded.
template <int W>
__device__ __forceinline__ uint32_t decide(const SweepArgs& p, int32_t seq, int32_t sweep,
                                           int total, bool record) {
    __shared__ double red_s[W];
    __shared__ uint32_t s_flag;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool need_sum = (p.norm == 1) || (p.test == TEST_RESID);
    const Slot* sl = &p.slots[seq % 3];
    const double* parts = p.parts + (size_t)(seq % 3) * kMaxParts;
    double S = 0.0;
    if (need_sum) {
        // fixed order: thread t adds parts t, t + W*64, ...; then lanes and
        // waves in order
        for (int b = tid; b < total; b += W * 64)
            S += __hip_atomic_load(&parts[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S = wave_sum(S);
        if (lane == 0) red_s[wave] = S;
        __syncthreads();
        S = 0.0;
        for (int w = 0; w < W; ++w) S += red_s[w];
    }
    if (tid == 0) {
        const uint32_t prior = ld_stop(p.ctl);
        const double dm = bitsd(__hip_atomic_load(&sl->dmax_bits, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
        const double xm = bitsd(__hip_atomic_load(&sl->xmax_bits, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
        if (prior != STOP_RUNNING) record = false;
        uint32_t st = STOP_RUNNING;
        double delta;
        if (p.test == TEST_RESID) {
            const double rn = sqrt(S);
            delta = p.bnorm > 0.0 ? rn / p.bnorm : rn;
            if (!isfinite(delta))
                st = STOP_DIVERGED;
            else if (S == 0.0 || delta < p.rel)
                st = STOP_CONVERGED;
        } else {
            delta = (p.norm == 1) ? sqrt(S) : dm;
            if (!isfinite(delta))
                st = STOP_DIVERGED;
            else if (p.test == TEST_ABS ? (delta < p.tol) : (delta <= p.rel * xm))
                st = STOP_CONVERGED;
        }
        if (record) {
            Ctl* c = p.ctl;
            __hip_atomic_store(&c->last_delta_bits, dbits(delta), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c->last_xmax_bits, dbits(xm), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c->sweeps_done, sweep, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (st != STOP_RUNNING) {
                __hip_atomic_store(&c->stop_sweep, sweep, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&c->stop, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        s_flag = prior != STOP_RUNNING ? prior : st;
    }
    __syncthreads();
    return s_flag;
}

// Decision for the last launch of a group (launch p.seq, logical sweep
// p.sweep) when no later launch of the phase takes it; a no-op once the
// phase has stopped.  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_decide(SweepArgs p, int total) {
    decide<4>(p, p.seq, p.sweep, total, true);
}

// ---------------------------------------------------------------------------
// Rows per pass: the cross-wave partial sums of one pass live in LDS.
template <typename TX, int KT, int W, int R>
constexpr int pass_rows() {
    int p = 8192 / (KT * W * (int)sizeof(TX));
    if (p > 64) p = 64;
    if (p < R) p = R;
    return (p / R) * R;
}

// The sweep (MODE 0) / residual (MODE 1) kernel.
//   grid.x : contiguous blocks of rows_per_wg rows (grid-stride if fewer WGs)
//   grid.y : column groups of KT right-hand sides (k > 32 only)
// Every wave of a workgroup works on the same R rows at a time (on different
// columns); each wave folds its lane sums into its own LDS slot per row, and
// after each pass of P rows one thread per (row, column) adds the W slots in
// wave order and applies the epilogue.
template <typename TA, typename TX, int KT, int R, int U, int W, int MODE>
__global__ __launch_bounds__(W * 64) void k_sweep(SweepArgs p) {
    constexpr int P = pass_rows<TX, KT, W, R>();
    __shared__ TX red[P * KT * W];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    TX* xs = reinterpret_cast<TX*>(lds_raw);
    if (p.seq == 1 && ld_stop(p.ctl) != STOP_RUNNING) return;
    if (p.seq > 1) {
        // the previous launch's outcome: every workgroup decides alike
        const bool first = blockIdx.x == 0 && blockIdx.y == 0;
        if (decide<W>(p, p.seq - 1, p.sweep - 1, gridDim.x * gridDim.y, first) !=
            STOP_RUNNING)
            return;
        // launch seq + 1 will publish into slot (seq + 1) % 3, last used by
        // launch seq - 2, whose decision launch seq - 1 took
        if (first && threadIdx.x == 0) {
            Slot* o = &p.slots[(p.seq + 1) % 3];
            __hip_atomic_store(&o->dmax_bits, (uint64_t)0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&o->xmax_bits, (uint64_t)0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = p.n;
    const int kp = p.kpad;
    const int cb = blockIdx.y * KT;
    const int kc = (p.k - cb) < KT ? (p.k - cb) : KT;
    const TA* A = reinterpret_cast<const TA*>(p.A);
    const TX* B = reinterpret_cast<const TX*>(p.B);
    const TX* xin = reinterpret_cast<const TX*>(p.xin);
    const TX* diag = reinterpret_cast<const TX*>(p.diag);
    const bool aligned = p.aligned != 0;
    const TX* xsrc = xin + cb;
    const float* dsrc = (MODE == 1 && p.dlt) ? (p.dlt + cb) : nullptr;
    const bool contiguous = (kp == KT);
    // the residual pass writes the reduced copy of A once (first column group)
    const bool cvt = MODE == 1 && p.alo != nullptr && blockIdx.y == 0;

    auto stage = [&](int64_t c0, int64_t cl) {
        if (contiguous) {
            stage_x<TX, KT, W * 64>(xs, xsrc, dsrc, c0, cl);
        } else {
            for (int64_t e = tid; e < cl * KT; e += W * 64) {
                const int64_t j = c0 + e / KT;
                const int c = (int)(e % KT);
                TX v = (TX)0;
                if (c < kc) {
                    v = xsrc[j * kp + c];
                    if (dsrc) v += (TX)dsrc[j * kp + c];
                }
                xs[e] = v;
            }
        }
    };

    uint64_t dmax = 0, xmax = 0;
    double sq = 0.0;
    const bool single = p.chunk >= n;
    if (single) {
        stage(0, n);
        __syncthreads();
    }
    const int64_t rpw = p.rows_per_wg;
    for (int64_t rb = (int64_t)blockIdx.x * rpw; rb < n; rb += (int64_t)gridDim.x * rpw) {
        const int64_t rbe = (rb + rpw) < n ? (rb + rpw) : n;
        for (int64_t ps = rb; ps < rbe; ps += P) {
            const int64_t pe = (ps + P) < rbe ? (ps + P) : rbe;
            for (int t = lane; t < P * KT; t += 64) red[t * W + wave] = (TX)0;
            for (int64_t c0 = 0; c0 < n; c0 += p.chunk) {
                const int64_t cl = (n - c0) < p.chunk ? (n - c0) : p.chunk;
                if (!single) {
                    __syncthreads();
                    stage(c0, cl);
                    __syncthreads();
                }
                for (int64_t g = ps; g < pe; g += R) {
                    TX acc[R][KT];
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int c = 0; c < KT; ++c) acc[r][c] = (TX)0;
                    accumulate<TA, TX, KT, R, U, W, MODE>(acc, A, p.lda, n, g, c0, cl, xs, lane,
                                                          wave, aligned, p.alo, p.ld_lo,
                                                          cvt ? p.lo_dtype : 0);
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int c = 0; c < KT; ++c) {
                            const TX v = wave_sum(acc[r][c]);
                            if (lane == 0 && g + r < pe)
                                red[((g - ps + r) * KT + c) * W + wave] += v;
                        }
                }
            }
            __syncthreads();
            for (int t = tid; t < (int)(pe - ps) * KT; t += W * 64) {
                const int64_t i = ps + t / KT;
                const int c = t % KT;
                if (c >= kc) continue;
                TX s = (TX)0;
#pragma unroll
                for (int w = 0; w < W; ++w) s += red[t * W + w];
                if (MODE == 0) {
                    const TX b = B[i * p.ldb + cb + c];
                    const TX xn = (b - s) / diag[i];
                    const TX xo = xin[i * kp + cb + c];
                    reinterpret_cast<TX*>(p.xout)[i * kp + cb + c] = xn;
                    const double dd = fabs((double)xn - (double)xo);
                    const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                    dmax = db > dmax ? db : dmax;
                    xmax = mb > xmax ? mb : xmax;
                    sq += dd * dd;
                } else {
                    // residual r = b - A x with x already updated in LDS; the
                    // owner of row i also stores the updated x.
                    const double rr = (double)B[i * p.ldb + cb + c] - (double)s;
                    p.r64[i * kp + cb + c] = rr;
                    p.rlo[i * kp + cb + c] = (float)rr;
                    double xnew = (double)xin[i * kp + cb + c];
                    if (dsrc) xnew += (double)dsrc[i * kp + c];
                    reinterpret_cast<double*>(p.xout)[i * kp + cb + c] = xnew;
                    sq += rr * rr;
                    const uint64_t mb = dbits(fabs(rr));
                    dmax = mb > dmax ? mb : dmax;
                }
            }
            __syncthreads();
        }
    }
    finish_launch<W>(p, dmax, xmax, sq);
}


// alpha_ii of a reduced-precision copy of A, widened to float.
template <typename TA>
__global__ void k_gather_diag(const TA* __restrict__ A, int64_t lda, int64_t n, float* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = widen<TA, float>(A[i * lda + i]);
}

// ||B||_2 over all n*k entries, one workgroup, fixed summation order.
__global__ void k_bnorm(const double* __restrict__ B, int64_t ldb, int64_t n, int k, double* out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        for (int c = 0; c < k; ++c) {
            const double v = B[i * ldb + c];
            s += v * v;
        }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) S += red[w];
        *out = sqrt(S);
    }
}

template <typename T>
__global__ void k_copy_rows(const T* __restrict__ src, int64_t lds, T* __restrict__ dst,
                            int64_t ldd, int64_t n, int k) {
    // one thread per (row, column); k is small, rows spread over the grid
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        for (int c = 0; c < k; ++c) dst[i * ldd + c] = src ? src[i * lds + c] : (T)0;
}

// ---------------------------------------------------------------------------
// Launchers.

static int blocks_for(int64_t work, int threads, int cap) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_init_ctl(Ctl* ctl, Slot* slots, int full, hipStream_t s) {
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, ctl, slots, full);
    return hipGetLastError();
}

hipError_t launch_setup(int32_t a_dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                        const void* X0, int64_t ldx0, int64_t n, int32_t k, int32_t kpad,
                        void* diag, void* w0, void* w1, Ctl* ctl, hipStream_t s) {
    const int threads = 256;
    const int blocks = blocks_for(n, threads, 1024);
    switch (a_dtype) {
        case 0:
            hipLaunchKernelGGL((k_setup<double, double>), dim3(blocks), dim3(threads), 0, s,
                               (const double*)A, lda, (const double*)B, ldb, (const double*)X0,
                               ldx0, n, k, kpad, (double*)diag, (double*)w0, (double*)w1, ctl);
            break;
        case 1:
            hipLaunchKernelGGL((k_setup<float, float>), dim3(blocks), dim3(threads), 0, s,
                               (const float*)A, lda, (const float*)B, ldb, (const float*)X0, ldx0,
                               n, k, kpad, (float*)diag, (float*)w0, (float*)w1, ctl);
            break;
        case 2:
            hipLaunchKernelGGL((k_setup<bf16_t, float>), dim3(blocks), dim3(threads), 0, s,
                               (const bf16_t*)A, lda, (const float*)B, ldb, (const float*)X0,
                               ldx0, n, k, kpad, (float*)diag, (float*)w0, (float*)w1, ctl);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TA, typename TX, int KT, int R, int U, int W, int MODE>
static hipError_t launch_one(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s) {
    if constexpr (R * KT * sizeof(TX) > 256 || (R > 1 && R * KT * sizeof(TX) > 128) || R * U > 8) {
        return hipErrorInvalidValue;
    } else {
        const int gy = (a.k + KT - 1) / KT;
        const size_t lds = (size_t)a.chunk * KT * sizeof(TX);
        auto kern = k_sweep<TA, TX, KT, R, U, W, MODE>;
        static size_t lds_allowed = 0;  // dynamic LDS already enabled for this kernel
        if (lds > 32768 && lds > lds_allowed) {
            hipError_t e = hipFuncSetAttribute((const void*)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            lds_allowed = lds;
        }
        hipLaunchKernelGGL(kern, dim3(cfg.grid, gy), dim3(W * 64), lds, s, a);
        return hipGetLastError();
    }
}

template <typename TA, typename TX, int KT, int W, int MODE>
static hipError_t launch_ru(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s) {
    const int r = cfg.rows, u = cfg.unroll;
    if (r == 1 && u == 2) return launch_one<TA, TX, KT, 1, 2, W, MODE>(a, cfg, s);
    if (r == 1 && u == 4) return launch_one<TA, TX, KT, 1, 4, W, MODE>(a, cfg, s);
    if (r == 2 && u == 2) return launch_one<TA, TX, KT, 2, 2, W, MODE>(a, cfg, s);
    if (r == 2 && u == 4) return launch_one<TA, TX, KT, 2, 4, W, MODE>(a, cfg, s);
    if (r == 4 && u == 2) return launch_one<TA, TX, KT, 4, 2, W, MODE>(a, cfg, s);
    return hipErrorInvalidValue;
}

template <typename TA, typename TX, int KT, int MODE>
static hipError_t launch_rw(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s) {
    if (cfg.waves == 8) return launch_ru<TA, TX, KT, 8, MODE>(a, cfg, s);
    if (cfg.waves == 4) return launch_ru<TA, TX, KT, 4, MODE>(a, cfg, s);
    if constexpr (KT <= 2) {
        if (cfg.waves == 16) return launch_ru<TA, TX, KT, 16, MODE>(a, cfg, s);
    }
    return hipErrorInvalidValue;
}

static int kt_for(int k) {
    int kt = 1;
    while (kt < k && kt < 32) kt <<= 1;
    return kt;
}

template <typename TA, typename TX, int MODE>
static hipError_t launch_kt(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s) {
    switch (kt_for(a.k)) {
        case 1: return launch_rw<TA, TX, 1, MODE>(a, cfg, s);
        case 2: return launch_rw<TA, TX, 2, MODE>(a, cfg, s);
        case 4: return launch_rw<TA, TX, 4, MODE>(a, cfg, s);
        case 8: return launch_rw<TA, TX, 8, MODE>(a, cfg, s);
        case 16: return launch_rw<TA, TX, 16, MODE>(a, cfg, s);
        case 32: return launch_rw<TA, TX, 32, MODE>(a, cfg, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(int32_t a_dtype, const SweepArgs& a, const LaunchCfg& cfg,
                        hipStream_t s) {
    SweepArgs p = a;
    p.chunk = cfg.chunk;
    p.rows_per_wg = cfg.rows_per_wg;
    switch (a_dtype) {
        case 0: return launch_kt<double, double, 0>(p, cfg, s);
        case 1: return launch_kt<float, float, 0>(p, cfg, s);
        case 2: return launch_kt<bf16_t, float, 0>(p, cfg, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_decide(const SweepArgs& a, int total, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, a, total);
    return hipGetLastError();
}

hipError_t launch_residual(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s) {
    SweepArgs p = a;
    p.chunk = cfg.chunk;
    p.rows_per_wg = cfg.rows_per_wg;
    return launch_kt<double, double, 1>(p, cfg, s);
}

hipError_t launch_gather_diag(int32_t a_dtype, const void* A, int64_t lda, int64_t n,
                              void* out, hipStream_t s) {
    const int blocks = blocks_for(n, 256, 1024);
    if (a_dtype == 1)
        hipLaunchKernelGGL((k_gather_diag<float>), dim3(blocks), dim3(256), 0, s, (const float*)A,
                           lda, n, (float*)out);
    else if (a_dtype == 2)
        hipLaunchKernelGGL((k_gather_diag<bf16_t>), dim3(blocks), dim3(256), 0, s,
                           (const bf16_t*)A, lda, n, (float*)out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bnorm(const double* B, int64_t ldb, int64_t n, int32_t k, double* out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_bnorm, dim3(1), dim3(1024), 0, s, B, ldb, n, k, out);
    return hipGetLastError();
}

hipError_t launch_copy_rows(int32_t elem_bytes, const void* src, int64_t lds, void* dst,
                            int64_t ldd, int64_t n, int32_t k, hipStream_t s) {
    const int threads = 256;
    const int blocks = blocks_for(n, threads, 4096);
    if (elem_bytes == 8)
        hipLaunchKernelGGL((k_copy_rows<double>), dim3(blocks), dim3(threads), 0, s,
                           (const double*)src, lds, (double*)dst, ldd, n, k);
    else if (elem_bytes == 4)
        hipLaunchKernelGGL((k_copy_rows<float>), dim3(blocks), dim3(threads), 0, s,
                           (const float*)src, lds, (float*)dst, ldd, n, k);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_zero_rows(int32_t elem_bytes, void* dst, int64_t ldd, int64_t n, int32_t k,
                            hipStream_t s) {
    return launch_copy_rows(elem_bytes, nullptr, 0, dst, ldd, n, k, s);
}

// ---------------------------------------------------------------------------
// Launch-shape heuristics.

// Dynamic LDS for the x chunk: 64 KiB when a workgroup may use more than
// 72 KiB of LDS (gfx950), else what is left after the static pass buffer.
static int64_t lds_chunk_bytes() {
    static int64_t cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        cached = v >= 73728 ? 65536 : (v - 8192 > 16384 ? v - 8192 : 16384);
    }
    return cached;
}

static int64_t span_of(int32_t a_dtype) { return a_dtype == 0 ? 128 : (a_dtype == 1 ? 256 : 512); }

LaunchCfg default_cfg(int32_t a_dtype, int64_t n, int32_t k, int num_cus) {
    LaunchCfg c;
    const int kt = kt_for(k);
    const int sx = (a_dtype == 0) ? 8 : 4;
    const int64_t span = span_of(a_dtype);
    // Waves share each row: a short row cannot keep 8 waves busy.
    c.waves = (n >= 8 * span) ? 8 : 4;
    // Rows accumulated together and loads in flight per row.
    if (kt * sx <= 8) {
        c.rows = 2;
        c.unroll = 2;
    } else if (kt * sx <= 32) {
        c.rows = 2;
        c.unroll = 2;
    } else {
        c.rows = 1;
        c.unroll = 2;
    }
    // x chunk staged in LDS (whole x when it fits in 64 KiB; the pass
    // reduction adds at most 8 KiB of static LDS, so two workgroups fit a CU).
    int64_t cap = lds_chunk_bytes() / ((int64_t)kt * sx);
    cap = (cap / span) * span;
    if (cap < span) cap = span;
    c.chunk = n <= cap ? n : cap;
    // One workgroup per CU, each owning a contiguous block of rows (measured
    // best for streaming: fewer concurrent row streams per HBM channel); small
    // systems get at least one row group per workgroup.
    int64_t gcap = (int64_t)num_cus;
    const int64_t gy = (k + 31) / 32;
    if (gcap * gy > kMaxParts) gcap = kMaxParts / gy;
    int64_t g = (n + c.rows - 1) / c.rows;
    if (g > gcap) g = gcap;
    if (g < 1) g = 1;
    // Tuning override "waves,rows,unroll,wg_per_cu" (JACOBI_SWEEP_CFG).
    if (const char* env = getenv("JACOBI_SWEEP_CFG")) {
        int w = 0, r = 0, u = 0, wpc = 0;
        if (sscanf(env, "%d,%d,%d,%d", &w, &r, &u, &wpc) == 4 &&
            (w == 4 || w == 8 || (w == 16 && kt <= 2)) &&
            (r == 1 || r == 2 || r == 4) && (u == 2 || u == 4) && wpc >= 1) {
            c.waves = w;
            c.rows = r;
            c.unroll = u;
            gcap = (int64_t)num_cus * wpc;
            if (gcap * gy > kMaxParts) gcap = kMaxParts / gy;
            g = (n + c.rows - 1) / c.rows;
            if (g > gcap) g = gcap;
        }
    }
    // At least four rows per workgroup: below that a small system's sweep is
    // a latency chain (the decision read, staging, a few rows and the distance
    // atomics) that more workgroups only lengthen (n = 512 FP64, measured with
    // an earlier last-workgroup decision: 19.6 us per sweep with 128
    // workgroups, 24.4 with 256).
    g = std::max<int64_t>(1, std::min<int64_t>(g, (n + 3) / 4));
    c.rows_per_wg = (n + g - 1) / g;
    c.grid = (int)((n + c.rows_per_wg - 1) / c.rows_per_wg);
    return c;
}

LaunchCfg residual_cfg(int64_t n, int32_t k, int num_cus) { return default_cfg(0, n, k, num_cus); }

size_t sweep_lds_bytes(int32_t a_dtype, int32_t k, const LaunchCfg& cfg) {
    const int sx = (a_dtype == 0) ? 8 : 4;
    return (size_t)cfg.chunk * kt_for(k) * sx;
}

}  // namespace jac
