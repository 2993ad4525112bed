// Persistent batched Jacobi sweeps on MFMA tiles (gfx950).
//
// One cooperative launch runs every sweep of many independent systems
// A_s X_s = B_s (each with k_s <= 32 right-hand sides).  The work of a sweep,
// S = (A - D) X followed by x_new = (b - s) / a_ii (the component equation of
// sec. 2 of the paper applied to every column), is a dense n x n by n x k
// contraction, done on v_mfma_f32_16x16x4_f32:
//   * a wave owns a 16-row tile; lane l loads row (l % 16) and 16 bytes of
//     consecutive columns (4 FP32 or 8 BF16 values) at column group l / 16,
//     so one 16-byte load per lane feeds 4 (FP32) or 8 (BF16) MFMA k-steps;
//   * the iterate chunk x[c0 .. c0+CH) is staged in LDS transposed (column c
//     of X is an LDS row), so the matching B operand of 4 k-steps is one
//     16-byte LDS read;
//   * the diagonal term is masked in the A operand (sum over j != i);
//   * the accumulator tile is the epilogue's input: division by a_ii, the
//     distance max|x_new - x_old| (or its Euclidean form) and the stop test.
// Systems are planned on the host: a large system is split over several
// workgroups that meet at a per-system barrier (atomic counter) after every
// sweep; small systems are owned whole by one workgroup (barrier = LDS
// barrier) and packed several per workgroup.  The launch is cooperative, so
// every workgroup is resident and the barrier waits always end; a wall-clock
// bound turns a stuck wait into an error instead of a hang.
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace jac {

typedef uint16_t bf16_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ float bf_to_f(uint32_t h) { return __uint_as_float(h << 16); }

template <typename TA>
__device__ __forceinline__ void unpack(const u32x4& v, float* a);
template <>
__device__ __forceinline__ void unpack<float>(const u32x4& v, float* a) {
    a[0] = __uint_as_float(v.x);
    a[1] = __uint_as_float(v.y);
    a[2] = __uint_as_float(v.z);
    a[3] = __uint_as_float(v.w);
}
template <>
__device__ __forceinline__ void unpack<bf16_t>(const u32x4& v, float* a) {
    a[0] = bf_to_f(v.x & 0xffffu);
    a[1] = bf_to_f(v.x >> 16);
    a[2] = bf_to_f(v.y & 0xffffu);
    a[3] = bf_to_f(v.y >> 16);
    a[4] = bf_to_f(v.z & 0xffffu);
    a[5] = bf_to_f(v.z >> 16);
    a[6] = bf_to_f(v.w & 0xffffu);
    a[7] = bf_to_f(v.w >> 16);
}

template <typename TA>
__device__ __forceinline__ float widen1(TA a);
template <>
__device__ __forceinline__ float widen1<float>(float a) {
    return a;
}
template <>
__device__ __forceinline__ float widen1<bf16_t>(bf16_t a) {
    return bf_to_f(a);
}

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

template <typename T>
__device__ __forceinline__ T wsum(T v) {
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

}  // namespace

// ---------------------------------------------------------------------------
// Setup: per system, gather alpha_ii, validate (zero / non-finite diagonal,
// non-finite B or X0), copy X0 (or zeros) into buf0 with zero padding
// columns, clear buf1.  grid = (row blocks, systems).
template <typename TA>
__global__ void k_batched_setup(const BSys* __restrict__ sys, BState* __restrict__ st, int kt) {
    const BSys S = sys[blockIdx.y];
    BState* T = &st[blockIdx.y];
    const TA* A = reinterpret_cast<const TA*>(S.A);
    float* diag = const_cast<float*>(S.diag);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += stride) {
        const float d = widen1<TA>(A[i * S.lda + i]);
        diag[i] = d;
        if (d == 0.0f)
            __hip_atomic_fetch_min(&T->bad_diag, 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!isfinite(d))
            __hip_atomic_fetch_min(&T->bad_diag, 2 * i + 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        bool bad = false;
        for (int c = 0; c < kt; ++c) {
            float x0 = 0.0f;
            if (c < S.k) {
                if (S.X0) x0 = S.X0[i * S.ldx + c];
                const float b = S.B[i * S.ldb + c];
                if (!isfinite(b) || !isfinite(x0)) bad = true;
            }
            S.buf0[i * kt + c] = x0;
            S.buf1[i * kt + c] = 0.0f;
        }
        if (bad)
            __hip_atomic_fetch_min(&T->bad_rhs, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// The persistent kernel.
template <typename TA, int KT, int W, int U>
__global__ __launch_bounds__(W * 64) void k_batched(BatchArgs p) {
    constexpr int VEC = 16 / (int)sizeof(TA);  // A values per 16-byte lane load
    constexpr int BW = 4 * VEC;                // columns of one A block (16 or 32)
    constexpr int NT = KT / 16;                // 16-column output tiles
    constexpr int NS = VEC / 4;                // 4-step MFMA groups per block
    extern __shared__ __attribute__((aligned(16))) float xsT[];  // [KT][CH + 4]
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ uint32_t s_flag;
    __shared__ double s_delta;

    const int CH = p.chunk, CHP = p.chunk + 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, li = lane & 15;

    for (int jb = p.job_off[blockIdx.x]; jb < p.job_off[blockIdx.x + 1]; ++jb) {
        const BJob job = p.jobs[jb];
        const BSys S = p.sys[job.sys];
        BState* st = &p.st[job.sys];
        if (__hip_atomic_load(&st->bad_diag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                INT64_MAX ||
            __hip_atomic_load(&st->bad_rhs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                INT64_MAX)
            continue;  // invalid input: no sweep runs, X untouched
        const TA* A = reinterpret_cast<const TA*>(S.A);
        const int64_t n = S.n;
        const int k = S.k;
        const bool split = S.nwg > 1;
        const float* xfinal = S.buf0;
        int32_t final_k = 0;
        uint32_t final_stop = STOP_RUNNING;
        double final_delta = -1.0;
        bool failed = false;

        for (int sweep = 1; sweep <= S.max_iter; ++sweep) {
            const float* xin = (sweep & 1) ? S.buf0 : S.buf1;
            float* xout = (sweep & 1) ? S.buf1 : S.buf0;
            uint64_t dmax = 0, xmax = 0;
            double sq = 0.0;
            for (int64_t pr = job.r0; pr < job.r1; pr += 16 * W) {
                const int64_t rt = pr + 16 * wave;
                const bool has_tile = rt < job.r1;
                const int64_t arow_i = (rt + li) < n ? (rt + li) : (n - 1);
                const TA* arow = A + arow_i * S.lda + VEC * grp;
                f32x4 acc[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
                for (int64_t c0 = 0; c0 < n; c0 += CH) {
                    const int cl = (int)((n - c0) < CH ? (n - c0) : CH);
                    const int clp = (cl + BW - 1) / BW * BW;
                    __syncthreads();
                    // stage x[c0 .. c0+cl) transposed, zero padded to clp
                    {
                        const float4* src = reinterpret_cast<const float4*>(xin + c0 * KT);
                        const int nv = cl * KT / 4;
                        for (int e4 = tid; e4 < nv; e4 += W * 64) {
                            const float4 v = src[e4];
                            const int j = (e4 * 4) / KT;
                            const int c = (e4 * 4) % KT;
                            xsT[(c + 0) * CHP + j] = v.x;
                            xsT[(c + 1) * CHP + j] = v.y;
                            xsT[(c + 2) * CHP + j] = v.z;
                            xsT[(c + 3) * CHP + j] = v.w;
                        }
                        for (int e = tid; e < (clp - cl) * KT; e += W * 64) {
                            const int j = cl + e / KT;
                            const int c = e % KT;
                            xsT[c * CHP + j] = 0.0f;
                        }
                    }
                    __syncthreads();
                    if (!has_tile) continue;
                    const int nb = clp / BW;
                    const int nbf = S.aligned ? (int)((n - c0 >= (int64_t)clp) ? nb : cl / BW) : 0;
                    const bool dchunk = (c0 < rt + 16) && (rt < c0 + cl);
                    auto mfma_block = [&](const float* a, int b) {
                        const int jrel = b * BW;
                        const int64_t colbase = c0 + jrel + VEC * grp;
                        float av[VEC];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) av[e] = a[e];
                        if (dchunk && c0 + jrel < rt + 16 && rt < c0 + jrel + BW) {
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                if (colbase + e == rt + li) av[e] = 0.0f;
                        }
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
#pragma unroll
                            for (int t = 0; t < NT; ++t) {
                                const f32x4 bv = *reinterpret_cast<const f32x4*>(
                                    xsT + (t * 16 + li) * CHP + jrel + VEC * grp + 4 * s);
#pragma unroll
                                for (int q = 0; q < 4; ++q)
                                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        av[4 * s + q], bv[q], acc[t], 0, 0, 0);
                            }
                        }
                    };
                    int b0 = 0;
                    for (; b0 + U <= nbf; b0 += U) {
                        u32x4 v[U];
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            v[u] = __builtin_nontemporal_load(
                                reinterpret_cast<const u32x4*>(arow + c0 + (b0 + u) * BW));
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            float a[VEC];
                            unpack<TA>(v[u], a);
                            mfma_block(a, b0 + u);
                        }
                    }
                    for (; b0 < nb; ++b0) {
                        float a[VEC];
                        if (b0 < nbf) {
                            const u32x4 v = __builtin_nontemporal_load(
                                reinterpret_cast<const u32x4*>(arow + c0 + b0 * BW));
                            unpack<TA>(v, a);
                        } else {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) {
                                const int64_t col = c0 + b0 * BW + VEC * grp + e;
                                a[e] = col < n ? widen1<TA>(arow[c0 + b0 * BW + e]) : 0.0f;
                            }
                        }
                        mfma_block(a, b0);
                    }
                }
                if (has_tile) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t i = rt + 4 * grp + v;
                            const int c = t * 16 + li;
                            if (i < job.r1 && c < k) {
                                const float s = acc[t][v];
                                const float xn = (S.B[i * S.ldb + c] - s) / S.diag[i];
                                const float xo = xin[i * KT + c];
                                xout[i * KT + c] = xn;
                                const double dd = fabs((double)xn - (double)xo);
                                const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                                dmax = db > dmax ? db : dmax;
                                xmax = mb > xmax ? mb : xmax;
                                sq += dd * dd;
                            }
                        }
                    }
                }
            }
            // ---- workgroup reduction of the distance statistics
            dmax = wmax(dmax);
            xmax = wmax(xmax);
            sq = wsum(sq);
            __syncthreads();
            if (lane == 0) {
                red_d[wave] = dmax;
                red_m[wave] = xmax;
                red_s[wave] = sq;
            }
            if (split) __threadfence();  // publish x_new before the system barrier
            __syncthreads();
            if (tid == 0) {
                uint64_t D = 0, M = 0;
                double Q = 0.0;
                for (int w = 0; w < W; ++w) {
                    D = red_d[w] > D ? red_d[w] : D;
                    M = red_m[w] > M ? red_m[w] : M;
                    Q += red_s[w];
                }
                uint32_t flag = STOP_RUNNING;
                if (split) {
                    const int slot = sweep % 3;
                    double* parts = p.parts + (size_t)(sweep & 1) * p.count * p.max_nwg +
                                    (size_t)job.sys * p.max_nwg;
                    if (S.norm == 1)
                        __hip_atomic_store(&parts[job.rank], Q, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_max(&st->dmax[slot], D, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_max(&st->xmax[slot], M, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (job.rank == 0) {
                        const int nxt = (sweep + 1) % 3;
                        __hip_atomic_store(&st->dmax[nxt], (uint64_t)0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->xmax[nxt], (uint64_t)0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                    __threadfence();
                    __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t target = (uint32_t)S.nwg * (uint32_t)sweep;
                    const uint64_t t0 = wall_clock64();
                    while (__hip_atomic_load(&st->counter, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT) < target) {
                        __builtin_amdgcn_s_sleep(2);
                        if ((int64_t)(wall_clock64() - t0) > p.spin_limit) {
                            __hip_atomic_store(&st->error, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            flag = 99;
                            break;
                        }
                    }
                    __threadfence();
                    D = __hip_atomic_load(&st->dmax[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    M = __hip_atomic_load(&st->xmax[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (S.norm == 1) {
                        Q = 0.0;
                        for (int r = 0; r < S.nwg; ++r)
                            Q += __hip_atomic_load(&parts[r], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                const double delta = (S.norm == 1) ? sqrt(Q) : bitsd(D);
                if (flag != 99) {
                    if (!isfinite(delta))
                        flag = STOP_DIVERGED;
                    else if (S.test == TEST_ABS ? (delta < S.tol) : (delta <= S.rel * bitsd(M)))
                        flag = STOP_CONVERGED;
                }
                s_flag = flag;
                s_delta = delta;
            }
            __syncthreads();
            if (split) __threadfence();  // acquire the other workgroups' x_new
            const uint32_t flag = s_flag;
            if (flag == 99) {
                failed = true;
                break;
            }
            if (flag != STOP_RUNNING || sweep == S.max_iter) {
                final_k = sweep;
                final_stop = flag;
                final_delta = s_delta;
                xfinal = xout;
                break;
            }
        }
        if (failed) continue;
        // Copy this workgroup's rows of the final iterate to the caller's X.
        // In the last sweep every element was written by the thread that
        // copies it here, so no further synchronisation is needed.
        if (final_k > 0) {
            for (int64_t pr = job.r0; pr < job.r1; pr += 16 * W) {
                const int64_t rt = pr + 16 * wave;
                if (rt >= job.r1) continue;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t i = rt + 4 * grp + v;
                        const int c = t * 16 + li;
                        if (i < job.r1 && c < k) S.X[i * S.ldx + c] = xfinal[i * KT + c];
                    }
            }
        } else {
            for (int64_t e = tid; e < (job.r1 - job.r0) * k; e += W * 64) {
                const int64_t i = job.r0 + e / k;
                const int c = (int)(e % k);
                S.X[i * S.ldx + c] = S.buf0[i * KT + c];
            }
        }
        if (tid == 0 && job.rank == 0) {
            __hip_atomic_store(&st->status, final_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->iterations, final_k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->final_delta, dbits(final_delta), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
constexpr int kBW = 8;   // waves per workgroup
constexpr int kBU = 2;   // A blocks in flight per wave

int batched_chunk(int32_t kt) { return kt <= 16 ? 1024 : 512; }

static size_t batched_lds(int32_t kt) { return (size_t)kt * (batched_chunk(kt) + 4) * sizeof(float); }

template <typename TA, int KT>
static const void* batched_fn() {
    return (const void*)k_batched<TA, KT, kBW, kBU>;
}

static const void* pick(int32_t a_dtype, int32_t kt) {
    if (a_dtype == 1) return kt <= 16 ? batched_fn<float, 16>() : batched_fn<float, 32>();
    if (a_dtype == 2) return kt <= 16 ? batched_fn<bf16_t, 16>() : batched_fn<bf16_t, 32>();
    return nullptr;
}

int batched_max_grid(int32_t a_dtype, int32_t kt, int num_cus) {
    const void* fn = pick(a_dtype, kt);
    if (!fn) return 0;
    const size_t lds = batched_lds(kt);
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBW * 64, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * num_cus;
}

hipError_t launch_batched_setup(int32_t a_dtype, int32_t kt, const BSys* sys, BState* st,
                                int32_t count, int64_t max_n, hipStream_t s) {
    int64_t bx = (max_n + 255) / 256;
    if (bx > 64) bx = 64;
    if (a_dtype == 1)
        hipLaunchKernelGGL((k_batched_setup<float>), dim3((unsigned)bx, count), dim3(256), 0, s,
                           sys, st, kt);
    else
        hipLaunchKernelGGL((k_batched_setup<bf16_t>), dim3((unsigned)bx, count), dim3(256), 0, s,
                           sys, st, kt);
    return hipGetLastError();
}

hipError_t launch_batched(int32_t a_dtype, int32_t kt, const BatchArgs& a, int grid,
                          hipStream_t s) {
    const void* fn = pick(a_dtype, kt);
    if (!fn) return hipErrorInvalidValue;
    const size_t lds = batched_lds(kt);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBW * 64), args, (unsigned)lds, s);
}

}  // namespace jac
