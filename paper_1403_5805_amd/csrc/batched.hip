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
//   * the iterate is kept transposed in global memory (column c of X is a
//     contiguous row of xld floats), so the matching B operand of 4 k-steps
//     is one 16-byte load that hits L1/L2 (X is small and every tile of the
//     system reads it); no LDS staging and no barrier inside a sweep: the
//     waves of a workgroup stream their 16-row tiles independently;
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

// x rows staged in LDS per chunk: 64 KiB of FP32 for the chunk.
template <int KT>
constexpr int batched_chunk_cols() {
    return KT <= 16 ? 1024 : 512;
}

// ---------------------------------------------------------------------------
// Setup: per system, gather alpha_ii, validate (zero / non-finite diagonal,
// non-finite B or X0), write X0 (or zeros) transposed into buf0 and clear
// buf1, padding included.  grid = (row blocks, systems).
template <typename TA>
__global__ void k_batched_setup(const BSys* __restrict__ sys, BState* __restrict__ st, int kt) {
    const BSys S = sys[blockIdx.y];
    BState* T = &st[blockIdx.y];
    const TA* A = reinterpret_cast<const TA*>(S.A);
    float* diag = const_cast<float*>(S.diag);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.xld; i += stride) {
        if (i >= S.n) {
            for (int c = 0; c < kt; ++c) {
                S.buf0[c * S.xld + i] = 0.0f;
                S.buf1[c * S.xld + i] = 0.0f;
            }
            continue;
        }
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
            S.buf0[c * S.xld + i] = x0;
            S.buf1[c * S.xld + i] = 0.0f;
        }
        if (bad)
            __hip_atomic_fetch_min(&T->bad_rhs, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// The persistent kernel.
//   W   waves per workgroup
//   TPW 16-row tiles per wave in one pass (they share every B operand read)
//   U   A blocks per pipeline stage (two stages in flight)
template <typename TA, int KT, int W, int TPW, int U>
__global__ __launch_bounds__(W * 64, 2) void k_batched(BatchArgs p) {
    constexpr int VEC = 16 / (int)sizeof(TA);  // A values per 16-byte lane load
    constexpr int BW = 4 * VEC;                // columns of one A block (16 or 32)
    constexpr int NT = KT / 16;                // 16-column output tiles
    constexpr int NS = VEC / 4;                // 4-step MFMA groups per block
    constexpr int CH = batched_chunk_cols<KT>();  // x rows staged per chunk
    constexpr int CHP = CH + 4;                // padded LDS row (bank spread)
    static_assert(CH % (BW * U) == 0, "a pipeline stage never straddles chunks");
    extern __shared__ __attribute__((aligned(16))) float xsT[];  // [KT][CHP]
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ uint32_t s_flag;
    __shared__ double s_delta;

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
        const int64_t xld = S.xld;
        const int k = S.k;
        const bool split = S.nwg > 1;
        const int64_t nb = (n + BW - 1) / BW;          // A blocks per row
        const int64_t nbf = S.aligned ? (n / BW) : 0;  // blocks fully inside n
        const int64_t nfull = (nbf / U) * U;           // blocks handled by the pipeline
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
            for (int64_t pr = job.r0; pr < job.r1; pr += 16 * W * TPW) {
                int64_t rt[TPW];
                const TA* arow[TPW];
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    rt[q] = pr + 16 * (wave + W * q);
                    int64_t ri = rt[q] + li;
                    if (rt[q] >= job.r1) ri = job.r0;  // idle tile: load a valid row, discard
                    if (ri >= n) ri = n - 1;
                    arow[q] = A + ri * S.lda + VEC * grp;
                }
                f32x4 acc[TPW][NT];
#pragma unroll
                for (int q = 0; q < TPW; ++q)
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[q][t] = (f32x4){0.f, 0.f, 0.f, 0.f};

                // x chunk staging: X is stored transposed, so a chunk is KT
                // contiguous row pieces (zero padded past n in global memory).
                int64_t cur_chunk = -1;
                auto ensure_chunk = [&](int64_t b) {
                    const int64_t ch = (b * BW) / CH;
                    if (ch == cur_chunk) return;
                    const int64_t c0 = ch * CH;
                    const int64_t cl = (n - c0) < CH ? (n - c0) : CH;
                    const int64_t clp = (cl + BW - 1) / BW * BW;
                    const int nq = (int)(clp / 4);
                    __syncthreads();
                    for (int e = tid; e < KT * nq; e += W * 64) {
                        const int c = e / nq, j4 = e - c * nq;
                        *reinterpret_cast<f32x4*>(xsT + c * CHP + 4 * j4) =
                            *reinterpret_cast<const f32x4*>(xin + (int64_t)c * xld + c0 + 4 * j4);
                    }
                    __syncthreads();
                    cur_chunk = ch;
                };
                // MFMAs of one A block (TPW tiles share the B operand).
                auto mfma_block = [&](float (&a)[TPW][VEC], int64_t b) {
                    const int jrel = (int)(b * BW - cur_chunk * CH);
                    f32x4 bx[NT][NS];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int sg = 0; sg < NS; ++sg)
                            bx[t][sg] = *reinterpret_cast<const f32x4*>(
                                xsT + (t * 16 + li) * CHP + jrel + VEC * grp + 4 * sg);
                    const int64_t colbase = b * BW + VEC * grp;
#pragma unroll
                    for (int q = 0; q < TPW; ++q) {
                        if (b * BW < rt[q] + 16 && rt[q] < b * BW + BW) {
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                if (colbase + e == rt[q] + li) a[q][e] = 0.0f;
                        }
#pragma unroll
                        for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                            for (int t = 0; t < NT; ++t)
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        a[q][4 * sg + r], bx[t][sg][r], acc[q][t], 0, 0, 0);
                    }
                };
                // Full blocks: two pipeline stages of U blocks; the A loads of
                // the next stage are in flight during the MFMAs (and the chunk
                // staging) of the current one.
                if (nfull > 0) {
                    u32x4 v0[U][TPW], v1[U][TPW];
                    auto issue = [&](u32x4 (&v)[U][TPW], int64_t bb) {
#pragma unroll
                        for (int u = 0; u < U; ++u)
#pragma unroll
                            for (int q = 0; q < TPW; ++q)
                                v[u][q] = __builtin_nontemporal_load(
                                    reinterpret_cast<const u32x4*>(arow[q] + (bb + u) * BW));
                    };
                    auto consume = [&](u32x4 (&v)[U][TPW], int64_t bb) {
                        ensure_chunk(bb);
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            float a[TPW][VEC];
#pragma unroll
                            for (int q = 0; q < TPW; ++q) unpack<TA>(v[u][q], a[q]);
                            mfma_block(a, bb + u);
                        }
                    };
                    issue(v0, 0);
                    int64_t b0 = 0;
                    for (; b0 + 2 * U <= nfull; b0 += 2 * U) {
                        issue(v1, b0 + U);
                        consume(v0, b0);
                        if (b0 + 2 * U < nfull) issue(v0, b0 + 2 * U);
                        consume(v1, b0 + U);
                    }
                    if (b0 < nfull) consume(v0, b0);
                }
                // Remaining blocks (ragged tail, or every block of unaligned rows).
                for (int64_t b = nfull; b < nb; ++b) {
                    ensure_chunk(b);
                    float a[TPW][VEC];
#pragma unroll
                    for (int q = 0; q < TPW; ++q) {
                        if (b < nbf) {
                            const u32x4 v = __builtin_nontemporal_load(
                                reinterpret_cast<const u32x4*>(arow[q] + b * BW));
                            unpack<TA>(v, a[q]);
                        } else {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) {
                                const int64_t col = b * BW + VEC * grp + e;
                                a[q][e] = col < n ? widen1<TA>(arow[q][b * BW + e]) : 0.0f;
                            }
                        }
                    }
                    mfma_block(a, b);
                }
                // epilogue: lane holds rows rt + 4*grp + v, column t*16 + li
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    if (rt[q] >= job.r1) continue;
                    const int64_t i0 = rt[q] + 4 * grp;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int c = t * 16 + li;
                        const f32x4 xo4 =
                            *reinterpret_cast<const f32x4*>(xin + (int64_t)c * xld + i0);
                        f32x4 xn4 = xo4;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t i = i0 + v;
                            if (i < job.r1 && c < k) {
                                const float xn = (S.B[i * S.ldb + c] - acc[q][t][v]) / S.diag[i];
                                xn4[v] = xn;
                                const double dd = fabs((double)xn - (double)xo4[v]);
                                const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                                dmax = db > dmax ? db : dmax;
                                xmax = mb > xmax ? mb : xmax;
                                sq += dd * dd;
                            }
                        }
                        // rows past r1 keep their value (zero padding or another
                        // workgroup's rows)
                        if (i0 + 3 < job.r1) {
                            *reinterpret_cast<f32x4*>(xout + (int64_t)c * xld + i0) = xn4;
                        } else {
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                if (i0 + v < job.r1) xout[(int64_t)c * xld + i0 + v] = xn4[v];
                        }
                    }
                }
            }
            // ---- workgroup reduction of the distance statistics
            dmax = wmax(dmax);
            xmax = wmax(xmax);
            sq = wsum(sq);
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
        // In the last sweep each element was written by the thread that copies
        // it here (same tile walk), so no further synchronisation is needed.
        if (final_k > 0) {
            for (int64_t rt = job.r0 + 16 * wave; rt < job.r1; rt += 16 * W) {
                // same (row, column) -> thread map as the epilogue: tile
                // pr + 16*(wave + W*q) is walked by this wave for every pass
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t i = rt + 4 * grp + v;
                        const int c = t * 16 + li;
                        if (i < job.r1 && c < k) S.X[i * S.ldx + c] = xfinal[(int64_t)c * xld + i];
                    }
            }
        } else {
            for (int64_t e = tid; e < (job.r1 - job.r0) * k; e += W * 64) {
                const int64_t i = job.r0 + e / k;
                const int c = (int)(e % k);
                S.X[i * S.ldx + c] = S.buf0[(int64_t)c * xld + i];
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
constexpr int kBW = 4;   // waves per workgroup
constexpr int kTPW = 2;  // 16-row tiles per wave per pass
constexpr int kBU = 2;   // A blocks per pipeline stage

int batched_waves() { return kBW * kTPW; }  // 16-row tiles per workgroup pass
int batched_unroll(int32_t) { return 2 * kBU; }

static size_t batched_lds(int32_t kt) {
    return (size_t)kt * ((kt <= 16 ? batched_chunk_cols<16>() : batched_chunk_cols<32>()) + 4) *
           sizeof(float);
}

template <typename TA, int KT>
static const void* batched_fn() {
    return (const void*)k_batched<TA, KT, kBW, kTPW, kBU>;
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
    int64_t bx = (max_n + 32 + 255) / 256;
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
