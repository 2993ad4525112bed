// Persistent batched Jacobi sweeps on MFMA tiles (gfx950).
//
// One persistent launch runs every sweep of many independent systems
// A_s X_s = B_s (each with k_s <= 32 right-hand sides).  The work of a sweep,
// S = (A - D) X followed by x_new = (b - s) / a_ii (the component equation of
// sec. 2 of the paper applied to every column), is a dense n x n by n x k
// contraction, done on v_mfma_f32_16x16x4_f32:
//   * a workgroup sweeps its rows in passes of TPW 16-row tiles; all W waves
//     work on the same tiles and split the columns (wave w takes every W-th
//     block), and their partial tiles are added in wave order through LDS, so
//     even a system of a few hundred rows keeps every wave streaming;
//   * lane l loads row (l % 16) of a tile with two 16-byte loads; in load j
//     the four lane groups g = l / 16 read bytes 64 j + 16 g of the block, so
//     each load covers 64 contiguous bytes of every row and the wave reads one
//     full 128-byte line of each row per block (a probe measured 5.5 TB/s for
//     whole lines per wave against 3.6 TB/s for lines split between two
//     waves; on rows that are not 16-byte aligned the contiguous 64-byte runs
//     measured 10% faster than 32-byte runs per lane); one block feeds 8
//     (FP32) or 16 (BF16) MFMA k-steps;
//   * A is read with ordinary (temporal) loads: on a row that is not 16-byte
//     aligned a block spans two cache lines, each shared with the neighbouring
//     wave's block, and non-temporal loads fetched such lines twice (64
//     systems of 4095 rows: 1.74x the bytes of A from the fabric, 3.2 TB/s;
//     with ordinary loads 1.13x and 4.2 TB/s; aligned rows also gain);
//   * the iterate is kept transposed in global memory (column c of X is a
//     contiguous row of xld floats, zero padded), so the matching B operand
//     of 4 k-steps is one 16-byte load that hits the L2 (X is small and every
//     tile of the system reads it); nothing is staged and no barrier runs
//     inside a pass;
//   * the diagonal term is masked in the A operand (sum over j != i);
//   * the reduced tile is the epilogue's input: division by a_ii, the
//     distance max|x_new - x_old| (or its Euclidean form) and the stop test.
// Three schedules run the same row sweep (sweep_rows):
//   * lockstep (k_rounds, the default): round r is sweep r of every running
//     system; rows of all systems are dealt out as work items from one
//     atomic ticket counter, one grid barrier closes each round;
//   * dataflow (k_flow): the same work items without rounds; a system's next
//     sweep is queued the moment the last item of its current sweep ends;
//   * planned (k_batched): a large system is split over several workgroups
//     that meet at a per-system barrier (atomic counter) after every sweep;
//     small systems are owned whole by one workgroup and taken from a queue.
// Residency: the grid never exceeds the occupancy-derived count of
// workgroups the device holds at once (workgroups per CU x CUs), so every
// workgroup is dispatched while the others wait at a barrier (other kernels
// running beside it only delay a dispatch: none of them waits for this one).
// An ordinary launch gives that guarantee, so no cooperative launch is used.
// A wall-clock bound on every barrier wait turns a wait that cannot end into
// an error instead of a hang.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "internal.h"

namespace jac {

typedef uint16_t bf16_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Iterate type of a launch: FP64 for FP64 A, FP32 (FP32 accumulation) for
// FP32 and BF16 A.
template <typename TA>
struct IterOf {
    using T = float;
};
template <>
struct IterOf<double> {
    using T = double;
};

namespace {

__device__ __forceinline__ float bf_to_f(uint32_t h) { return __uint_as_float(h << 16); }

// Pointers into global memory.  The system descriptors live in device memory,
// so the compiler cannot infer the address space of the pointers they hold and
// would emit flat loads, which force a full wait on every outstanding load and
// defeat the load pipeline below.
template <typename T>
using gptr = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> gbl(const T* p) {
    return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ T __attribute__((address_space(1)))* gout(T* p) {
    return (T __attribute__((address_space(1)))*)p;
}

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
__device__ __forceinline__ typename IterOf<TA>::T widen1(TA a);
template <>
__device__ __forceinline__ float widen1<float>(float a) {
    return a;
}
template <>
__device__ __forceinline__ float widen1<bf16_t>(bf16_t a) {
    return bf_to_f(a);
}
template <>
__device__ __forceinline__ double widen1<double>(double a) {
    return a;
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
// non-finite B or X0), write X0 (or zeros) and B transposed into buf0 and bT
// and clear buf1, padding included.  grid = (row blocks, systems).
template <typename TA>
__global__ void k_batched_setup(const BSys* __restrict__ sys, BState* __restrict__ st, int kt) {
    using TX = typename IterOf<TA>::T;
    const BSys S = sys[blockIdx.y];
    BState* T = &st[blockIdx.y];
    const TA* A = reinterpret_cast<const TA*>(S.A);
    TX* diag = (TX*)const_cast<void*>(S.diag);
    TX* buf0 = (TX*)S.buf0;
    TX* buf1 = (TX*)S.buf1;
    TX* bT = (TX*)S.bT;
    const TX* X0 = (const TX*)S.X0;
    const TX* B = (const TX*)S.B;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.xld; i += stride) {
        if (i >= S.n) {
            for (int c = 0; c < kt; ++c) {
                buf0[c * S.xld + i] = TX(0);
                buf1[c * S.xld + i] = TX(0);
                bT[c * S.xld + i] = TX(0);
            }
            continue;
        }
        const TX d = widen1<TA>(A[i * S.lda + i]);
        diag[i] = d;
        if (d == TX(0))
            __hip_atomic_fetch_min(&T->bad_diag, 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if (!isfinite(d))
            __hip_atomic_fetch_min(&T->bad_diag, 2 * i + 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        bool bad = false;
        for (int c = 0; c < kt; ++c) {
            TX x0 = TX(0), b = TX(0);
            if (c < S.k) {
                b = B[i * S.ldb + c];
                if (S.first_free) {
                    // the first sweep from zero: (b - 0) / a_ii, as the sweep's epilogue
                    x0 = b / d;
                    if (!isfinite(b)) bad = true;
                } else {
                    if (X0) x0 = X0[i * S.ldx + c];
                    if (!isfinite(b) || !isfinite(x0)) bad = true;
                }
            }
            buf0[c * S.xld + i] = x0;
            buf1[c * S.xld + i] = TX(0);
            bT[c * S.xld + i] = b;
        }
        if (bad)
            __hip_atomic_fetch_min(&T->bad_rhs, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// One sweep over rows [r0, r1) of system S: x_new = (b - (A - D) x_old) / a_ii
// for every column of those rows, read from `xin` and written to `xout` (both
// transposed), with this thread's share of the distance statistics added to
// dmax, xmax (double bits of max |x_new - x_old| and max |x_new|) and sq (sum
// of squares).  Every thread of the workgroup calls it; `red` is the LDS tile
// of the wave-order reduction.  A row's value depends only on the row, its
// system and W, not on [r0, r1): the same X comes out of any row split.
template <typename TA, int KT, int W, int TPW, int U>
__device__ __forceinline__ void sweep_rows(const BSys& S, int64_t r0, int64_t r1,
                                           const float* xin, float* xout, float* red, int tid,
                                           int wave, uint64_t& dmax, uint64_t& xmax, double& sq,
                                           int64_t c0, int64_t c1, float* part) {
    constexpr int LPL = 2;                     // 16-byte loads per lane and block
    constexpr int V16 = 16 / (int)sizeof(TA);  // A values per 16-byte load
    constexpr int VEC = LPL * V16;             // A values per lane and block
    constexpr int BW = 4 * VEC;                // columns of one A block (32 or 64)
    constexpr int NT = KT / 16;                // 16-column output tiles
    constexpr int NS = VEC / 4;                // 4-step MFMA groups per block
    const int lane = tid & 63, grp = lane >> 4, li = lane & 15;
    // Lane layout of a block: load j of lane group grp holds columns
    // j * 4 * V16 + grp * V16 + [0, V16), so the four groups of one load read
    // 64 contiguous bytes of a row.  Element e of a lane sits at column
    // grp * V16 + ecol(e) of the block; the B operand follows the same map.
    auto ecol = [](int e) { return (e / V16) * 4 * V16 + e % V16; };
    const TA* A = reinterpret_cast<const TA*>(S.A);
    const int64_t n = S.n;
    const int64_t xld = S.xld;
    const int k = S.k;
    // Columns [c0, c1) of the rows (the whole row unless the system's columns
    // are split over workgroups; c0 is a multiple of W * BW, so block b
    // stays with wave b % W).
    const int64_t cn = c1 < n ? c1 : n;
    const int64_t bst = c0 / BW;                   // first block
    const int64_t nb = (cn + BW - 1) / BW;         // end of the blocks
    // Full blocks are read with 16-byte loads whatever the row alignment (a
    // row of n FP32 values starts 16-byte aligned only when n % 4 == 0): the
    // runtime runs kernels in unaligned access mode, where such a load costs
    // at most one more cache-line access and returns the same values.
    const int64_t nbf = cn / BW;                   // end of the full blocks
    // this wave's vector-loadable blocks: b = bst + wave + W * t, t < ntw
    const int64_t ntw = nbf > bst + wave ? (nbf - bst - wave + W - 1) / W : 0;
    const int64_t nfull = (ntw / U) * U;
    gptr<float> xrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        xrow[t] = gbl(xin + (int64_t)(t * 16 + li) * xld + V16 * grp);
    // Row pointers of the pass starting at row pr.  Rows past the job
    // (a short last pass) re-read the job's last row, which the cache
    // serves, and are discarded.
    auto rows_of = [&](gptr<TA> (&rows)[TPW], int64_t pr) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            int64_t ri = pr + 16 * q + li;
            if (ri >= r1) ri = r1 - 1;
            rows[q] = gbl(A + ri * S.lda + V16 * grp);
        }
    };
    auto load_b = [&](f32x4 (&bx)[NT][NS], int64_t b) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int sg = 0; sg < NS; ++sg)
                bx[t][sg] = *(gptr<f32x4>)(xrow[t] + b * BW + ecol(4 * sg));
    };
    // Loads of U blocks starting at this wave's block t0.
    auto issue = [&](const gptr<TA> (&rows)[TPW], u32x4 (&v)[U][TPW][LPL],
                     f32x4 (&bx)[U][NT][NS], int64_t t0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t b = bst + wave + W * (t0 + u);
#pragma unroll
            for (int q = 0; q < TPW; ++q)
#pragma unroll
                for (int j = 0; j < LPL; ++j)
                    v[u][q][j] = *(gptr<u32x4>)(rows[q] + b * BW + j * 4 * V16);
            load_b(bx[u], b);
        }
    };
    // First pipeline stage of the next pass, loaded while the current
    // pass finishes its reduction and epilogue.
    u32x4 v0[U][TPW][LPL];
    f32x4 b0[U][NT][NS];
    bool preloaded = false;
    gptr<TA> arow[TPW];
    rows_of(arow, r0);
    for (int64_t pr = r0; pr < r1; pr += 16 * TPW) {
        int64_t rt[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) rt[q] = pr + 16 * q;
        f32x4 acc[TPW][NT];
#pragma unroll
        for (int q = 0; q < TPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[q][t] = (f32x4){0.f, 0.f, 0.f, 0.f};

        // MFMAs of one A block (the TPW tiles share the B operand).
        auto mfma_block = [&](float (&a)[TPW][VEC], const f32x4 (&bx)[NT][NS], int64_t b) {
            // Tile q's diagonal lies in block rt[q] / BW (BW is 32 or
            // 64, tiles start at multiples of 16): only that block,
            // a wave-uniform test, masks the lane's element dpos.
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (b == rt[q] / BW) {
                    const int rel = (int)(rt[q] - b * BW) + li;  // diagonal column in the block
                    const int rem = rel % (4 * V16);
                    const int dpos =
                        rem / V16 == grp ? (rel / (4 * V16)) * V16 + rem % V16 : -1;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) a[q][e] = (e == dpos) ? 0.0f : a[q][e];
                }
            }
            // Consecutive MFMAs update different accumulators.
#pragma unroll
            for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < TPW; ++q)
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                a[q][4 * sg + r], bx[t][sg][r], acc[q][t], 0, 0, 0);
        };
        // Vector-loadable blocks: two pipeline stages of U blocks; the
        // loads of one stage are in flight during the MFMAs of the other.
        if (nfull > 0) {
            u32x4 v1[U][TPW][LPL];
            f32x4 b1[U][NT][NS];
            auto consume = [&](u32x4 (&v)[U][TPW][LPL], f32x4 (&bx)[U][NT][NS],
                               int64_t t0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    float a[TPW][VEC];
#pragma unroll
                    for (int q = 0; q < TPW; ++q)
#pragma unroll
                        for (int j = 0; j < LPL; ++j) unpack<TA>(v[u][q][j], a[q] + j * V16);
                    mfma_block(a, bx[u], bst + wave + W * (t0 + u));
                }
            };
            // The scheduling barriers keep the compiler from sinking
            // the loads below the MFMAs that should hide them.
            if (!preloaded) issue(arow, v0, b0, 0);
            int64_t t = 0;
            for (; t + 3 * U <= nfull; t += 2 * U) {
                issue(arow, v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v0, b0, t);
                __builtin_amdgcn_sched_barrier(0);
                issue(arow, v0, b0, t + 2 * U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (t + 2 * U <= nfull) {
                issue(arow, v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v0, b0, t);
                __builtin_amdgcn_sched_barrier(0);
                consume(v1, b1, t + U);
            } else {
                consume(v0, b0, t);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // Start the next pass's first stage now (A and the iterate do
        // not change within a sweep).
        gptr<TA> arow_next[TPW];
        const bool more = pr + 16 * TPW < r1;
        if (more) rows_of(arow_next, pr + 16 * TPW);
        preloaded = more && nfull > 0;
        if (preloaded) issue(arow_next, v0, b0, 0);
        // Remaining blocks of this wave (the ragged tail).
        for (int64_t b = bst + wave + W * nfull; b < nb; b += W) {
            float a[TPW][VEC];
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (b < nbf) {
#pragma unroll
                    for (int j = 0; j < LPL; ++j) {
                        const u32x4 v = *(gptr<u32x4>)(arow[q] + b * BW + j * 4 * V16);
                        unpack<TA>(v, a[q] + j * V16);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int64_t col = b * BW + V16 * grp + ecol(e);
                        a[q][e] = col < n ? widen1<TA>(arow[q][b * BW + ecol(e)]) : 0.0f;
                    }
                }
            }
            f32x4 bx[NT][NS];
            load_b(bx, b);  // zero padded past n
            mfma_block(a, bx, b);
        }
        // Add the W partial tiles in wave order.  Tile element (i, j)
        // sits in lane 16 * (i / 4) + j, register i % 4.
#pragma unroll
        for (int q = 0; q < TPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[(((wave * TPW + q) * NT + t) * 4 + v) * 64 + lane] = acc[q][t][v];
        // Epilogue: thread element u is e = tid + u * W * 64: column cc of
        // tile (q, t), row ri, so consecutive threads touch consecutive rows
        // of the transposed iterate and right-hand side.  Its operands are
        // all requested here, before the barrier, so their latencies overlap
        // one another and the reduction instead of adding up.
        constexpr int EPT = TPW * NT * 256 / (W * 64);
        static_assert(EPT * W * 64 == TPW * NT * 256, "epilogue elements per thread");
        float e_xo[EPT], e_b[EPT], e_d[EPT];
        if (!part) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = tid + u * W * 64;
                const int ri = e & 15, cc = (e >> 4) & 15, qt = e >> 8;
                const int q = qt / NT, t = qt - q * NT;
                const int64_t i = pr + 16 * q + ri;
                const int c = t * 16 + cc;
                const bool ok = i < r1 && c < k;
                const int64_t is = ok ? i : r0;  // a row and column that exist
                const int cs = ok ? c : 0;
                e_xo[u] = *gbl(xin + (int64_t)cs * xld + is);
                e_b[u] = *gbl((const float*)S.bT + (int64_t)cs * xld + is);
                e_d[u] = *gbl((const float*)S.diag + is);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * W * 64;
            const int ri = e & 15, cc = (e >> 4) & 15, qt = e >> 8;
            const int q = qt / NT, t = qt - q * NT;
            const int l = 16 * (ri >> 2) + cc, v = ri & 3;
            float s = 0.0f;
#pragma unroll
            for (int w = 0; w < W; ++w) s += red[(((w * TPW + q) * NT + t) * 4 + v) * 64 + l];
            const int64_t i = pr + 16 * q + ri;
            const int c = t * 16 + cc;
            if (part) {
                // split columns: this chunk's partial sum, transposed
                if (i < r1 && c < k) *gout(part + (int64_t)c * xld + i) = s;
            } else if (i < r1 && c < k) {
                const float xo = e_xo[u];
                const float xn = (e_b[u] - s) / e_d[u];
                *gout(xout + (int64_t)c * xld + i) = xn;
                const double dd = fabs((double)xn - (double)xo);
                const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                dmax = db > dmax ? db : dmax;
                xmax = mb > xmax ? mb : xmax;
                sq += dd * dd;
            }
        }
        __syncthreads();  // red is reused by the next pass
        if (more) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) arow[q] = arow_next[q];
        }
    }
}

// ---------------------------------------------------------------------------
// The FP64 row sweep: sweep_rows with FP64 A, iterate and accumulation, on
// v_mfma_f64_16x16x4f64.  A block is 16 columns (128 bytes of a row): lane
// l loads row (l % 16) of a tile with two 16-byte loads, load j of lane group
// g = l / 16 holding columns 8 j + 2 g + {0, 1}, so each load covers 64
// contiguous bytes of every row and the two loads the whole line.  Element e
// of a lane (load e / 2, half e % 2) is MFMA k-step e of the block; the B
// operand of the same k-steps is two 16-byte loads of the transposed iterate.
// The output tile puts element (i, j) in lane 16 (i % 4) + j, register i / 4.
template <int KT, int W, int TPW, int U>
__device__ __forceinline__ void sweep_rows_f64(const BSys& S, int64_t r0, int64_t r1,
                                               const double* xin, double* xout, double* red,
                                               int tid, int wave, uint64_t& dmax,
                                               uint64_t& xmax, double& sq, int64_t c0,
                                               int64_t c1, double* part) {
    constexpr int BW = 16;       // columns of one A block
    constexpr int NT = KT / 16;  // 16-column output tiles
    const int lane = tid & 63, grp = lane >> 4, li = lane & 15;
    const double* A = reinterpret_cast<const double*>(S.A);
    const int64_t n = S.n;
    const int64_t xld = S.xld;
    const int k = S.k;
    // columns [c0, c1), as in sweep_rows
    const int64_t cn = c1 < n ? c1 : n;
    const int64_t bst = c0 / BW;            // first block
    const int64_t nb = (cn + BW - 1) / BW;  // end of the blocks
    const int64_t nbf = cn / BW;            // end of the blocks entirely inside the row
    const int64_t ntw = nbf > bst + wave ? (nbf - bst - wave + W - 1) / W : 0;
    const int64_t nfull = (ntw / U) * U;
    gptr<double> xrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) xrow[t] = gbl(xin + (int64_t)(t * 16 + li) * xld + 2 * grp);
    auto rows_of = [&](gptr<double> (&rows)[TPW], int64_t pr) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            int64_t ri = pr + 16 * q + li;
            if (ri >= r1) ri = r1 - 1;
            rows[q] = gbl(A + ri * S.lda + 2 * grp);
        }
    };
    auto load_b = [&](f64x2 (&bx)[NT][2], int64_t b) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 2; ++j) bx[t][j] = *(gptr<f64x2>)(xrow[t] + b * BW + 8 * j);
    };
    auto issue = [&](const gptr<double> (&rows)[TPW], f64x2 (&v)[U][TPW][2],
                     f64x2 (&bx)[U][NT][2], int64_t t0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t b = bst + wave + W * (t0 + u);
#pragma unroll
            for (int q = 0; q < TPW; ++q)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    v[u][q][j] = *(gptr<f64x2>)(rows[q] + b * BW + 8 * j);
            load_b(bx[u], b);
        }
    };
    f64x2 v0[U][TPW][2];
    f64x2 b0[U][NT][2];
    bool preloaded = false;
    gptr<double> arow[TPW];
    rows_of(arow, r0);
    for (int64_t pr = r0; pr < r1; pr += 16 * TPW) {
        int64_t rt[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) rt[q] = pr + 16 * q;
        f64x4 acc[TPW][NT];
#pragma unroll
        for (int q = 0; q < TPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[q][t] = (f64x4){0.0, 0.0, 0.0, 0.0};
        // MFMAs of one block; tile q's diagonal lies in block rt[q] / 16,
        // at block column li, held by lane group (li % 8) / 2 as element
        // 2 (li / 8) + li % 2.
        auto mfma_block = [&](f64x2 (&a)[TPW][2], const f64x2 (&bx)[NT][2], int64_t b) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (b == rt[q] / BW) {
                    const int dpos = ((li & 7) >> 1) == grp ? 2 * (li >> 3) + (li & 1) : -1;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e == dpos) a[q][e >> 1][e & 1] = 0.0;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int q = 0; q < TPW; ++q)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            a[q][e >> 1][e & 1], bx[t][e >> 1][e & 1], acc[q][t], 0, 0, 0);
        };
        if (nfull > 0) {
            f64x2 v1[U][TPW][2];
            f64x2 b1[U][NT][2];
            auto consume = [&](f64x2 (&v)[U][TPW][2], f64x2 (&bx)[U][NT][2], int64_t t0) {
#pragma unroll
                for (int u = 0; u < U; ++u) mfma_block(v[u], bx[u], bst + wave + W * (t0 + u));
            };
            if (!preloaded) issue(arow, v0, b0, 0);
            int64_t t = 0;
            for (; t + 3 * U <= nfull; t += 2 * U) {
                issue(arow, v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v0, b0, t);
                __builtin_amdgcn_sched_barrier(0);
                issue(arow, v0, b0, t + 2 * U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (t + 2 * U <= nfull) {
                issue(arow, v1, b1, t + U);
                __builtin_amdgcn_sched_barrier(0);
                consume(v0, b0, t);
                __builtin_amdgcn_sched_barrier(0);
                consume(v1, b1, t + U);
            } else {
                consume(v0, b0, t);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        gptr<double> arow_next[TPW];
        const bool more = pr + 16 * TPW < r1;
        if (more) rows_of(arow_next, pr + 16 * TPW);
        preloaded = more && nfull > 0;
        if (preloaded) issue(arow_next, v0, b0, 0);
        // Remaining blocks of this wave (the ragged tail).
        for (int64_t b = bst + wave + W * nfull; b < nb; b += W) {
            f64x2 a[TPW][2];
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (b < nbf) {
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        a[q][j] = *(gptr<f64x2>)(arow[q] + b * BW + 8 * j);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int off = 8 * (e >> 1) + (e & 1);
                        const int64_t col = b * BW + 2 * grp + off;
                        a[q][e >> 1][e & 1] = col < n ? arow[q][b * BW + off] : 0.0;
                    }
                }
            }
            f64x2 bx[NT][2];
            load_b(bx, b);  // zero padded past n
            mfma_block(a, bx, b);
        }
        // Add the W partial tiles in wave order.
#pragma unroll
        for (int q = 0; q < TPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[(((wave * TPW + q) * NT + t) * 4 + v) * 64 + lane] = acc[q][t][v];
        constexpr int EPT = TPW * NT * 256 / (W * 64);
        static_assert(EPT * W * 64 == TPW * NT * 256, "epilogue elements per thread");
        double e_xo[EPT], e_b[EPT], e_d[EPT];
        if (!part) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = tid + u * W * 64;
                const int ri = e & 15, cc = (e >> 4) & 15, qt = e >> 8;
                const int q = qt / NT, t = qt - q * NT;
                const int64_t i = pr + 16 * q + ri;
                const int c = t * 16 + cc;
                const bool ok = i < r1 && c < k;
                const int64_t is = ok ? i : r0;
                const int cs = ok ? c : 0;
                e_xo[u] = *gbl(xin + (int64_t)cs * xld + is);
                e_b[u] = *gbl((const double*)S.bT + (int64_t)cs * xld + is);
                e_d[u] = *gbl((const double*)S.diag + is);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * W * 64;
            const int ri = e & 15, cc = (e >> 4) & 15, qt = e >> 8;
            const int q = qt / NT, t = qt - q * NT;
            const int l = 16 * (ri & 3) + cc, v = ri >> 2;
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) s += red[(((w * TPW + q) * NT + t) * 4 + v) * 64 + l];
            const int64_t i = pr + 16 * q + ri;
            const int c = t * 16 + cc;
            if (part) {
                if (i < r1 && c < k) *gout(part + (int64_t)c * xld + i) = s;
            } else if (i < r1 && c < k) {
                const double xo = e_xo[u];
                const double xn = (e_b[u] - s) / e_d[u];
                *gout(xout + (int64_t)c * xld + i) = xn;
                const double dd = fabs(xn - xo);
                const uint64_t db = dbits(dd), mb = dbits(fabs(xn));
                dmax = db > dmax ? db : dmax;
                xmax = mb > xmax ? mb : xmax;
                sq += dd * dd;
            }
        }
        __syncthreads();  // red is reused by the next pass
        if (more) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) arow[q] = arow_next[q];
        }
    }
}

// The row sweep of a launch's element type.
// Columns [c0, c1) only, with `part` non-null: the rows' partial sums over
// those columns are written to `part` (transposed like the iterate) instead
// of the epilogue.
template <typename TA, int KT, int W, int TPW, int U>
__device__ __forceinline__ void sweep_any(const BSys& S, int64_t r0, int64_t r1, const void* xin,
                                          void* xout, void* red, int tid, int wave,
                                          uint64_t& dmax, uint64_t& xmax, double& sq,
                                          int64_t c0, int64_t c1, void* part) {
    if constexpr (std::is_same<TA, double>::value)
        sweep_rows_f64<KT, W, TPW, U>(S, r0, r1, (const double*)xin, (double*)xout,
                                      (double*)red, tid, wave, dmax, xmax, sq, c0, c1,
                                      (double*)part);
    else
        sweep_rows<TA, KT, W, TPW, U>(S, r0, r1, (const float*)xin, (float*)xout, (float*)red,
                                      tid, wave, dmax, xmax, sq, c0, c1, (float*)part);
}

// Rows [r0, r1) of a final iterate (transposed: column c at xsrc + c * xld)
// into the caller's row-major X, through an LDS tile of 64 rows (tile, the
// row sweep's reduction area, holds 64 x (KT + 1) values): each column's run
// of rows is read contiguously, each row's run of columns is written
// contiguously.  Every thread of the workgroup calls it.
template <typename TX, int KT, int W>
__device__ __forceinline__ void copy_out(const BSys& S, int64_t r0, int64_t r1, const TX* xsrc,
                                         TX* tile, int tid) {
    constexpr int ROWS = 64, LD = KT + 1;  // odd stride: no bank conflicts either way
    const int k = S.k;
    TX* X = (TX*)S.X;
    for (int64_t t0 = r0; t0 < r1; t0 += ROWS) {
        const int nr = (int)(r1 - t0 < ROWS ? r1 - t0 : ROWS);
        for (int e = tid; e < k * ROWS; e += W * 64) {
            const int c = e / ROWS, i = e - c * ROWS;
            if (i < nr) tile[i * LD + c] = xsrc[(int64_t)c * S.xld + t0 + i];
        }
        __syncthreads();
        for (int e = tid; e < nr * k; e += W * 64) {
            const int i = e / k, c = e - i * k;
            X[(t0 + i) * S.ldx + c] = tile[i * LD + c];
        }
        __syncthreads();  // the tile is reused
    }
}

// ---------------------------------------------------------------------------
// The persistent kernel.
//   W   waves per workgroup (they split the columns of every tile)
//   TPW 16-row tiles per pass (they share every B operand load)
//   U   column blocks per pipeline stage (two stages in flight)
//   MINB workgroups per CU the register budget is sized for
template <typename TA, int KT, int W, int TPW, int U, int MINB>
__global__ __launch_bounds__(W * 64, MINB) void k_batched(BatchArgs p) {
    using TX = typename IterOf<TA>::T;
    constexpr int NT = KT / 16;                // 16-column output tiles
    __shared__ TX red[W * TPW * NT * 256];
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ uint32_t s_flag;
    __shared__ double s_delta;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: block tests stay scalar

    __shared__ int32_t s_next;
    int jb = p.job_off[blockIdx.x];
    const int jend = p.job_off[blockIdx.x + 1];
    for (;;) {
        // The workgroup's fixed jobs (shares of split systems), then whole
        // systems from the queue until it runs dry.
        BJob job;
        if (jb < jend) {
            job = p.jobs[jb++];
        } else {
            __syncthreads();
            if (tid == 0)
                s_next = p.queue_len > 0 ? (int32_t)__hip_atomic_fetch_add(
                                               p.queue_head, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                                         : INT32_MAX;
            __syncthreads();
            const int32_t qi = s_next;
            if (qi >= p.queue_len) break;
            job.sys = p.queue[qi];
            job.rank = 0;
            job.r0 = 0;
            job.r1 = (int32_t)p.sys[job.sys].n;
        }
        const BSys S = p.sys[job.sys];
        BState* st = &p.st[job.sys];
        if (__hip_atomic_load(&st->bad_diag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                INT64_MAX ||
            __hip_atomic_load(&st->bad_rhs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                INT64_MAX)
            continue;  // invalid input: no sweep runs, X untouched
        const int64_t xld = S.xld;
        const int k = S.k;
        const bool split = S.nwg > 1;
        const TX* xfinal = (const TX*)S.buf0;
        int32_t final_k = 0;
        uint32_t final_stop = STOP_RUNNING;
        double final_delta = -1.0;
        bool failed = false;

        for (int sweep = 1; sweep <= S.max_iter; ++sweep) {
            const TX* xin = (const TX*)((sweep & 1) ? S.buf0 : S.buf1);
            TX* xout = (TX*)((sweep & 1) ? S.buf1 : S.buf0);
            uint64_t dmax = 0, xmax = 0;
            double sq = 0.0;
            sweep_any<TA, KT, W, TPW, U>(S, job.r0, job.r1, xin, xout, red, tid, wave, dmax,
                                         xmax, sq, 0, S.n, nullptr);
            // ---- workgroup reduction of the distance statistics
            dmax = wmax(dmax);
            xmax = wmax(xmax);
            sq = wsum(sq);
            if (lane == 0) {
                red_d[wave] = dmax;
                red_m[wave] = xmax;
                red_s[wave] = sq;
            }
            __syncthreads();  // every wave's x_new stores precede tid 0's release below
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
                    // One release (the atomic) and one acquire (the fence after
                    // the wait) per sweep: each writes back or invalidates the
                    // L2, so the wait itself polls with relaxed loads.
                    __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t target = (uint32_t)S.nwg * (uint32_t)sweep;
                    const uint64_t t0 = wall_clock64();
                    while (__hip_atomic_load(&st->counter, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < target) {
                        __builtin_amdgcn_s_sleep(2);
                        if ((int64_t)(wall_clock64() - t0) > p.spin_limit) {
                            __hip_atomic_store(&st->error, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            flag = 99;
                            break;
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
            __syncthreads();  // tid 0's acquire precedes every wave's next loads
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
        // Every thread of the workgroup wrote its share of them before the
        // barriers that closed the last sweep.
        const TX* xsrc = final_k > 0 ? xfinal : (const TX*)S.buf0;
        for (int64_t e = tid; e < (job.r1 - job.r0) * k; e += W * 64) {
            const int64_t i = job.r0 + e / k;
            const int c = (int)(e % k);
            ((TX*)S.X)[i * S.ldx + c] = xsrc[(int64_t)c * xld + i];
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
// The lockstep schedule.  Round r is sweep r of every system still running:
// the rows of all systems are cut into work items and every workgroup takes
// items from atomic ticket counters until the round's items are gone, then
// waits at one grid barrier.  No workgroup ever waits for one system: a few
// large systems and many small ones load the chip evenly.  The items form one
// group per XCD (each system's items in one group, largest systems first);
// workgroup g, which runs on XCD g % ngroups, drains its own group's queue
// and then helps the other groups in turn, so a system's iterate, read in
// full by each of its items, is mostly read from one XCD's L2.
//
// Each item adds its distance maxima to its system's slot for the round (and
// its sum of squares to its own slot for the Euclidean norm).  The stop test
// of sweep r - 1 is taken at the start of round r, after the grid barrier
// has made every item's contribution visible, by every item of the system
// alike (the Euclidean sum in item order, so the distance does not depend on
// the schedule): no item waits for, or fences against, the other items of
// its system inside a round.  A system that stops after sweep r - 1 has its
// rows copied to the caller's X by its items in round r; its first item
// records the outcome.  The loop ends after the first round in which no
// system swept (its copies done): every workgroup reads that round's count
// after the barrier, and nothing changes the count after the barrier, so all
// workgroups leave after the same round.
//   SPLIT  compiled with the column split (one system per launch); the
//          batched launches run the variant without it
template <typename TA, int KT, int W, int TPW, int U, int MINB, bool SPLIT>
__global__ __launch_bounds__(W * 64, MINB) void k_rounds(BatchArgs p) {
    using TX = typename IterOf<TA>::T;
    constexpr int NT = KT / 16;
    __shared__ TX red[W * TPW * NT * 256];
    static_assert(64 * (KT + 1) <= W * TPW * NT * 256, "the copy-out tile fits in red");
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ int32_t s_item, s_act;
    __shared__ uint32_t s_flag;
    __shared__ double s_delta;
    __shared__ uint32_t s_swept, s_abort;
    enum { ACT_SKIP = 0, ACT_COPY = 1, ACT_STOP = 2, ACT_SWEEP = 3, ACT_INVALID = 4 };

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int r = 1;; ++r) {
        const int par = r & 1;
        // the other parity's tickets were last drawn in round r - 1, which
        // every workgroup has left; they are next drawn in round r + 1
        if (blockIdx.x == 0 && tid < p.ngroups)
            __hip_atomic_store(&p.ctl->qhead[par ^ 1][tid], 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (blockIdx.x == 0 && tid == 0)
            __hip_atomic_store(&p.ctl->swept[(r + 1) % 3], 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        int qoff = 0;  // thread 0: groups of this round found empty, own group first
        for (;;) {
            __syncthreads();  // the shared words and red are reused
            if (tid == 0) {
                int32_t it = -1;
                while (qoff < p.ngroups) {
                    const int g = (int)((blockIdx.x + qoff) % (uint32_t)p.ngroups);
                    const int32_t cnt = p.group_off[g + 1] - p.group_off[g];
                    const uint32_t t = cnt > 0 ? __hip_atomic_fetch_add(
                                                     &p.ctl->qhead[par][g], 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                               : 0u;
                    if ((int32_t)t < cnt) {
                        it = p.group_off[g] + (int32_t)t;
                        break;
                    }
                    ++qoff;
                }
                s_item = it;
                if (it >= 0) {
                    // What this item does in round r, decided by one thread
                    // for the workgroup.  `done` is 0 while the system runs,
                    // r when it is copied out in this round (max_iter = 0,
                    // or set by its first item below: either way the same
                    // action), and otherwise final.
                    const int32_t sys = p.items[it].sys;
                    BState* st = &p.st[sys];
                    const int32_t done =
                        __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const bool bad = __hip_atomic_load(&st->bad_diag, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) != INT64_MAX ||
                                     __hip_atomic_load(&st->bad_rhs, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) != INT64_MAX;
                    int32_t act = ACT_SKIP;
                    uint32_t flag = STOP_RUNNING;
                    double delta = -1.0;
                    if (done == r) {
                        act = bad ? ACT_SKIP : ACT_COPY;
                    } else if (done == 0) {
                        if (bad) {
                            act = ACT_INVALID;
                        } else if (r == 1) {
                            act = ACT_SWEEP;
                        } else {
                            // the stop test of sweep r - 1
                            const int32_t it0 = p.sys[sys].it0, it1 = p.sys[sys].it1;
                            const int32_t norm = p.sys[sys].norm;
                            const int slot = (r - 1) % 3;
                            const uint64_t D = __hip_atomic_load(&st->dmax[slot], __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                            const uint64_t M = __hip_atomic_load(&st->xmax[slot], __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                            if (norm == 1) {
                                const double* ip = p.item_parts + (size_t)((r - 1) & 1) * p.nitems;
                                double Q = 0.0;  // item order: independent of the schedule
                                for (int32_t j = it0; j < it1; ++j)
                                    Q += __hip_atomic_load(&ip[j], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                                delta = sqrt(Q);
                            } else {
                                delta = bitsd(D);
                            }
                            const int32_t test = p.sys[sys].test;
                            if (!isfinite(delta))
                                flag = STOP_DIVERGED;
                            else if (test == TEST_ABS ? (delta < p.sys[sys].tol)
                                                      : (delta <= p.sys[sys].rel * bitsd(M)))
                                flag = STOP_CONVERGED;
                            act = (flag != STOP_RUNNING || r - 1 == p.sys[sys].max_iter)
                                      ? ACT_STOP
                                      : ACT_SWEEP;
                        }
                    }
                    s_act = act;
                    s_flag = flag;
                    s_delta = delta;
                }
            }
            __syncthreads();
            const int32_t it = s_item;
            if (it < 0) break;
            const int32_t act = s_act;
            if (act == ACT_SKIP) continue;
            const BJob item = p.items[it];
            BState* st = &p.st[item.sys];
            const BSys S = p.sys[item.sys];
            const bool first = it == S.it0;
            if (act == ACT_INVALID) {
                if (first && tid == 0)
                    __hip_atomic_store(&st->done, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (act == ACT_COPY || act == ACT_STOP) {
                // stopped after sweep r - 1: this item's rows of the final
                // iterate (one chunk of a split row range copies them)
                const TX* xsrc = (const TX*)(((r - 1) & 1) ? S.buf1 : S.buf0);
                if (!(SPLIT && item.rank != 0))
                    copy_out<TX, KT, W>(S, item.r0, item.r1, xsrc, red, tid);
                if (act == ACT_STOP && first && tid == 0) {
                    __hip_atomic_store(&st->status, s_flag, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st->iterations, r - 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st->final_delta, dbits(s_delta), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st->done, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                continue;
            }
            // ACT_SWEEP: sweep r of this item's rows
            if (first && tid == 0) {
                // slot (r + 1) % 3 was last read in round r - 1; round r + 1 fills it
                const int nxt = (r + 1) % 3;
                __hip_atomic_store(&st->dmax[nxt], (uint64_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->xmax[nxt], (uint64_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&p.ctl->swept[r % 3], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            uint64_t dmax = 0, xmax = 0;
            double sq = 0.0;
            const TX* xin = (const TX*)((r & 1) ? S.buf0 : S.buf1);
            TX* xout = (TX*)((r & 1) ? S.buf1 : S.buf0);
            int32_t qslot = it;  // where this item's sum of squares goes
            if constexpr (!SPLIT) {
                sweep_any<TA, KT, W, TPW, U>(S, item.r0, item.r1, xin, xout, red, tid, wave,
                                             dmax, xmax, sq, 0, S.n, nullptr);
            } else {
                // Column chunk item.rank of rows [r0, r1): partial sums only.
                const int32_t cs = S.csplit;
                const int32_t rr0 = S.it0 + (it - S.it0) / cs * cs;  // the range's first item
                const int64_t c0 = (int64_t)item.rank * S.cw;
                const int64_t c1 = c0 + S.cw < S.n ? c0 + S.cw : S.n;
                TX* part = (TX*)S.part;
                sweep_any<TA, KT, W, TPW, U>(S, item.r0, item.r1, xin, xout, red, tid, wave,
                                             dmax, xmax, sq, c0, c1,
                                             part + (size_t)item.rank * KT * S.xld);
                // every partial-sum store precedes thread 0's release (the
                // row sweep ends with a workgroup barrier)
                if (tid == 0) {
                    const uint32_t t = __hip_atomic_fetch_add(&p.rcnt[rr0], 1u, __ATOMIC_RELEASE,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                    const bool lastc = t + 1 == (uint32_t)cs;
                    if (lastc) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        __hip_atomic_store(&p.rcnt[rr0], 0u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                    s_act = lastc ? 1 : 0;
                }
                __syncthreads();
                if (s_act) {
                    // the last chunk: chunk sums in chunk order, then the epilogue
                    const int64_t rows = item.r1 - item.r0;
                    const int k = S.k;
                    const int64_t xld = S.xld;
                    for (int64_t e = tid; e < rows * k; e += W * 64) {
                        const int c = (int)(e / rows);
                        const int64_t i = item.r0 + e % rows;
                        TX acc = TX(0);
                        for (int32_t ch = 0; ch < cs; ++ch)
                            acc += part[(size_t)ch * KT * xld + (int64_t)c * xld + i];
                        const TX xo = xin[(int64_t)c * xld + i];
                        const TX xn = (((const TX*)S.bT)[(int64_t)c * xld + i] - acc) /
                                      ((const TX*)S.diag)[i];
                        xout[(int64_t)c * xld + i] = xn;
                        const double dd = fabs((double)xn - (double)xo);
                        const uint64_t db = dbits(dd), mb = dbits(fabs((double)xn));
                        dmax = db > dmax ? db : dmax;
                        xmax = mb > xmax ? mb : xmax;
                        sq += dd * dd;
                    }
                }
                qslot = s_act ? rr0 : -1;
                if (s_act && tid == 0)
                    for (int32_t j = 1; j < cs; ++j)  // the range's other slots hold zero
                        __hip_atomic_store(&p.item_parts[(size_t)par * p.nitems + rr0 + j], 0.0,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            dmax = wmax(dmax);
            xmax = wmax(xmax);
            sq = wsum(sq);
            if (lane == 0) {
                red_d[wave] = dmax;
                red_m[wave] = xmax;
                red_s[wave] = sq;
            }
            __syncthreads();
            if (tid == 0) {
                uint64_t D = 0, M = 0;
                double Q = 0.0;
                for (int w = 0; w < W; ++w) {
                    D = red_d[w] > D ? red_d[w] : D;
                    M = red_m[w] > M ? red_m[w] : M;
                    Q += red_s[w];
                }
                const int slot = r % 3;
                if (S.norm == 1 && qslot >= 0)
                    __hip_atomic_store(&p.item_parts[(size_t)par * p.nitems + qslot], Q,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&st->dmax[slot], D, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&st->xmax[slot], M, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // ---- grid barrier: one release (the arrival) and one acquire per round
        if (tid == 0) {
            __hip_atomic_fetch_add(&p.ctl->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = gridDim.x * (uint32_t)r;
            const uint64_t t0 = wall_clock64();
            uint32_t abort = 0;
            while (__hip_atomic_load(&p.ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                   target) {
                __builtin_amdgcn_s_sleep(2);
                if (__hip_atomic_load(&p.ctl->abort, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    (int64_t)(wall_clock64() - t0) > p.spin_limit) {
                    __hip_atomic_store(&p.ctl->abort, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    abort = 1;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_abort = abort;
            s_swept = __hip_atomic_load(&p.ctl->swept[r % 3], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (s_abort) break;
        // No system swept in round r: every system has been copied out (in
        // this round or earlier).  Every running system is copied out by the
        // round after its max_iter-th sweep, so the second test never decides
        // alone; it bounds the loop whatever the counters say.
        if (s_swept == 0 || r > p.max_rounds) break;
    }
}

// ---------------------------------------------------------------------------
// Dataflow schedule (k_flow): the lockstep schedule's work items and row
// sweep, without rounds.  Sweep r + 1 of a system needs only that system's
// x^(r), so its items are queued the moment the last item of its sweep r
// finishes: no workgroup waits at a grid barrier for systems it does not
// touch, and the sweeps of different systems overlap.
//
// Queue: a sequence of work items.  Positions [0, nitems) are every system's
// first work, item p at position p (the items are listed system by system,
// largest system first); later positions are published in `ring` as
// (gen << 32) | (item + 1).  A workgroup takes the next position with one
// fetch-and-add on fhead and, if nothing is published there yet, waits for
// it (or for the end of the run).  The system's `work` says what its queued
// items do (2 r: sweep r; 2 r + 1: copy x^(r) to the caller's X); it changes
// only when every item of the current work has finished.  Positions are
// never reused within a launch (the host sizes the ring for every system's
// max_iter works), so nothing is ever read stale.
//
// Completion: each item adds one to the system's `fin` with release order
// after all of its stores; the item that completes the count takes an
// acquire fence and runs the system's step: the stop test of sweep r (the
// same test, from the same maximum or item-ordered sums, as the lockstep
// schedule: the outcome does not depend on the schedule), then queues the
// items of sweep r + 1 or of the copy-out, or, after a copy-out or on invalid
// input, retires the system.  Publishing: `work`, the cleared statistics and
// count, a release fence, then the ring entries; a claimer reads its entry
// with acquire order.  The kernel ends when no system is left (`active`).
// Deadlock freedom: a workgroup only waits for its own position to be
// published, and while a system is active some item of it is running or its
// next items are being published by a running workgroup.
template <typename TA, int KT, int W, int TPW, int U, int MINB>
__global__ __launch_bounds__(W * 64, MINB) void k_flow(BatchArgs p) {
    using TX = typename IterOf<TA>::T;
    constexpr int NT = KT / 16;
    __shared__ TX red[W * TPW * NT * 256];
    static_assert(64 * (KT + 1) <= W * TPW * NT * 256, "the copy-out tile fits in red");
    __shared__ uint64_t red_d[W], red_m[W];
    __shared__ double red_s[W];
    __shared__ int32_t s_item, s_work, s_bad;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    BCtl* ctl = p.ctl;
    for (;;) {
        __syncthreads();  // the shared words and red are reused
        if (tid == 0) {
            int32_t it = -1, work = 0, bad = 0;
            const uint32_t pos =
                __hip_atomic_fetch_add(&ctl->fhead, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t t_wait = 0;
            for (;;) {
                int32_t cand = -1;
                if (pos < (uint32_t)p.nitems) {
                    cand = (int32_t)pos;
                } else if (pos - (uint32_t)p.nitems < p.ring_cap) {
                    const uint64_t v = __hip_atomic_load(&p.ring[pos - (uint32_t)p.nitems],
                                                         __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if ((uint32_t)(v >> 32) == p.gen) cand = (int32_t)(uint32_t)v - 1;
                }
                if (cand >= 0) {
                    it = cand;
                    BState* st = &p.st[p.items[cand].sys];
                    work = __hip_atomic_load(&st->work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (work == 2)
                        bad = __hip_atomic_load(&st->bad_diag, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) != INT64_MAX ||
                              __hip_atomic_load(&st->bad_rhs, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) != INT64_MAX;
                    break;
                }
                // nothing published at this position yet: every remaining
                // item is running, or the run is over
                if (__hip_atomic_load(&ctl->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                        0 ||
                    __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                    break;
                __builtin_amdgcn_s_sleep(8);
                // a wait that cannot end becomes an error
                const uint64_t now = wall_clock64();
                if (t_wait == 0) {
                    t_wait = now;
                } else if ((int64_t)(now - t_wait) > p.spin_limit) {
                    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            s_item = it;
            s_work = work;
            s_bad = bad;
        }
        __syncthreads();
        const int32_t it = s_item;
        if (it < 0) break;
        const int32_t work = s_work;
        const BJob item = p.items[it];
        BState* st = &p.st[item.sys];
        const BSys S = p.sys[item.sys];
        const int32_t r = work >> 1;
        if (work & 1) {
            // copy-out: this item's rows of x^(r) (r = 0: X0) into X
            const TX* xsrc = (const TX*)((r & 1) ? S.buf1 : S.buf0);
            copy_out<TX, KT, W>(S, item.r0, item.r1, xsrc, red, tid);
        } else if (!s_bad) {
            // sweep r of this item's rows (x^(r-1) in buf[(r-1) & 1])
            uint64_t dmax = 0, xmax = 0;
            double sq = 0.0;
            const TX* xin = (const TX*)((r & 1) ? S.buf0 : S.buf1);
            TX* xout = (TX*)((r & 1) ? S.buf1 : S.buf0);
            sweep_any<TA, KT, W, TPW, U>(S, item.r0, item.r1, xin, xout, red, tid, wave, dmax,
                                         xmax, sq, 0, S.n, nullptr);
            dmax = wmax(dmax);
            xmax = wmax(xmax);
            sq = wsum(sq);
            if (lane == 0) {
                red_d[wave] = dmax;
                red_m[wave] = xmax;
                red_s[wave] = sq;
            }
            __syncthreads();
            if (tid == 0) {
                uint64_t D = 0, M = 0;
                double Q = 0.0;
                for (int w = 0; w < W; ++w) {
                    D = red_d[w] > D ? red_d[w] : D;
                    M = red_m[w] > M ? red_m[w] : M;
                    Q += red_s[w];
                }
                if (S.norm == 1)
                    __hip_atomic_store(&p.item_parts[(size_t)(r & 1) * p.nitems + it], Q,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&st->dmax[r & 1], D, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&st->xmax[r & 1], M, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();  // every store of the item precedes thread 0's release
        if (tid == 0) {
            const uint32_t ni = (uint32_t)(S.it1 - S.it0);
            const uint32_t f = __hip_atomic_fetch_add(&st->fin, 1u, __ATOMIC_RELEASE,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (f + 1 == ni) {
                // the system's work is complete: its step
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                int32_t next = 0;  // work to queue (0: retire the system)
                if (work & 1) {
                    next = 0;
                } else if (s_bad) {
                    __hip_atomic_store(&st->done, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    const uint64_t D = __hip_atomic_load(&st->dmax[r & 1], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t M = __hip_atomic_load(&st->xmax[r & 1], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    double delta;
                    if (S.norm == 1) {
                        const double* ip = p.item_parts + (size_t)(r & 1) * p.nitems;
                        double Q = 0.0;  // item order: independent of the schedule
                        for (int32_t j = S.it0; j < S.it1; ++j)
                            Q += __hip_atomic_load(&ip[j], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        delta = sqrt(Q);
                    } else {
                        delta = bitsd(D);
                    }
                    uint32_t flag = STOP_RUNNING;
                    if (!isfinite(delta))
                        flag = STOP_DIVERGED;
                    else if (S.test == TEST_ABS ? (delta < S.tol) : (delta <= S.rel * bitsd(M)))
                        flag = STOP_CONVERGED;
                    if (flag != STOP_RUNNING || r == S.max_iter) {
                        __hip_atomic_store(&st->status, flag, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->iterations, r, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->final_delta, dbits(delta), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->done, r + 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        next = 2 * r + 1;
                    } else {
                        // sweep r + 1 accumulates in the other statistics slot
                        __hip_atomic_store(&st->dmax[(r + 1) & 1], (uint64_t)0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->xmax[(r + 1) & 1], (uint64_t)0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        next = 2 * (r + 1);
                    }
                }
                if (next == 0) {
                    __hip_atomic_fetch_sub(&ctl->active, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    __hip_atomic_store(&st->work, next, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st->fin, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t q = __hip_atomic_fetch_add(&ctl->ftail, ni, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) -
                                       (uint32_t)p.nitems;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    for (uint32_t j = 0; j < ni; ++j) {
                        if (q + j >= p.ring_cap) {
                            // cannot happen with the host's sizing; end the launch
                            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                        __hip_atomic_store(&p.ring[q + j],
                                           ((uint64_t)p.gen << 32) | (uint32_t)(S.it0 + j + 1),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
constexpr int kBW = 4;   // waves per workgroup
constexpr int kBU = 1;   // A blocks per pipeline stage (each block is two loads per row)

// Two shapes of the kernel:
//   wide  two workgroups per CU; 4 tiles per pass for FP32 with <= 16 columns,
//         else 2 (registers).  Many small systems: more workgroups to pack.
//   deep  one workgroup per CU (the register file doubles, accumulators move
//         to AGPRs) and 4 or 8 tiles per pass, so each B operand load serves
//         4 or 8 tiles.  Few large systems: less L2 traffic per A byte.
//   FP64 A takes 2 tiles per pass in the wide shape, 4 in the deep one.
//   The deep lockstep kernel without column split (`wide8`) takes 8 tiles
//   per pass for FP32 A and for BF16 A with <= 16 columns: each B operand
//   load then serves 8 tiles (256 FP32 systems of 256..4096 rows, 32
//   columns: 5.00 -> 4.70 ms; 64 systems of 4096 rows: 4.33 -> 4.82 TB/s).
//   The planned and split kernels and BF16 with 32 columns would spill
//   registers at 8, and the split plan cuts rows in ranges of 64 (one pass
//   of 4 tiles), so they keep 4.
template <typename TA>
constexpr int tiles_per_pass(int kt, int variant, bool wide8 = false) {
    if (variant == 1)
        return (wide8 && (sizeof(TA) == 4 || (sizeof(TA) == 2 && kt <= 16))) ? 8 : 4;
    return (kt <= 16 && sizeof(TA) == 4) ? 4 : 2;
}

// Shape parameters seen by the host planner: tiles per pass and the columns
// one wave covers per pipeline round trip.
int batched_tiles_per_pass(int32_t a_dtype, int32_t kt, int variant, bool lockstep_whole) {
    if (a_dtype == 0) return tiles_per_pass<double>(kt, variant, lockstep_whole);
    return a_dtype == 1 ? tiles_per_pass<float>(kt, variant, lockstep_whole)
                        : tiles_per_pass<bf16_t>(kt, variant, lockstep_whole);
}
int batched_unroll(int32_t) { return 2 * kBU; }
int batched_block_cols(int32_t a_dtype) {
    return kBW * (a_dtype == 0 ? 16 : (a_dtype == 1 ? 32 : 64));
}

template <typename TA, int KT>
static const void* batched_fn(int variant) {
    if (variant == 1) return (const void*)k_batched<TA, KT, kBW, tiles_per_pass<TA>(KT, 1), kBU, 1>;
    return (const void*)k_batched<TA, KT, kBW, tiles_per_pass<TA>(KT, 0), kBU, 2>;
}

static const void* pick(int32_t a_dtype, int32_t kt, int variant) {
    if (a_dtype == 0)
        return kt <= 16 ? batched_fn<double, 16>(variant) : batched_fn<double, 32>(variant);
    if (a_dtype == 1)
        return kt <= 16 ? batched_fn<float, 16>(variant) : batched_fn<float, 32>(variant);
    if (a_dtype == 2)
        return kt <= 16 ? batched_fn<bf16_t, 16>(variant) : batched_fn<bf16_t, 32>(variant);
    return nullptr;
}

int batched_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus) {
    const void* fn = pick(a_dtype, kt, variant);
    if (!fn) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBW * 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * num_cus;
}

hipError_t launch_batched_setup(int32_t a_dtype, int32_t kt, const BSys* sys, BState* st,
                                int32_t count, int64_t max_n, hipStream_t s) {
    int64_t bx = (max_n + 32 + 255) / 256;
    if (bx > 64) bx = 64;
    if (a_dtype == 0)
        hipLaunchKernelGGL((k_batched_setup<double>), dim3((unsigned)bx, count), dim3(256), 0, s,
                           sys, st, kt);
    else if (a_dtype == 1)
        hipLaunchKernelGGL((k_batched_setup<float>), dim3((unsigned)bx, count), dim3(256), 0, s,
                           sys, st, kt);
    else
        hipLaunchKernelGGL((k_batched_setup<bf16_t>), dim3((unsigned)bx, count), dim3(256), 0, s,
                           sys, st, kt);
    return hipGetLastError();
}

template <typename TA, int KT, bool SPLIT>
static const void* rounds_fn(int variant) {
    if (variant == 1)
        return (const void*)k_rounds<TA, KT, kBW, tiles_per_pass<TA>(KT, 1, !SPLIT), kBU, 1, SPLIT>;
    return (const void*)k_rounds<TA, KT, kBW, tiles_per_pass<TA>(KT, 0), kBU, 2, SPLIT>;
}

template <bool SPLIT>
static const void* pick_rounds_t(int32_t a_dtype, int32_t kt, int variant) {
    if (a_dtype == 0)
        return kt <= 16 ? rounds_fn<double, 16, SPLIT>(variant)
                        : rounds_fn<double, 32, SPLIT>(variant);
    if (a_dtype == 1)
        return kt <= 16 ? rounds_fn<float, 16, SPLIT>(variant)
                        : rounds_fn<float, 32, SPLIT>(variant);
    if (a_dtype == 2)
        return kt <= 16 ? rounds_fn<bf16_t, 16, SPLIT>(variant)
                        : rounds_fn<bf16_t, 32, SPLIT>(variant);
    return nullptr;
}

static const void* pick_rounds(int32_t a_dtype, int32_t kt, int variant, bool split) {
    return split ? pick_rounds_t<true>(a_dtype, kt, variant)
                 : pick_rounds_t<false>(a_dtype, kt, variant);
}

int rounds_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus, bool split) {
    const void* fn = pick_rounds(a_dtype, kt, variant, split);
    if (!fn) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBW * 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * num_cus;
}

hipError_t launch_rounds(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                         hipStream_t s, bool split) {
    const void* fn = pick_rounds(a_dtype, kt, variant, split);
    if (!fn) return hipErrorInvalidValue;
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBW * 64), args, 0, s);
}

template <typename TA, int KT>
static const void* flow_fn(int variant) {
    if (variant == 1)
        return (const void*)k_flow<TA, KT, kBW, tiles_per_pass<TA>(KT, 1, true), kBU, 1>;
    return (const void*)k_flow<TA, KT, kBW, tiles_per_pass<TA>(KT, 0), kBU, 2>;
}

static const void* pick_flow(int32_t a_dtype, int32_t kt, int variant) {
    if (a_dtype == 0) return kt <= 16 ? flow_fn<double, 16>(variant) : flow_fn<double, 32>(variant);
    if (a_dtype == 1) return kt <= 16 ? flow_fn<float, 16>(variant) : flow_fn<float, 32>(variant);
    if (a_dtype == 2) return kt <= 16 ? flow_fn<bf16_t, 16>(variant) : flow_fn<bf16_t, 32>(variant);
    return nullptr;
}

int flow_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus) {
    const void* fn = pick_flow(a_dtype, kt, variant);
    if (!fn) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBW * 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * num_cus;
}

hipError_t launch_flow(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                       hipStream_t s) {
    const void* fn = pick_flow(a_dtype, kt, variant);
    if (!fn) return hipErrorInvalidValue;
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBW * 64), args, 0, s);
}

hipError_t launch_batched(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                          hipStream_t s) {
    const void* fn = pick(a_dtype, kt, variant);
    if (!fn) return hipErrorInvalidValue;
    BatchArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBW * 64), args, 0, s);
}

}  // namespace jac
