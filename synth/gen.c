/*
 * Seeded synthetic inputs for the Jacobi solver: dense systems A X = B.
 *
 * This module only draws inputs.  It holds none of the Jacobi method's
 * arithmetic and is shared by the tests, the benchmark and the oracle checks.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: the value for (seed, stream, index) is the finalizer applied to
 * key(seed, stream) + (index + 1) * gamma, so any entry can be drawn
 * independently and the result does not depend on the thread count.
 *
 * Workload recipes:
 *   synth_dominant*: off-diagonals iid U[-1,1]; rowsum_i = sum_{j != i}|a_ij|
 *     (j ascending); the diagonal is rowsum_i + U[lo,hi] (additive margin) or
 *     rowsum_i * (1 + U[lo,hi]) (multiplicative margin), which makes A
 *     strictly diagonally dominant (the paper's sufficient condition, sec. 2);
 *     X_true iid U[-1,1]; B = A X_true summed in FP64, j ascending.
 *     Mode 2 draws the off-diagonals iid U[0,1] instead (the sign pattern of
 *     the paper's experiments, sec. 4) with the multiplicative margin: with
 *     a_ii = 1.05 rowsum_i every row of |D^-1 (A - D)| sums to 1/1.05, so the
 *     Jacobi matrix has spectral radius 0.952 and the iteration converges
 *     slowly (hundreds of sweeps to 1e-10).
 *   synth_paper_uniform: A, B and X iid U[0,1], as in the paper's experiments
 *     (sec. 4); such matrices are not diagonally dominant.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define SYNTH_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t synth_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t synth_key(uint64_t seed, uint64_t stream) {
    return synth_mix(seed ^ (stream * 0xD1B54A32D192ED03ULL));
}

static inline uint64_t synth_draw(uint64_t key, uint64_t idx) {
    return synth_mix(key + (idx + 1) * SYNTH_GAMMA);
}

static inline double synth_unit(uint64_t key, uint64_t idx) {
    return (double)(synth_draw(key, idx) >> 11) * 0x1.0p-53;
}

static inline double synth_range(uint64_t key, uint64_t idx, double lo, double hi) {
    return lo + (hi - lo) * synth_unit(key, idx);
}

enum { STREAM_OFFDIAG = 1, STREAM_MARGIN = 2, STREAM_XTRUE = 3, STREAM_SIZES = 4,
       STREAM_ARRIVALS = 5, STREAM_PAPER_A = 6, STREAM_PAPER_B = 7, STREAM_PAPER_X = 8 };

uint64_t synth_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
    return synth_draw(synth_key(seed, stream), idx);
}

double synth_uniform(uint64_t seed, uint64_t stream, uint64_t idx, double lo, double hi) {
    return synth_range(synth_key(seed, stream), idx, lo, hi);
}

static void synth_xtrue(int64_t n, int64_t k, uint64_t seed, double* X) {
    uint64_t kx = synth_key(seed, STREAM_XTRUE);
    for (int64_t t = 0; t < n * k; ++t) X[t] = synth_range(kx, (uint64_t)t, -1.0, 1.0);
}

static double synth_diag(double rowsum, uint64_t km, int64_t i, int32_t mode, double lo,
                         double hi) {
    double u = synth_range(km, (uint64_t)i, lo, hi);
    return mode == 0 ? rowsum + u : rowsum * (1.0 + u);
}

static inline double synth_offdiag(uint64_t ka, uint64_t idx, int32_t mode) {
    return mode == 2 ? synth_range(ka, idx, 0.0, 1.0) : synth_range(ka, idx, -1.0, 1.0);
}

/* FP64 system.  A is n x lda (row-major), X_true and B are n x k contiguous.
 * mode 0: additive margin, mode 1: multiplicative margin, mode 2:
 * non-negative off-diagonals with the multiplicative margin. */
void synth_dominant(int64_t n, int64_t k, uint64_t seed, int32_t mode, double lo, double hi,
                    double* A, int64_t lda, double* Xtrue, double* B) {
    uint64_t ka = synth_key(seed, STREAM_OFFDIAG);
    uint64_t km = synth_key(seed, STREAM_MARGIN);
    synth_xtrue(n, k, seed, Xtrue);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* row = A + i * lda;
        double rowsum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double a = synth_offdiag(ka, (uint64_t)(i * n + j), mode);
            row[j] = a;
            rowsum += fabs(a);
        }
        row[i] = synth_diag(rowsum, km, i, mode, lo, hi);
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += row[j] * Xtrue[j * k + c];
            B[i * k + c] = s;
        }
    }
}

/* FP32 system of record: A32 = fl32(A64) with A64 drawn exactly as in
 * synth_dominant, B32 = fl32(A32 X_true) with the product summed in FP64. */
void synth_dominant_f32(int64_t n, int64_t k, uint64_t seed, int32_t mode, double lo, double hi,
                        float* A, int64_t lda, double* Xtrue, float* B) {
    uint64_t ka = synth_key(seed, STREAM_OFFDIAG);
    uint64_t km = synth_key(seed, STREAM_MARGIN);
    synth_xtrue(n, k, seed, Xtrue);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float* row = A + i * lda;
        double rowsum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double a = synth_offdiag(ka, (uint64_t)(i * n + j), mode);
            row[j] = (float)a;
            rowsum += fabs(a);
        }
        row[i] = (float)synth_diag(rowsum, km, i, mode, lo, hi);
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += (double)row[j] * Xtrue[j * k + c];
            B[i * k + c] = (float)s;
        }
    }
}

/* The paper's experimental inputs (sec. 4): A, B and X^0 iid U[0,1]. */
void synth_paper_uniform(int64_t n, uint64_t seed, double* A, double* B, double* X0) {
    uint64_t ka = synth_key(seed, STREAM_PAPER_A);
    uint64_t kb = synth_key(seed, STREAM_PAPER_B);
    uint64_t kx = synth_key(seed, STREAM_PAPER_X);
    for (int64_t t = 0; t < n * n; ++t) A[t] = synth_unit(ka, (uint64_t)t);
    for (int64_t i = 0; i < n; ++i) {
        B[i] = synth_unit(kb, (uint64_t)i);
        X0[i] = synth_unit(kx, (uint64_t)i);
    }
}

/* Sizes drawn log-uniformly: floor(exp(U[ln lo, ln hi])), clamped to [lo, hi]. */
void synth_log_uniform_sizes(int64_t count, uint64_t seed, int64_t lo, int64_t hi,
                             int64_t* out) {
    uint64_t ks = synth_key(seed, STREAM_SIZES);
    double a = log((double)lo), b = log((double)hi);
    for (int64_t t = 0; t < count; ++t) {
        int64_t v = (int64_t)floor(exp(synth_range(ks, (uint64_t)t, a, b)));
        if (v < lo) v = lo;
        if (v > hi) v = hi;
        out[t] = v;
    }
}

/* Poisson arrival times at rate lambda: exponential gaps -ln(1-u)/lambda. */
void synth_poisson_arrivals(int64_t count, uint64_t seed, double rate, double* t_out) {
    uint64_t kt = synth_key(seed, STREAM_ARRIVALS);
    double t = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        t += -log(1.0 - synth_unit(kt, (uint64_t)i)) / rate;
        t_out[i] = t;
    }
}
