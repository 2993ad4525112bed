/*
 * Serial FP64 Jacobi oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the GPU library; its status codes are its own and merely use
 * the same numeric values as the library's, so that tests can compare them.
 *
 * What it computes (Margaris, Souravlas & Roumeliotis, "Parallel
 * implementations of the Jacobi linear algebraic systems solver", sec. 2):
 *
 *   component update (sec. 2, displayed equation for x_i^(k)):
 *       x_i^(k) = ( beta_i - sum_{j != i} alpha_ij x_j^(k-1) ) / alpha_ii
 *   driver (sec. 2, serial pseudocode):
 *       X^t = X^0; k = 1; while k <= L: sweep; if ||X - X^t|| < tol return X;
 *       k = k + 1; X^t = X.   Terminate when the cap L is reached.
 *
 * Readings taken where the paper is garbled or silent (each also listed in the
 * design notes):
 *   - the pseudocode's update puts beta inside the sum with the wrong sign; the
 *     displayed component equation is used instead;
 *   - the norm: sec. 2 and eq. of sec. 3.1 say Euclidean, the pseudocode leaves
 *     it open; both are offered (ORACLE_NORM_INF = max-norm, ORACLE_NORM_L2);
 *   - the test is a strict "<" against an absolute tolerance, run after every
 *     sweep including sweep L; on success the NEW iterate is returned;
 *   - on the cap, X^(L) is returned with status NOT_CONVERGED;
 *   - a non-finite distance stops the iteration with status DIVERGED (the
 *     paper's own U[0,1] workload overflows; the paper says nothing);
 *   - several right-hand sides: every column is swept, the distance is taken
 *     over all n*k entries, so all columns stop together;
 *   - alpha_ii = 0 fails (sec. 2, the remark after the convergence condition);
 *     non-finite diagonal, B or X^0 entries are rejected as well.
 *
 * Arithmetic: plain IEEE double, separate multiply and add (built with
 * -ffp-contract=off), the j loop ascending, correctly rounded division.
 * Matrices are row-major with a leading dimension.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_NOT_CONVERGED 1
#define ORACLE_DIVERGED 2
#define ORACLE_ERR_INVALID_ARG (-1)
#define ORACLE_ERR_ZERO_DIAGONAL (-2)
#define ORACLE_ERR_NONFINITE_INPUT (-3)
#define ORACLE_ERR_OUT_OF_MEMORY (-4)

#define ORACLE_NORM_INF 0
#define ORACLE_NORM_L2 1

typedef struct {
    int32_t status;
    int32_t iterations;     /* sweeps executed */
    int64_t bad_index;      /* first offending row, or -1 */
    double final_delta;     /* distance of the last executed sweep, -1 if none */
} oracle_info;

/* Input check.  Diagonal first (sec. 2: the method fails when alpha_ii = 0),
 * scanning i ascending; the first bad diagonal decides the status.  Then B and
 * X0, scanning rows ascending. */
static int32_t oracle_check_inputs(int64_t n, int64_t k, const double* A, int64_t lda,
                                   const double* B, int64_t ldb, const double* X0,
                                   int64_t ldx, int64_t* bad) {
    *bad = -1;
    for (int64_t i = 0; i < n; ++i) {
        double d = A[i * lda + i];
        if (d == 0.0) { *bad = i; return ORACLE_ERR_ZERO_DIAGONAL; }
        if (!isfinite(d)) { *bad = i; return ORACLE_ERR_NONFINITE_INPUT; }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t c = 0; c < k; ++c) {
            if (!isfinite(B[i * ldb + c])) { *bad = i; return ORACLE_ERR_NONFINITE_INPUT; }
            if (X0 && !isfinite(X0[i * ldx + c])) { *bad = i; return ORACLE_ERR_NONFINITE_INPUT; }
        }
    }
    return ORACLE_OK;
}

/* One Jacobi update of row i, column c (sec. 2, component equation). */
static double oracle_component(int64_t n, int64_t k, const double* A, int64_t lda,
                               const double* B, int64_t ldb, const double* Xold,
                               int64_t ldo, int64_t i, int64_t c) {
    double s = 0.0;
    const double* row = A + i * lda;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double p = row[j] * Xold[j * ldo + c];
        s = s + p;
    }
    (void)k;
    return (B[i * ldb + c] - s) / row[i];
}

/* Distance between consecutive iterates.  Max-norm, or the Euclidean distance
 * of sec. 3.1 summed in ascending flat order.  Any NaN makes the result NaN. */
static double oracle_distance(int64_t n, int64_t k, const double* Xn, const double* Xt,
                              int32_t norm) {
    int nan_seen = 0;
    double acc = 0.0;
    for (int64_t t = 0; t < n * k; ++t) {
        double d = fabs(Xn[t] - Xt[t]);
        if (isnan(d)) nan_seen = 1;
        if (norm == ORACLE_NORM_L2) {
            acc = acc + d * d;
        } else if (d > acc) {
            acc = d;
        }
    }
    if (nan_seen) return NAN;
    return norm == ORACLE_NORM_L2 ? sqrt(acc) : acc;
}

/* The serial Jacobi driver (sec. 2, pseudocode) for n x k right-hand sides.
 * X0 may be NULL (zero start) and may alias X; X0 and X use leading dim ldx. */
int32_t oracle_jacobi(int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                      int64_t ldb, const double* X0, double* X, int64_t ldx, double tol,
                      int32_t max_iter, int32_t norm, oracle_info* info) {
    oracle_info local;
    if (!info) info = &local;
    info->status = ORACLE_ERR_INVALID_ARG;
    info->iterations = 0;
    info->bad_index = -1;
    info->final_delta = -1.0;
    if (n < 1 || k < 1 || lda < n || ldb < k || ldx < k || !A || !B || !X || isnan(tol) ||
        tol < 0.0 || max_iter < 0 || (norm != ORACLE_NORM_INF && norm != ORACLE_NORM_L2))
        return info->status;

    int32_t st = oracle_check_inputs(n, k, A, lda, B, ldb, X0, ldx, &info->bad_index);
    if (st != ORACLE_OK) { info->status = st; return st; }

    double* Xt = (double*)malloc(sizeof(double) * (size_t)(n * k));
    double* Xn = (double*)malloc(sizeof(double) * (size_t)(n * k));
    if (!Xt || !Xn) {
        free(Xt); free(Xn);
        info->status = ORACLE_ERR_OUT_OF_MEMORY;
        return info->status;
    }
    /* X^t = X^0, zero when none is given (pseudocode input (c)). */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < k; ++c) Xt[i * k + c] = X0 ? X0[i * ldx + c] : 0.0;

    int32_t status = ORACLE_NOT_CONVERGED;
    int32_t iters = 0;
    double delta = -1.0;
    double* result = Xt;
    for (int32_t it = 1; it <= max_iter; ++it) {           /* while k <= L */
        for (int64_t c = 0; c < k; ++c)                   /* step (a) */
            for (int64_t i = 0; i < n; ++i)
                Xn[i * k + c] = oracle_component(n, k, A, lda, B, ldb, Xt, k, i, c);
        delta = oracle_distance(n, k, Xn, Xt, norm);      /* step (b) */
        iters = it;
        if (!isfinite(delta)) { status = ORACLE_DIVERGED; result = Xn; break; }
        if (delta < tol) { status = ORACLE_OK; result = Xn; break; }
        double* tmp = Xt; Xt = Xn; Xn = tmp;              /* steps (c), (d) */
        result = Xt;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < k; ++c) X[i * ldx + c] = result[i * k + c];
    free(Xt); free(Xn);
    info->status = status;
    info->iterations = iters;
    info->final_delta = delta;
    return status;
}

/* One update of selected rows only, from a given previous iterate (the
 * component equation of sec. 2).  Used to check a single sweep of a large
 * system at sampled rows.  out is nrows x k, contiguous. */
void oracle_update_rows(int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                        int64_t ldb, const double* Xold, int64_t ldo, const int64_t* rows,
                        int64_t nrows, double* out) {
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t c = 0; c < k; ++c)
            out[r * k + c] = oracle_component(n, k, A, lda, B, ldb, Xold, ldo, rows[r], c);
}

/* Same as oracle_update_rows with A stored in float (the promoted FP32
 * system: every float is exactly representable in double). */
void oracle_update_rows_f32(int64_t n, int64_t k, const float* A, int64_t lda, const double* B,
                            int64_t ldb, const double* Xold, int64_t ldo, const int64_t* rows,
                            int64_t nrows, double* out) {
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        const float* row = A + i * lda;
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double p = (double)row[j] * Xold[j * ldo + c];
                s = s + p;
            }
            out[r * k + c] = (B[i * ldb + c] - s) / (double)row[i];
        }
    }
}

/* Residual R = B - A X, every term in order j ascending (plain definition). */
void oracle_residual(int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                     int64_t ldb, const double* X, int64_t ldx, double* R, int64_t ldr) {
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double p = A[i * lda + j] * X[j * ldx + c];
                s = s + p;
            }
            R[i * ldr + c] = B[i * ldb + c] - s;
        }
    }
}

/* Round a double to the nearest bfloat16 value (8 significant bits, the
 * exponent range of binary32), ties to even, returned as a double.  Written
 * from the definition with frexp/ldexp: x = m * 2^e, 0.5 <= |m| < 1; the
 * quantum of a normal bf16 at that binade is 2^(e-8), and below 2^-126 the
 * quantum is fixed at 2^-133. */
double oracle_round_bf16(double x) {
    if (isnan(x) || isinf(x) || x == 0.0) return x;
    int e;
    (void)frexp(x, &e);
    int q = e - 8;                       /* exponent of one unit in the last place */
    if (q < -133) q = -133;              /* subnormal bf16 range */
    double scaled = ldexp(x, -q);        /* exact: only the exponent changes */
    double r = nearbyint(scaled);        /* default rounding mode: to nearest, ties to even */
    double y = ldexp(r, q);
    /* largest finite bf16: (2 - 2^-7) * 2^127; anything rounding above it is inf */
    double maxbf = ldexp(255.0, 120);
    if (fabs(y) > maxbf) return x > 0 ? INFINITY : -INFINITY;
    return y;
}

void oracle_round_bf16_array(const double* in, double* out, int64_t count) {
    for (int64_t t = 0; t < count; ++t) out[t] = oracle_round_bf16(in[t]);
}
