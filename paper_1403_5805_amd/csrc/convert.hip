// FP64 -> FP32 / BF16 copy of A for the reduced-precision sweeps of the
// refinement (round to nearest, ties to even, from FP64 in one rounding).
#include <math.h>
#include <stdint.h>

#include "internal.h"
#include "round.h"

namespace jac {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));


// One row per workgroup iteration; with aligned rows each thread converts 4
// consecutive values (two 16-byte loads, one 8- or 16-byte store).
template <typename TO, bool VEC>
__global__ void k_convert(const double* __restrict__ A, int64_t lda, int64_t n,
                          TO* __restrict__ out, int64_t ldo) {
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const double* a = A + i * lda;
        TO* o = out + i * ldo;
        int64_t j0 = 0;
        if (VEC) {
            // UN groups of 4 per thread and iteration keep 2 * UN loads in flight
            constexpr int UN = 4;
            const int64_t n4 = n / 4 * 4;
            const int64_t step = 4 * (int64_t)blockDim.x;
            for (int64_t jb = 4 * (int64_t)threadIdx.x; jb < n4; jb += UN * step) {
                f64x2 v[UN][2];
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int64_t j = jb + u * step;
                    if (j < n4) {
                        const f64x2* src = reinterpret_cast<const f64x2*>(a + j);
                        v[u][0] = __builtin_nontemporal_load(src);
                        v[u][1] = __builtin_nontemporal_load(src + 1);
                    }
                }
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const int64_t j = jb + u * step;
                    if (j >= n4) continue;
                    if constexpr (sizeof(TO) == 4) {
                        const f32x4 w = {narrow<TO>(v[u][0].x), narrow<TO>(v[u][0].y),
                                         narrow<TO>(v[u][1].x), narrow<TO>(v[u][1].y)};
                        __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(o + j));
                    } else {
                        // element j in the low half of the first word (little endian)
                        const uint32_t lo = (uint32_t)narrow<TO>(v[u][0].x) |
                                            ((uint32_t)narrow<TO>(v[u][0].y) << 16);
                        const uint32_t hi = (uint32_t)narrow<TO>(v[u][1].x) |
                                            ((uint32_t)narrow<TO>(v[u][1].y) << 16);
                        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
                        const u32x2 w = {lo, hi};
                        __builtin_nontemporal_store(w, reinterpret_cast<u32x2*>(o + j));
                    }
                }
            }
            j0 = n4;
        }
        for (int64_t j = j0 + threadIdx.x; j < n; j += blockDim.x) o[j] = narrow<TO>(a[j]);
    }
}

hipError_t launch_convert(const double* A, int64_t lda, int64_t n, int32_t to_dtype, void* out,
                          int64_t ldo, hipStream_t s) {
    const int threads = 256;
    const int blocks = (int)(n < 16384 ? n : 16384);
    const size_t eo = to_dtype == 1 ? 4 : 2;
    const bool vec = (uintptr_t)A % 16 == 0 && lda % 2 == 0 && (uintptr_t)out % (4 * eo) == 0 &&
                     ldo % 4 == 0;
    if (to_dtype == 1) {
        if (vec)
            hipLaunchKernelGGL((k_convert<float, true>), dim3(blocks), dim3(threads), 0, s, A, lda,
                               n, (float*)out, ldo);
        else
            hipLaunchKernelGGL((k_convert<float, false>), dim3(blocks), dim3(threads), 0, s, A,
                               lda, n, (float*)out, ldo);
    } else if (to_dtype == 2) {
        if (vec)
            hipLaunchKernelGGL((k_convert<uint16_t, true>), dim3(blocks), dim3(threads), 0, s, A,
                               lda, n, (uint16_t*)out, ldo);
        else
            hipLaunchKernelGGL((k_convert<uint16_t, false>), dim3(blocks), dim3(threads), 0, s, A,
                               lda, n, (uint16_t*)out, ldo);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The first residual of a refinement that starts from x = 0: r = B exactly
// (B - A 0), kept in FP64 (r64) and rounded to FP32 (rlo), leading dimension
// kp, columns [0, k).
__global__ void k_rhs_residual(const double* __restrict__ B, int64_t ldb, int64_t n, int k,
                               int64_t kp, double* __restrict__ r64, float* __restrict__ rlo) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * k; e += stride) {
        const int64_t i = e / k;
        const int c = (int)(e % k);
        const double b = B[i * ldb + c];
        r64[i * kp + c] = b;
        rlo[i * kp + c] = (float)b;
    }
}

// The first inner sweep from d = 0: every off-diagonal term multiplies zero,
// so d^(1) = r / a_ii (the sweep's IEEE division of the same FP32 operands),
// written without a pass over A_lo; padding columns [k, kp) are zero.
__global__ void k_first_sweep(const float* __restrict__ rlo, const float* __restrict__ diag,
                              int64_t n, int k, int64_t kp, float* __restrict__ d) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * kp; e += stride) {
        const int64_t i = e / kp;
        const int c = (int)(e % kp);
        d[e] = c < k ? rlo[e] / diag[i] : 0.0f;
    }
}

hipError_t launch_first_sweep(const float* rlo, const float* diag, int64_t n, int32_t k,
                              int64_t kp, float* d, hipStream_t s) {
    const int threads = 256;
    int64_t blocks = (n * kp + threads - 1) / threads;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_first_sweep, dim3((unsigned)blocks), dim3(threads), 0, s, rlo, diag, n,
                       k, kp, d);
    return hipGetLastError();
}

hipError_t launch_rhs_residual(const double* B, int64_t ldb, int64_t n, int32_t k, int64_t kp,
                               double* r64, float* rlo, hipStream_t s) {
    const int threads = 256;
    int64_t blocks = (n * k + threads - 1) / threads;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_rhs_residual, dim3((unsigned)blocks), dim3(threads), 0, s, B, ldb, n, k,
                       kp, r64, rlo);
    return hipGetLastError();
}

}  // namespace jac
