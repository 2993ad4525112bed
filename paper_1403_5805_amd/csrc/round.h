// Rounding of FP64 values to the reduced-precision copy of A used by the
// refinement's inner sweeps: round to nearest, ties to even, in one rounding
// from FP64.  Shared by the conversion kernel and the first residual pass,
// which writes the same copy while it streams A.
#pragma once

#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace jac {

__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x) {
    if (isnan(x)) return (uint16_t)0x7fc0u;
    const double ax = fabs(x);
    const uint32_t sign = (x < 0.0 || (x == 0.0 && signbit(x))) ? 0x8000u : 0u;
    double r;
    if (ax < 0x1.0p-126) {
        // subnormal bf16 range: the quantum is 2^-133
        r = __builtin_rint(ax * 0x1.0p133) * 0x1.0p-133;
    } else {
        // keep 8 significant bits of the double (7 explicit): round at bit 45
        uint64_t u = (uint64_t)__double_as_longlong(ax);
        const uint64_t lsb = (u >> 45) & 1u;
        u += (((uint64_t)1 << 44) - 1) + lsb;
        u &= ~(((uint64_t)1 << 45) - 1);
        r = __longlong_as_double((long long)u);
    }
    // r is exactly a bf16 magnitude (or >= 2^128 -> overflow to inf)
    uint32_t fb;
    if (r >= 0x1.0p128)
        fb = 0x7f800000u;
    else
        fb = __float_as_uint((float)r);
    return (uint16_t)(sign | (fb >> 16));
}

template <typename TO>
__device__ __forceinline__ TO narrow(double x);
template <>
__device__ __forceinline__ float narrow<float>(double x) {
    return (float)x;
}
template <>
__device__ __forceinline__ uint16_t narrow<uint16_t>(double x) {
    return f64_to_bf16_rne(x);
}

}  // namespace jac
