// Achievable read bandwidth of the device's HBM (gfx950).
//
// A read-only streaming kernel: every thread reads 16-byte pieces of the
// buffer with non-temporal loads, U of them in flight, in a grid-stride loop
// over the whole buffer, and folds them into one word per workgroup (kept in
// a file-scope sink so the loads are not removed).  The same load width and
// hint as the vector sweep's stream of A, with nothing else to do: the
// ceiling the sweep is measured against, beside the published 8 TB/s.  The
// host entry tries a few launch shapes and keeps the fastest.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ctx.h"

namespace jac {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeMaxGrid = 1 << 14;
__device__ uint32_t probe_sink[kProbeMaxGrid];

template <int U>
__global__ __launch_bounds__(256) void k_stream_read(const u32x4* __restrict__ p, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (U - 1) * stride < n16; i += U * stride) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // one word per workgroup: lane 0 of every wave folds in atomically
    for (int o = 32; o >= 1; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(&probe_sink[blockIdx.x], acc);
}

}  // namespace

}  // namespace jac

using namespace jac;

extern "C" jacobi_status jacobi_stream_probe(const void* buf, int64_t bytes, int32_t reps,
                                             hipStream_t stream, double* gbps,
                                             int32_t* wg_per_cu) {
    if (!buf || bytes < 16 || reps < 1 || !gbps || ((uintptr_t)buf % 16) != 0) {
        set_error("stream probe: buffer (16-byte aligned, >= 16 bytes), reps >= 1, output");
        return JACOBI_ERR_INVALID_ARG;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        set_error("stream probe: no device");
        return JACOBI_ERR_DEVICE;
    }
    const int cus = std::max(1, prop.multiProcessorCount);
    const int64_t n16 = bytes / 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        set_error("stream probe: event creation failed");
        return JACOBI_ERR_DEVICE;
    }
    double best = 0.0;
    int best_w = 0;
    hipError_t err = hipSuccess;
    for (const int w : {2, 4, 8, 16}) {
        const int grid = std::min(kProbeMaxGrid, cus * w);
        // one launch to settle clocks and caches, then the timed ones
        for (int r = 0; r <= reps && err == hipSuccess; ++r) {
            if (r > 0) err = hipEventRecord(e0, stream);
            if (err == hipSuccess) {
                hipLaunchKernelGGL(k_stream_read<4>, dim3(grid), dim3(256), 0, stream,
                                   (const u32x4*)buf, n16);
                err = hipGetLastError();
            }
            if (r == 0) continue;
            if (err == hipSuccess) err = hipEventRecord(e1, stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && ms > 0.f) {
                const double g = (double)n16 * 16.0 / (ms * 1e-3) / 1e9;
                if (g > best) {
                    best = g;
                    best_w = w;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) {
        set_error("stream probe: %s", hipGetErrorString(err));
        return JACOBI_ERR_DEVICE;
    }
    *gbps = best;
    if (wg_per_cu) *wg_per_cu = best_w;
    return JACOBI_OK;
}
