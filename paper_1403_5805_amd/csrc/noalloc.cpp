// No-allocation variant of the plain solve, for callers that cannot allocate
// device memory (tight serving loops, harnesses that forbid the allocator).
//
// It runs the vector sweep path of jacobi_solve (one or two right-hand
// sides) with its whole workspace -- control block, reduction slots, partial
// sums, diagonal and the two iterate buffers -- carved out of one file-scope
// device array.  Each device holds its own copy of the array (allocated with
// the code object, kept until the process ends); its device address is taken
// once per device with hipGetSymbolAddress and only that address is ever
// passed to kernels.  The call allocates nothing: no hipMalloc, no pinned
// host memory, no events.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/jacobi.h"
#include "ctx.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = JACOBI_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;
constexpr int64_t kMaxCols = 2;

}  // namespace

// Workspace of jacobi_solve_noalloc on each device.  In host code this name is
// only a stand-in for the device symbol: never pass it to a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace jac {
namespace {

struct NoAllocDevice {
    std::mutex mu;             // serialises calls on this device (one array per device)
    bool ready = false;
    unsigned char* ptr = nullptr;  // device address of `scratch` on this device
    int num_cus = 0;
    Ctl h_ctl;                 // host mirror of the control block (pageable)
};

NoAllocDevice g_dev[kMaxDevices];

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of workspace the vector path needs for this shape.
size_t need_bytes(int32_t a_dtype, int64_t n, int64_t k) {
    const size_t sx = a_dtype == JACOBI_F64 ? 8 : 4;
    const size_t kp = (size_t)kpad_for(k);
    return up256(sizeof(Ctl)) + up256(3 * sizeof(Slot)) + up256(3 * sizeof(double) * kMaxParts) +
           up256(sx * (size_t)n) + 2 * up256(sx * (size_t)n * kp);
}

// Set-up of one device, with that device current: the device address of the
// array and the compute-unit count.
jacobi_status setup_device(NoAllocDevice& d, int dev) {
    if (d.ready) return JACOBI_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
        return JACOBI_ERR_DEVICE;
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus < 1) {
        set_error("hipDeviceGetAttribute(multiprocessor count) failed on device %d", dev);
        return JACOBI_ERR_DEVICE;
    }
    d.ptr = (unsigned char*)p;
    d.num_cus = cus;
    d.ready = true;
    return JACOBI_OK;
}

}  // namespace
}  // namespace jac

extern "C" {

jacobi_status jacobi_solve_noalloc(int64_t n, int64_t k, int32_t a_dtype, const void* A,
                                   int64_t lda, const void* B, int64_t ldb, const void* X0,
                                   void* X, int64_t ldx, const jacobi_options* opt,
                                   hipStream_t stream, jacobi_info* info) {
    using namespace jac;
    try {
        jacobi_info local;
        if (!info) info = &local;
        std::memset(info, 0, sizeof(*info));
        info->status = JACOBI_ERR_INVALID_ARG;
        info->bad_index = -1;
        info->final_delta = -1.0;
        info->rel_residual = -1.0;
        info->device_ms = -1.0;
        jacobi_options o;
        jacobi_options_default(&o);
        if (opt) o = *opt;
        jacobi_status st = check_common(n, k, a_dtype, A, lda, B, ldb, X, ldx, o);
        if (st != JACOBI_OK) return (jacobi_status)(info->status = st);
        if (o.mode != JACOBI_MODE_PLAIN || o.profile != 0 || k > kMaxCols) {
            set_error("jacobi_solve_noalloc: PLAIN mode, profile = 0 and k <= %d only",
                      (int)kMaxCols);
            return (jacobi_status)(info->status = JACOBI_ERR_INVALID_ARG);
        }
        const size_t need = need_bytes(a_dtype, n, k);
        if (need > kScratchBytes) {
            set_error("jacobi_solve_noalloc: n = %lld, k = %lld needs %zu bytes of workspace, "
                      "above the fixed %zu",
                      (long long)n, (long long)k, need, kScratchBytes);
            return (jacobi_status)(info->status = JACOBI_ERR_INVALID_ARG);
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
            set_error("jacobi_solve_noalloc: no usable current device");
            return (jacobi_status)(info->status = JACOBI_ERR_DEVICE);
        }
        NoAllocDevice& d = g_dev[dev];
        std::lock_guard<std::mutex> g(d.mu);
        st = setup_device(d, dev);
        if (st != JACOBI_OK) return (jacobi_status)(info->status = st);
        // carve the array: control block, slots, partial sums, diagonal, iterates
        const size_t sx = a_dtype == JACOBI_F64 ? 8 : 4;
        const size_t kp = (size_t)kpad_for(k);
        unsigned char* p = d.ptr;
        Ctl* ctl = (Ctl*)p;
        p += up256(sizeof(Ctl));
        Slot* slots = (Slot*)p;
        p += up256(3 * sizeof(Slot));
        double* parts = (double*)p;
        p += up256(3 * sizeof(double) * kMaxParts);
        void* diag = p;
        p += up256(sx * (size_t)n);
        void* w0 = p;
        p += up256(sx * (size_t)n * kp);
        void* w1 = p;
        PlainWs w{SweepCtl{ctl, &d.h_ctl, nullptr}, slots, parts, diag, w0, w1, nullptr,
                  nullptr, d.num_cus};
        st = solve_plain_vec(w, n, k, a_dtype, A, lda, B, ldb, X0, X, ldx, o, stream, info);
        info->status = st;
        return st;
    } catch (...) {
        set_error("internal exception");
        if (info) info->status = JACOBI_ERR_INTERNAL;
        return JACOBI_ERR_INTERNAL;
    }
}

}  // extern "C"
