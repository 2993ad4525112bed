// Solver context: per-device workspaces reused across calls.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jacobi.h"
#include "internal.h"

namespace jac {

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t b);
    void release();
};

// Barrier count and slot rotation left by the last fused small-system
// launch on a control block (see k_small_reg).
struct SmallChain {
    bool ready = false;
    uint32_t bar_base = 0;
    int32_t slot_base = 0;
};

// Variant of a batched launch; every variant gives bitwise the same results.
struct BatchTune {
    int shape = 1;   // 0 wide (two workgroups per CU), 1 deep (one)
    int sched = 1;   // 0 planned, 1 lockstep, 2 dataflow
    int groups = 1;  // lockstep: XCD groups of work items (1 = none)
    int per_wg = 8;  // lockstep: work items per workgroup and round
    int csplit = 1;  // lockstep, one system: column chunks (split-K); 1 = none
};

// Grow-only pinned, device-mapped host buffer for the small per-call
// descriptor uploads and outcome read-backs.  They are moved by a copy kernel
// on the caller's stream rather than by the DMA engines, so they never queue
// behind large host transfers running on other streams.
struct HostStage {
    void* h = nullptr;  // host address
    void* d = nullptr;  // device address of the same memory
    size_t bytes = 0;
    hipError_t ensure(size_t b);
    void release();
};

}  // namespace jac

struct jacobi_ctx {
    int device = 0;
    int num_cus = 256;
    std::mutex mu;
    jac::Ctl* ctl = nullptr;      // device control block
    jac::Slot* slots = nullptr;   // device reduction slots [3]
    double* parts = nullptr;      // device partial sums [3][kMaxParts]
    jac::Ctl* h_ctl = nullptr;    // pinned host mirror of ctl
    jac::Ctl* h_ctl_dev = nullptr;  // its device-visible address (null: not mapped)
    // State of ctl and slots left by the last fused small-system launch, so
    // that the next one can skip k_init_ctl: the barrier count it ended at and
    // the slot rotation that leaves its first slot clear (ready = false after
    // any other use of ctl, a timeout or invalid input: initialise again).
    jac::SmallChain small_chain;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    std::vector<hipEvent_t> prof_ev;
    // plain solve
    jac::DevBuf diag, w0, w1;
    // refinement
    jac::DevBuf alo, diag_lo, xa, xb, r64, rlo, d0, d1, scal;
    // batched solver: per-system buffers and descriptors
    jac::DevBuf bws, bmeta;
    // batched launch timing: the call (setup included) and its persistent kernel
    hipEvent_t bev_begin = nullptr, bev_kernel = nullptr, bev_end = nullptr;
    // batched FP64 residual: descriptors, transposed iterate, pinned outcomes
    jac::DevBuf rmeta, xT;
    // staging for descriptor uploads and outcome read-backs
    jac::HostStage stage;
    // batched launch variant measured fastest per class of batch (also kept
    // in a cache file); `warm` holds the empty tables of the warm-up launches
    std::map<uint64_t, jac::BatchTune> batched_tune;
    bool tune_loaded = false;
    std::string tune_path;
    jac::DevBuf warm;
    // dataflow schedule: queue ring (entries tagged with the launch's gen)
    jac::DevBuf fring;
    uint32_t flow_gen = 0;
};

namespace jac {

void set_error(const char* fmt, ...);
jacobi_status ctx_init(jacobi_ctx* c, int device);
void ctx_release(jacobi_ctx* c);
jacobi_ctx* default_ctx(jacobi_status* st);
jacobi_status check_common(int64_t n, int64_t k, int32_t a_dtype, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* X, int64_t ldx,
                           const jacobi_options& o);
// Control block of a run of sweeps: the device block, its host mirror and
// the events of per-sweep profiling (null: profiling unavailable).
struct SweepCtl {
    Ctl* ctl;
    Ctl* h_ctl;
    std::vector<hipEvent_t>* prof_ev;
};
inline SweepCtl sweep_ctl(jacobi_ctx* c) { return SweepCtl{c->ctl, c->h_ctl, &c->prof_ev}; }

jacobi_status run_sweeps(const SweepCtl& sc, int32_t a_dtype, SweepArgs args,
                         const LaunchCfg& cfg, void* bufs[2], int32_t cap, int32_t sync_every,
                         int profile, hipStream_t s, uint32_t* stop_out, int32_t* k_out,
                         double* delta_out, double* xmax_out, double* kernel_ms,
                         int64_t* launches);

// Workspace of a plain solve on the vector sweep kernel (device pointers
// except h_ctl): diag holds n elements of the iterate type, w0 and w1 n x kp.
struct PlainWs {
    SweepCtl sc;
    Slot* slots;        // [3]
    double* parts;      // [3][kMaxParts]
    void* diag;
    void* w0;
    void* w1;
    hipEvent_t ev_begin, ev_end;  // null: device_ms is not measured (-1)
    int num_cus;
    // device-visible address of sc.h_ctl, or null (then the small-system
    // kernel's outcome is copied back from sc.ctl)
    Ctl* h_ctl_dev = nullptr;
    SmallChain* chain = nullptr;  // the context's, or null: initialise every time
};

// Padded column count of the iterate buffers for k right-hand sides.
int kpad_for(int64_t k);
// Fewest right-hand sides a plain solve of this A type runs on MFMA tiles
// (fewer stay on the vector sweep kernel).
int mfma_min_cols(int32_t a_dtype);

// Plain Jacobi solve on the vector sweep kernel with the given workspace
// (no allocation).  Arguments as jacobi_solve; the caller has validated them.
jacobi_status solve_plain_vec(const PlainWs& w, int64_t n, int64_t k, int32_t a_dtype,
                              const void* A, int64_t lda, const void* B, int64_t ldb,
                              const void* X0, void* X, int64_t ldx, const jacobi_options& o,
                              hipStream_t s, jacobi_info* info);

// One system of a batched FP64 residual pass (device pointers; x, d, xnew,
// r64 and rlo are n x ldx row-major).  xT is workspace of
// resid_xT_bytes(n, k) bytes.
struct ResidItem {
    int64_t n, k, ldx;
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    const double* x;
    const float* d;
    double* xnew;
    double* r64;
    float* rlo;
    double* xT;
    double bnorm, rel;
};

size_t resid_xT_bytes(int64_t n, int64_t k);
// Residual pass of `count` systems (k <= 32 each); out[i] receives system i's
// outcome (host array).  Waits for completion.
jacobi_status run_resid(jacobi_ctx* c, int32_t count, const ResidItem* items, hipStream_t s,
                        RState* out);

// A reduced-precision copy of an FP64 A built ahead of the solves (a prepared
// matrix): refinement then neither converts A nor gathers its diagonal.
struct PreparedLo {
    const void* alo;     // lo_dtype values, n x ld_lo
    int64_t ld_lo;
    const float* diag;   // diagonal of alo, widened to FP32
    int32_t lo_dtype;    // JACOBI_F32 or JACOBI_BF16
};

jacobi_status solve_refine(jacobi_ctx* c, int64_t n, int64_t k, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* X0, void* X, int64_t ldx,
                           const jacobi_options& o, hipStream_t s, jacobi_info* info,
                           const PreparedLo* pre = nullptr);

}  // namespace jac
