// Internal declarations shared by the kernels and the host runtime of libjacobi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace jac {

// Stop codes written by the device into Ctl::stop.
enum : uint32_t {
    STOP_RUNNING = 0,
    STOP_CONVERGED = 1,  // distance met the test (or residual target reached)
    STOP_DIVERGED = 2,   // distance NaN/Inf
    STOP_INVALID = 3,    // validation failed: sweeps must not run
    STOP_TIMEOUT = 4     // a grid barrier wait of the small-system kernel timed out
};

// How the decider judges a sweep.
enum : int32_t {
    TEST_ABS = 0,     // distance < tol (strict), sec. 2 pseudocode step (b)
    TEST_REL = 1,     // distance <= rel * max|x_new| (inner refinement sweeps)
    TEST_RESID = 2    // residual pass: ||r||_2 < rel * ||b||_2, or ||r||_2 == 0
};

// Per-solve control block on the device.  The host copies it back once per
// group of sweeps.
struct alignas(64) Ctl {
    uint32_t stop;           // STOP_*
    int32_t stop_sweep;      // sweep number at which stop was decided
    int32_t sweeps_done;     // last sweep whose decision ran
    int32_t timeout;         // host mirror only: a barrier wait of k_small_reg timed out
    uint64_t last_delta_bits;  // double bits of the last decided distance
    uint64_t last_xmax_bits;   // double bits of max|x_new| of the last sweep
    int64_t bad_zero;        // min row with alpha_ii == 0         (INT64_MAX if none)
    int64_t bad_nonfinite;   // min row with non-finite alpha_ii   (INT64_MAX if none)
    int64_t bad_rhs;         // min row with non-finite B or X0    (INT64_MAX if none)
    uint32_t setup_ticket;
    uint32_t bar;            // grid barrier arrivals of the small-system kernel (all sweeps)
};

// Per-launch reduction slot (three of them, launch seq uses slot seq % 3).
struct alignas(64) Slot {
    uint64_t dmax_bits;  // atomic max of |x_new - x_old| (double bits, >= 0; NaN wins)
    uint64_t xmax_bits;  // atomic max of |x_new|
    uint32_t ticket;     // workgroups finished
    uint32_t pad;
};

constexpr int kMaxParts = 1 << 16;  // per-slot partial sums (one per workgroup)

// Arguments of one sweep (or residual) launch.
struct SweepArgs {
    const void* A;
    int64_t lda;
    const void* B;     // TX, n x k (ldb)
    int64_t ldb;
    const void* xin;   // TX, n x k (ldin)
    int64_t ldin;
    void* xout;        // TX (sweep) or double (residual: updated x)
    int64_t ldout;
    const void* diag;  // TX[n]
    int64_t n;
    int32_t k;
    int32_t sweep;     // logical sweep number reported to the host, 1-based
    int32_t seq;       // launch number within the current phase (selects the slot)
    int32_t aligned;   // 1: rows of A are 16-byte aligned (vector loads allowed)
    int64_t chunk;     // columns of x staged in LDS at once
    int64_t rows_per_wg;  // rows owned by one workgroup (contiguous block)
    int32_t kpad;      // leading dimension of the iterate buffers (>= k)
    Ctl* ctl;
    Slot* slots;       // [3], launch seq publishes into slot seq % 3
    double* parts;     // [3][kMaxParts]
    double tol;        // TEST_ABS threshold
    double rel;        // TEST_REL / TEST_RESID factor
    double bnorm;      // TEST_RESID: ||b||_2
    int32_t test;      // TEST_*
    int32_t norm;      // 0 inf, 1 l2
    // residual pass extras
    const float* dlt;  // correction d (float, ld k) added to xin while staging, or null
    double* r64;       // residual out (double, ld k)
    float* rlo;        // residual out (float, ld k)
    // residual pass: also write A rounded to FP32 / BF16 (lo_dtype 1 / 2)
    // into alo (ld_lo), or nothing when alo is null
    void* alo;
    int64_t ld_lo;
    int32_t lo_dtype;
};

// Arguments of the small-system kernel (k_small, small.hip): every sweep of
// one system in one launch.  buf0 holds x^(0) (n x kp, row-major, from
// k_setup), sweep r writes buf[r & 1]; slots and parts as for the vector
// kernel; cap = max_iter.
struct SmallArgs {
    const void* A;
    int64_t lda;
    const void* B;     // TX, n x k (ldb)
    int64_t ldb;
    const void* diag;  // TX[n]
    int64_t n;
    int32_t k;
    int32_t cap;
    void* buf0;
    void* buf1;
    Ctl* ctl;
    Slot* slots;       // [3]
    double* parts;     // [3][kMaxParts]
    double tol;        // TEST_ABS threshold
    int32_t norm;      // 0 inf, 1 l2
    int32_t aligned;   // rows of A 16-byte aligned (k_small_reg's one-time load)
    int64_t spin_limit;  // wall-clock ticks before a barrier wait gives up
    // k_small_reg only, fused = 1: the kernel also takes the set-up's place
    // (a_ii from A, x^(0) read from X0 or zero, the input checks) and writes
    // X itself; hctl (if not null, device-visible host memory) receives the
    // final control block.  Needs cap >= 1.
    int32_t fused;
    int32_t slot_base;  // fused: sweep r uses slot (slot_base + r) % 3
    uint32_t bar_base;  // fused: barrier r completes at count bar_base + G r (wrapping)
    int32_t atomic_max_grid;  // k_small_reg: grids up to this gather maxima with atomics
    const void* X0;    // TX, n x k packed (ldx0 = k, 16-byte aligned), or null: x^(0) = 0
    int64_t ldx0;
    void* X;           // TX, n x k (ldx)
    int64_t ldx;
    Ctl* hctl;
};
// Largest n whose iterate (n x kp of the launch's iterate type) fits the
// kernel's LDS; grid <= resident workgroups (one per CU).
int64_t small_max_rows(int32_t a_dtype, int32_t kp);
hipError_t launch_small(int32_t a_dtype, const SmallArgs& a, int kp, bool aligned, int grid,
                        hipStream_t s);
// Default of SmallArgs::atomic_max_grid: k_small_reg grids of at most this
// many workgroups gather the distance's maximum with atomics in the rotating
// slots; larger ones store one word per workgroup and leave the slots
// untouched (the host advances the slot rotation only after the former).
constexpr int kSmallAtomicMaxGrid = 64;
// Register-resident variant (k_small_reg): np = 16-byte pieces per lane and
// row (1, 2, 4, 8, 12 or 16; 0 if n needs more than 16), rows per wave it holds.
int small_reg_np(int32_t a_dtype, int64_t n);
// waves = 4 or 8 per workgroup (8 only for np <= 8); 0 rows: no such variant.
int small_reg_rows_per_wave(int32_t a_dtype, int kp, int np, int waves);
hipError_t launch_small_reg(int32_t a_dtype, const SmallArgs& a, int kp, int np, int waves,
                            int grid, hipStream_t s);

// Host-side launch configuration chosen per call.
struct LaunchCfg {
    int waves;       // waves per workgroup (all waves share each row)
    int rows;        // rows accumulated together by every wave
    int unroll;      // 16-byte loads per row kept in flight by every lane
    int64_t chunk;   // columns of x staged in LDS at once
    int grid;        // workgroups along rows
    int64_t rows_per_wg;  // contiguous rows owned by one workgroup
};

// Kernel launchers (defined in sweep.hip).  Return hipSuccess or the launch error.
hipError_t launch_init_ctl(Ctl* ctl, Slot* slots, int full, hipStream_t s);
hipError_t launch_setup(int32_t a_dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                        const void* X0, int64_t ldx0, int64_t n, int32_t k, int32_t kpad,
                        void* diag, void* w0, void* w1, Ctl* ctl, hipStream_t s);
hipError_t launch_sweep(int32_t a_dtype, const SweepArgs& a, const LaunchCfg& cfg,
                        hipStream_t s);
hipError_t launch_residual(const SweepArgs& a, const LaunchCfg& cfg, hipStream_t s);
// Stop decision for launch a.seq (sweep a.sweep) of a phase, whose grid had
// `total` workgroups, when no later launch takes it; records it in a.ctl.
hipError_t launch_decide(const SweepArgs& a, int total, hipStream_t s);
hipError_t launch_convert(const double* A, int64_t lda, int64_t n, int32_t to_dtype, void* out,
                          int64_t ldo, hipStream_t s);
// r = B (the residual at x = 0) into r64 (FP64) and rlo (FP32), ld kp.
hipError_t launch_rhs_residual(const double* B, int64_t ldb, int64_t n, int32_t k, int64_t kp,
                               double* r64, float* rlo, hipStream_t s);
hipError_t launch_gather_diag(int32_t a_dtype, const void* A, int64_t lda, int64_t n,
                              void* out, hipStream_t s);
hipError_t launch_bnorm(const double* B, int64_t ldb, int64_t n, int32_t k, double* out,
                        hipStream_t s);
// d = r / a_ii (FP32, n x kp, padding zero): the refinement's first inner
// sweep from d = 0, which needs no pass over A_lo.
hipError_t launch_first_sweep(const float* rlo, const float* diag, int64_t n, int32_t k,
                              int64_t kp, float* d, hipStream_t s);
hipError_t launch_copy_rows(int32_t elem_bytes, const void* src, int64_t lds, void* dst,
                            int64_t ldd, int64_t n, int32_t k, hipStream_t s);
hipError_t launch_zero_rows(int32_t elem_bytes, void* dst, int64_t ldd, int64_t n, int32_t k,
                            hipStream_t s);

// ---------------------------------------------------------------------------
// Batched persistent sweeps (MFMA tiles), one launch for many systems.

// Per-system descriptor (device copy).  A is FP64, FP32 or BF16 (the
// launch's dtype); B, X, the iterate buffers and the diagonal are FP64 for an
// FP64 launch and FP32 otherwise (the iterate type).  The iterate buffers
// hold X transposed: kt rows (16 or 32) of xld >= n values, padding zero.
struct BSys {
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    void* X;           // caller's output (ldx), written once at the end
    int64_t ldx;
    const void* X0;    // caller's initial approximation (ldx), or null for zero
    void* buf0;        // x^(0) on entry (transposed); ping-pong with buf1
    void* buf1;
    void* bT;          // B transposed (kt x xld, padding zero)
    int64_t xld;       // leading dimension of the transposed iterate (multiple of 64)
    const void* diag;
    int64_t n;
    int32_t k;
    int32_t nwg;       // workgroups sharing this system (1 = owned by one WG)
    int32_t max_iter;
    int32_t test;      // TEST_ABS or TEST_REL
    double tol;        // TEST_ABS threshold
    double rel;        // TEST_REL factor
    int32_t norm;      // 0 inf, 1 l2
    int32_t it0, it1;  // lockstep schedule: the system's work items [it0, it1)
    // Column split (lockstep schedule, one system per launch): the columns
    // are cut into csplit chunks of cw columns (a multiple of the workgroup's
    // block span); item it0 + r * csplit + c covers chunk c of row range r and
    // writes its partial sums to part + c * kt * xld (transposed); the last
    // chunk of a row range to finish adds them in chunk order.  csplit = 1:
    // no split.
    int32_t csplit;
    int32_t first_free;  // 1: x^(0) := B / a_ii (the first sweep from zero, no pass over A)
    int64_t cw;
    void* part;
};

// Per-system control state (device), zeroed before the launch.
struct alignas(64) BState {
    uint32_t counter;        // barrier arrivals (split systems)
    uint32_t status;         // STOP_* (STOP_RUNNING = cap reached / not started)
    int32_t iterations;      // sweeps executed
    uint32_t error;          // 1: a barrier wait timed out
    uint64_t dmax[3];        // per-sweep max |dx| (double bits), slot = sweep % 3
    uint64_t xmax[3];        // per-sweep max |x_new|
    uint64_t final_delta;    // double bits
    int64_t bad_diag;        // validation: min over bad diagonals of 2*row + (non-finite ? 1 : 0)
    int64_t bad_rhs;         // validation: first row with a non-finite B or X0 entry
    int32_t done;            // lockstep schedule: 0 running, r + 1 stopped after sweep r
                             // (its X is copied out in round r + 1), -1 invalid input;
                             // the host sets 1 for max_iter = 0 (X0 copied out in round 1)
    // dataflow schedule
    uint32_t fin;            // items of the current work finished
    int32_t work;            // current work: 2 r = sweep r, 2 r + 1 = copy x^(r) out to X
};

constexpr int kMaxGroups = 8;  // work-item groups of the lockstep schedule (XCDs)

// Grid-wide control words of the lockstep schedule (device), zeroed before
// the launch except `active`.
struct alignas(64) BCtl {
    uint32_t bar;     // grid barrier arrivals (all rounds)
    uint32_t active;  // systems with sweeps to run (set by the host)
    uint32_t abort;   // 1: a barrier wait timed out
    uint32_t pad;
    // systems that swept in round r, in swept[r % 3]: read by every
    // workgroup after the round's barrier (the loop ends when it is zero);
    // workgroup 0 clears swept[(r + 1) % 3] during round r, when every
    // workgroup has read it
    uint32_t swept[3];
    uint32_t pad2;
    // work-item tickets of each group, by round parity: round r draws from
    // qhead[r & 1]; workgroup 0 clears the other parity during round r
    uint32_t qhead[2][kMaxGroups];
    // dataflow schedule: queue positions [0, ftail) are reserved for
    // publication (ftail starts at the item count), [0, fhead) are claimed
    uint32_t ftail;
    uint32_t fhead;
};

struct BatchArgs {
    const BSys* sys;
    BState* st;
    const BJob* jobs;
    const int32_t* job_off;   // [grid + 1]: jobs of workgroup g are [job_off[g], job_off[g+1])
    double* parts;            // [2][count][max_nwg] L2 partial sums
    const int32_t* queue;     // systems run whole by whichever workgroup is free
    uint32_t* queue_head;     // next queue entry (zero at launch)
    int32_t queue_len;
    int32_t max_nwg;
    int32_t count;
    int64_t spin_limit;       // wall-clock ticks (100 MHz) before a barrier wait gives up
    // lockstep schedule (k_rounds): one grid barrier per sweep, rows dealt
    // out as work items
    const BJob* items;        // rows [r0, r1) of system sys; `rank` unused
    double* item_parts;       // [2][nitems] L2 partial sums of the sweep, by round parity
    BCtl* ctl;
    const int32_t* group_off; // [ngroups + 1]: items of group q are [group_off[q], group_off[q+1])
    uint32_t* rcnt;           // [nitems]: chunks of a row range done this round (split systems,
                              // at the range's first item), zero between rounds
    int32_t ngroups;          // 0 (no items) .. kMaxGroups
    int32_t nitems;
    int32_t active0;          // systems with max_iter > 0
    int32_t max_rounds;       // largest max_iter among them: the last round is max_rounds + 1
    // dataflow schedule (k_flow): queue position q holds work item q for
    // q < nitems (every system's first work), else ring[q - nitems] =
    // (gen << 32) | (item + 1) once published
    uint64_t* ring;
    uint32_t ring_cap;        // entries of ring
    uint32_t gen;             // this launch's tag (never 0)
};

hipError_t launch_batched_setup(int32_t a_dtype, int32_t kt, const BSys* sys, BState* st,
                                int32_t count, int64_t max_n, hipStream_t s);
hipError_t launch_batched(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                          hipStream_t s);
// The lockstep schedule: every workgroup sweeps work items of any system, all
// systems advance one sweep per round, one grid barrier per round.
// split: the kernel compiled with the column split of a single system.
hipError_t launch_rounds(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                         hipStream_t s, bool split = false);
int rounds_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus, bool split = false);
// The dataflow schedule: no rounds; a system's next sweep (or its copy-out)
// is queued as soon as the last item of its current one has finished.
hipError_t launch_flow(int32_t a_dtype, int32_t kt, int variant, const BatchArgs& a, int grid,
                       hipStream_t s);
int flow_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus);
int batched_max_grid(int32_t a_dtype, int32_t kt, int variant, int num_cus);

// ---------------------------------------------------------------------------
// Batched FP64 residual pass (resid.hip): for many systems at once,
// x_new = x + d, r = B - A x_new, ||r||_2 and the outer stop test of the
// refinement loop, with the contraction on v_mfma_f64_16x16x4f64 tiles.

// Per-system outcome, written by the last workgroup of the system.
struct alignas(32) RState {
    uint32_t stop;       // STOP_RUNNING, STOP_CONVERGED or STOP_DIVERGED
    uint32_t ticket;     // workgroups of this system done
    uint64_t rel_bits;   // ||r||_2 / ||b||_2 (||r||_2 when b = 0), double bits
    uint64_t rmax_bits;  // max |r_ic|, double bits
    uint64_t pad;
};

// One system of a batched residual pass (device pointers).  x, d, x_new,
// r64 and rlo are n x ldx row-major (ldx = padded right-hand-side count).
struct RSys {
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    const double* x;
    const float* d;      // correction added to x first, or null
    double* xnew;        // x + d
    double* r64;         // residual, FP64
    float* rlo;          // residual rounded to FP32 (right-hand side of the inner solve)
    double* xT;          // workspace: (x + d) transposed, kt rows of xld doubles
    int64_t ldx;
    int64_t xld;         // multiple of 8, >= n (zero padded)
    int64_t n;
    int32_t k;
    int32_t job0;        // first job (workgroup) of this system
    int32_t njobs;
    int32_t aligned;     // rows of A are 16-byte aligned
    double bnorm;        // ||B||_2 over the k columns
    double rel;          // stop when ||r||_2 < rel * ||b||_2 (or r == 0)
};

struct RArgs {
    const RSys* sys;
    RState* st;
    const int32_t* job_sys;  // system of each job
    double* parts;           // per-job sum of r^2
};

// Copy `bytes` (a multiple of 16, 16-byte aligned ends) with a kernel.
hipError_t launch_copy16(const void* src, void* dst, size_t bytes, hipStream_t s);

int resid_tiles(int32_t kt, int64_t n, int num_cus);
hipError_t launch_resid_prep(int32_t kt, const RSys* sys, RState* st, int32_t count,
                             int64_t max_xld, hipStream_t s);
hipError_t launch_resid(int32_t kt, int32_t tiles, const RArgs& a, int32_t jobs, hipStream_t s);
int batched_tiles_per_pass(int32_t a_dtype, int32_t kt, int variant, bool lockstep_whole);
int batched_unroll(int32_t a_dtype);
int batched_block_cols(int32_t a_dtype);

// Default launch configuration for a sweep of this shape.
LaunchCfg default_cfg(int32_t a_dtype, int64_t n, int32_t k, int num_cus);
LaunchCfg residual_cfg(int64_t n, int32_t k, int num_cus);
size_t sweep_lds_bytes(int32_t a_dtype, int32_t k, const LaunchCfg& cfg);

}  // namespace jac
