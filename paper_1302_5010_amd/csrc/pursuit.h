// Argument blocks of the per-signal pursuit kernels (pursuit.hip).
#pragma once

#include "bmpl_internal.h"

namespace bmpl {

struct PrepArgs {
    Workspace w;
    const float* B; int64_t ldb;   // caller's signals
    float* Bw;                     // [p][kpad] padded float32 copy
    const double* lambda_dev;      // per-signal lambda or null
    double lambda_abs;
    int lam_rel_mode;              // lambda set later from the first correlation pass
};

struct StatusArgs {
    Workspace w;
    const int* act_in; const int* n_in_dev; int n_in;
    int* act_out; int* n_out_dev;
    int initial;        // first call: keep every finite signal
    int max_outer;
    double kkt_tol;
    int warm_check;     // pass right after a warm-started master solve
    double eps_early;   // Eq. (13) tolerance, 0 = off
    double r_inf_rel;   // Eq. (10) correlation radius relative to ||A^T b_i||_inf, 0 = off
    double r2_rel;      // Eq. (10) residual radius relative to ||b_i||, 0 = off
    int rho;            // atoms per outer iteration in the Eq. (13) normalisation
    // slot-block reserve: the doubles the kept signals may request from the arena during the next
    // reserve_iters outer iterations (rho_pass slots each at most), written to arena->reserve
    int reserve_iters; int rho_pass; int slack; int kcap;
    int* clear_cert;    // the selection's certification list count, set to 0 at the end (or null)
    int* grow_list; int* n_grow;   // kept signals whose block must grow for this pass's selection
    unsigned long long* grow_off;  // their new blocks' offsets from arena->grow_base (one fetch-and-add)
    int kmin;                      // smallest capacity handed out (as GrowArgs::kmin)
};

struct WarmArgs {
    Workspace w;
    const int* act; const int* n_act_dev;
    const int32_t* warm; int warm_k;
    int max_active;
};

// Internal status bit (never returned): the solve kernel could not run this signal's master problem
// and the next stop test ends it.
constexpr int ST_HALT = 1 << 20;

// Atoms per block append of the inverse factor, and the LDS layout of the solve kernel's vectors: by
// slot (K of them: x, c, g as float64, atoms as int, theta and exclusion bytes) and by support position
// (P = min(K, n) of them, since |S| <= n: w, z, x_new and the cached z as float64, support order as int).
constexpr int SOLVE_JB = 8;
__host__ __device__ inline size_t vec_area_bytes(int K, int P) { return ((size_t)K * 30 + (size_t)P * 36 + 15) / 16 * 16; }
__host__ __device__ inline size_t block_scratch_bytes(int K) { return (size_t)K * SOLVE_JB * 8; }
constexpr size_t GRAM_STAGE_BYTES = 64 * 16 * 8;   // direct Gram rows' atom staging (only without the table)

struct SolveArgs {
    Workspace w;
    const float* At; int64_t lda;
    const float* Bw;
    const double* Q; int64_t ldq;   // Gram table A^T A (float64) or null
    const int* act; const int* n_act_dev;
    int max_steps_per_slot;         // active-set step cap: max_steps_per_slot * capacity + 256
    int rinv_lds;                   // inverse factor in LDS (capacity kl positions)
    int kl;
    int vec_lds;                    // per-slot vectors in LDS
    int kv;                         // their stride by slot: a bound on |I| during the launch
    int kp;                         // by support position: >= min(kv, n) (and >= the candidates of an
                                    // exploratory pass, whose scratch lists live there)
    int zs_lds;                     // block-append scratch in LDS after the vectors (else single appends)
    int smpl_keep;                  // > 0: subspace exploratory matching keeps this many of the new atoms
    uint64_t* phase;                // [PHASE_SLOTS]: wall-clock ticks of phases 0-5 summed over workgroups,
                                    // counts of factor appends, drops and solves, then ticks of the
                                    // active-set steps (drops, minimiser, gradients, violator list,
                                    // ratio test) and of the residual; or null
};


constexpr int PHASE_SLOTS = 15;     // solve-kernel phase ticks and counters (SolveArgs::phase)

struct GrowArgs {
    Workspace w;
    const int* list; const int* n_list;   // the signals to grow (written by the stop test)
    const unsigned long long* off;        // their blocks' offsets from arena->grow_base
    int slack, kcap;                // grow_capacity's parameters; kcap = max_active
    int kmin;                       // smallest capacity handed out (a block sized for the whole solve)
};

struct PackArgs {
    Workspace w;
    float* x_val; int32_t* x_idx; int32_t* supp_len; int32_t* iters;
    double* kkt; double* lambda; double* objective; int32_t* status;
    int ld_x;
    int stage;          // the support's atoms and values are staged in dynamic LDS (12 bytes per position)
    int stage_max;      // positions that fit that staging
};

__global__ void prep_kernel(PrepArgs a);
__global__ void status_compact_kernel(StatusArgs a);
__global__ void warm_select_kernel(WarmArgs a);
__global__ void solve_kernel(SolveArgs a);         // single appends only (zs_lds ignored)
__global__ void solve_fold_kernel(SolveArgs a);    // solve_kernel with one-pass appends and solves on
                                                   // factors in global memory (launches with rinv_lds = 0)
__global__ void solve_block_kernel(SolveArgs a);   // block appends when zs_lds
__global__ void pack_kernel(PackArgs a);
__global__ void grow_kernel(GrowArgs a);

}  // namespace bmpl
