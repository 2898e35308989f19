// Internal declarations shared by the HIP translation units of libbmpl.
// Not part of the public ABI (include/bmpl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpl {

// Packed lower-triangular row-major storage: row i starts at tri(i) and holds
// columns 0..i.  A matrix of order s occupies the prefix tri(s).
__host__ __device__ inline int64_t tri(int64_t i) { return i * (i + 1) / 2; }

// Symmetric lookup in a packed lower triangle.
__device__ inline double sym_at(const double* P, int u, int v)
{
    return u >= v ? P[tri(u) + v] : P[tri(v) + u];
}

// Per-signal state of the batched pursuit.  Arrays indexed [signal * stride + ...].
// "slot" = position in the active set I (insertion order, never removed);
// "position" = position in the support S (order of entry into S).
struct Workspace {
    int n;          // signal length
    int kpad;       // n rounded up to a multiple of 32 (rows of the residual buffer)
    int m;          // atoms
    int words;      // ceil(m / 32): bitmap words per signal
    int K;          // slot capacity per signal
    int p;          // signals in the current solve

    float* R;           // [p_cap + 1][kpad] float32 residuals xi_i (zero rows past n; row p_cap all zero)
    double* bnorm2;     // [p] ||b_i||^2
    double* lam;        // [p] lambda_i
    int* status;        // [p] BMPL_SIG_* bits
    int* iters;         // [p] outer iterations that added atoms
    int* nI;            // [p] |I|
    int* nS;            // [p] |S|
    int* nsel;          // [p] atoms selected in this iteration
    int* sel;           // [p][selcap] atoms selected in this iteration
    int selcap;         // capacity of sel per signal
    float* vmax;        // [p] max |g_j| outside I in the last correlation pass
    double* kkt_on;     // [p] restricted optimality residual on I (absolute)
    double* obj;        // [p] objective after the last master solve
    double* kkt;        // [p] final certificate (relative to lambda_i)
    uint32_t* inI;      // [p][words] membership bitmap of I
    int* slot_atom;     // [p][K]
    double* x;          // [p][K] coefficient per slot
    double* c;          // [p][K] a_u^T b per slot
    signed char* theta; // [p][K] sign per slot (0 = not in S)
    unsigned char* excl;// [p][K] slot excluded from S (linearly dependent)
    int* sord;          // [p][K] slot of each support position
    double* G;          // [p][K*K] Gram of I, row-major by slot
    double* Rinv;       // [p][tri(K)] inverse Cholesky factor of G_SS, packed by position
    double* vscratch;   // [p][8K] vectors when they do not fit LDS
    // reduced-precision screening (null in float32 mode)
    uint16_t* R16;      // [p_cap + 1][kpad] bfloat16 copy of R (row p_cap all zero)
    double* rnorm;      // [p] ||xi_i||_2
};

// Launchers (all asynchronous on `stream`).

// G[a*ldg + j] = a_j^T r_{act[a]} for a < n_active, j < m, float32 MFMA.
// At: atom-major [m + 1][lda] float32 with lda % 4 == 0, zero-padded to kpad, row m all zero.
// Rbuf: [*][ldr] float32, ldr % 4 == 0, columns zero-padded to kpad; row `zero_row` all zero.
// act == nullptr means the identity map.  If n_act_dev != nullptr the active count is
// read on the device and `p_grid` only sizes the grid.
// `variant` selects the tile shape (0..5, see corr_shape_name).
constexpr int CORR_VARIANTS = 6;
const char* corr_shape_name(int variant);
hipError_t launch_corr_gemm_f32(int variant, const float* At, int64_t lda, int m, int kpad,
                                const float* Rbuf, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                int n_lo, int n_hi, hipStream_t stream);   // runs only if n_lo <= count < n_hi

// Q = A^T A in float64 (m x m, leading dimension ldq), from the padded float32 atoms.
hipError_t launch_gram_table(const float* At, int64_t lda, int m, int kpad, double* Q, int64_t ldq,
                             hipStream_t stream);

// The same product with bfloat16 operands (raw 16-bit storage), float32 accumulation.
hipError_t launch_corr_gemm_bf16(int variant, const uint16_t* At, int64_t lda, int m, int kpad,
                                 const uint16_t* Rbuf, int64_t ldr, const int* act,
                                 const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                 int n_lo, int n_hi, hipStream_t stream);

// Top-k selection per row (worst-case analysis).  See bmpl_select in bmpl.h; here
// `lam_rel` > 0 computes lambda[sig] = lam_rel * max_j |G| first (first pass).
struct SelectArgs {
    const float* G; int64_t ldg; int m;
    const int* act; const int* n_act_dev; int p_grid;
    double* lam; double lam_rel;
    const uint32_t* excl; int words;
    int k;                 // atoms per row requested
    int* sel; int selcap; int* nsel; float* vmax;
    // pursuit bookkeeping (may be null in the diagnostic entry point)
    const int* nI; int max_active;
};
hipError_t launch_select(const SelectArgs& a, hipStream_t stream);

// Reduced-precision screening (screen.hip).
struct ScreenArgs {
    const float* G; int64_t ldg; int m;
    const int* act; const int* n_act_dev; int p_grid;
    const double* lam; double lam_rel;       // lam_rel > 0: first pass of the relative rule
    const double* rnorm; double gamma_amax;  // band eps_i = gamma_amax * rnorm[sig]
    const uint32_t* excl; int words;
    int k; const int* nI; int max_active;
    int* cand; int candcap; int* ncand;
};
struct RescoreArgs {
    const float* At; int64_t lda; int kpad;  // float32 atoms
    const float* R; int64_t ldr;             // float32 residuals
    const float* G; int64_t ldg;             // screening product (row per running signal)
    const double* rnorm; double gamma_amax;  // the band
    const int* act; const int* n_act_dev; int p_grid;
    const int* cand; int candcap; int candcap_lds; const int* ncand;
    double* lam; double lam_rel;
    int k; const int* nI; int max_active;
    int* sel; int selcap; int* nsel; float* vmax; int* status;
};
hipError_t launch_to_bf16(const float* src, int64_t lds, uint16_t* dst, int64_t ldd, int rows, int cols,
                          hipStream_t stream);
hipError_t launch_atom_norms(const float* At, int64_t lda, int n, float* norms, int m, hipStream_t stream);
hipError_t launch_screen(const ScreenArgs& a, hipStream_t stream);
hipError_t launch_rescore(const RescoreArgs& a, hipStream_t stream);

// Round-to-nearest-even float32 -> bfloat16 (raw bits).
__device__ inline uint16_t bf16_round(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x0040u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace bmpl
