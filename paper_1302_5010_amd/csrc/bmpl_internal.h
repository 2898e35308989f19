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

// Device arena of the per-signal slot blocks: a list of chunks viewed as one range of doubles.  Blocks
// are handed out by bumping `top` (a block never straddles two chunks); a signal whose active set
// outgrows its block takes a larger one and copies its state over.  The arena is reset for every solve.
constexpr int ARENA_CHUNKS = 32;
struct Arena {
    int n_act[2];                 // running-signal counts of the two running lists (read back with the rest)
    unsigned long long top;       // doubles handed out in this solve (offset in the chunk list)
    unsigned long long starved;   // block requests that found no room (the host adds a chunk)
    unsigned long long reserve;   // doubles the running signals may request during the next iterations
    unsigned long long grow_base; // offset of the blocks the last stop test placed for the grow list
    int nchunks;
    int pad_;
    double* base[ARENA_CHUNKS];
    unsigned long long start[ARENA_CHUNKS];   // offset of each chunk in the list (start[c+1] = start[c] + size[c])
    unsigned long long size[ARENA_CHUNKS];    // doubles
};

// N chunks of four consecutive correlations of a row per thread (thread t: g[base0 + 1024 q + 4 t ..
// + 3], q < N) with their bits of the I bitmap (bit set: in I; `absent` for lanes past the vector part
// of the row, m4, whose values read as zeros).  When every lane's chunks lie inside the row (a test that
// is the same for the whole workgroup) the loads are unconditional, so all of a thread's loads are in
// flight at once: a guarded load compiles to a branch that waits for its data at the branch's end.
template <int N>
__device__ __forceinline__ void row_chunks(const float* g, const uint32_t* ex, int base0, int m4, uint32_t absent,
                                           float4 (&f)[N], uint32_t (&w)[N])
{
    const int t4 = 4 * (int)threadIdx.x;
    if (base0 + 1024 * N <= m4) {
#pragma unroll
        for (int q = 0; q < N; ++q) f[q] = *reinterpret_cast<const float4*>(g + base0 + 1024 * q + t4);
        if (ex) {
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const int j0 = base0 + 1024 * q + t4;
                w[q] = ex[j0 >> 5] >> (j0 & 31);
            }
        } else {
#pragma unroll
            for (int q = 0; q < N; ++q) w[q] = 0u;
        }
        return;
    }
    // the row's tail: clamped indices, so the loads are still issued together (a guarded load compiles to
    // a branch whose end waits for it); lanes past the vector part read as zeros
    if (m4 == 0 || base0 >= m4) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            f[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            w[q] = absent;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int j0 = base0 + 1024 * q + t4;
        const int jl = j0 < m4 ? j0 : m4 - 4;
        f[q] = *reinterpret_cast<const float4*>(g + jl);
        w[q] = ex ? (ex[jl >> 5] >> (jl & 31)) : 0u;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const bool in = base0 + 1024 * q + t4 < m4;
        f[q] = in ? f[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        w[q] = in ? w[q] : absent;
    }
}

// One signal's slot block for capacity K (slots of I) and signal length n:
//   G [K][K] float64 (Gram of I, row-major by slot) | Rinv [tri(min(K, n))] float64 (inverse Cholesky
//   factor of G_SS, packed by support position; |S| <= n) | x [K] | c [K] | vs [8K] float64 scratch |
//   atom [K] int | sord [K] int | theta [K] int8 | excl [K] uint8, padded to 256 bytes.
__host__ __device__ inline int64_t block_doubles(int K, int n)
{
    const int64_t F = K < n ? K : n;
    const int64_t d = (int64_t)K * K + tri(F) + 10 * (int64_t)K + (10 * (int64_t)K + 7) / 8;
    return (d + 31) / 32 * 32;
}

struct SlotBlock {
    double* G; double* Rinv; double* x; double* c; double* vs;
    int* atom; int* sord; signed char* theta; unsigned char* excl;
};

__host__ __device__ inline SlotBlock slot_block(double* base, int K, int n)
{
    SlotBlock b;
    const int64_t F = K < n ? K : n;
    b.G = base;
    b.Rinv = b.G + (int64_t)K * K;
    b.x = b.Rinv + tri(F);
    b.c = b.x + K;
    b.vs = b.c + K;
    b.atom = reinterpret_cast<int*>(b.vs + 8 * (int64_t)K);
    b.sord = b.atom + K;
    b.theta = reinterpret_cast<signed char*>(b.sord + K);
    b.excl = reinterpret_cast<unsigned char*>(b.theta + K);
    return b;
}

// Capacity a block grows to when it must hold `need` slots: at least twice the current capacity and
// `need + slack`, a multiple of 32 (64 at least), at most kcap (>= need).
__host__ __device__ inline int grow_capacity(int K, int need, int slack, int kcap)
{
    int a = need + slack, b = 2 * K;
    int t = a > b ? a : b;
    t = t < 64 ? 64 : t;
    t = (t + 31) / 32 * 32;
    return t < kcap ? (t > need ? t : need) : (kcap > need ? kcap : need);
}

// Per-signal state of the batched pursuit.  Arrays indexed [signal * stride + ...].
// "slot" = position in the active set I (insertion order, never removed);
// "position" = position in the support S (order of entry into S).
struct Workspace {
    int n;          // signal length
    int kpad;       // n rounded up to a multiple of 32 (rows of the residual buffer)
    int m;          // atoms
    int words;      // ceil(m / 32): bitmap words per signal
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
    double* obj_prev;   // [p] objective after the master solve before it (Eq. (13))
    double* rr2;        // [p] ||xi_i||^2 after the last master solve, float64 (Eq. (10))
    float* g0max;       // [p] ||A^T b_i||_inf from the first correlation pass (Eq. (10))
    double* kkt;        // [p] final certificate (relative to lambda_i)
    uint32_t* inI;      // [p][words] membership bitmap of I
    int* jadd;          // [p] violators the next active-set step admits (adapted per signal, 1..32)
    int* glazy;         // [p] 1: G holds only the entries against S members (and the diagonal); a slot's
                        //     column is gathered when it enters S (set once a pass adds many slots)
    int* cap;           // [p] slot capacity of the signal's block (0: none yet)
    double** blk;       // [p] the signal's slot block in the arena (layout: slot_block)
    Arena* arena;       // allocator of the blocks
    // reduced-precision screening (null in float32 mode)
    uint16_t* R16;      // [p_cap + 1][kpad] bfloat16 copy of R (row p_cap all zero)
    double* rnorm;      // [p] ||xi_i||_2
    double* dxnorm;     // [p] ||bf16(xi_i) - xi_i||_2 (the residual's own rounding)
    uint8_t* R8;        // [p_cap + 1][kpad] e4m3 copy of R / rscale8 (FP8 ranking only; row p_cap zero)
    float* rscale8;     // [p_cap + 1] power-of-two scale of each R8 row
};

// Launchers (all asynchronous on `stream`).

// G[a*ldg + j] = a_j^T r_{act[a]} for a < n_active, j < m, float32 MFMA.
// At: atom-major [m + 1][lda] float32 with lda % 4 == 0, zero-padded to kpad, row m all zero.
// Rbuf: [*][ldr] float32, ldr % 4 == 0, columns zero-padded to kpad; row `zero_row` all zero.
// act == nullptr means the identity map.  If n_act_dev != nullptr the active count is
// read on the device and `p_grid` only sizes the grid.
// `variant` selects the tile shape (see corr_shape_name; 8..10 exist for bfloat16 only).
constexpr int CORR_VARIANTS = 15;  // == BMPL_CORR_SHAPES (8..10: bfloat16 only)
const char* corr_shape_name(int variant);
hipError_t launch_corr_gemm_f32(int variant, const float* At, int64_t lda, int m, int kpad,
                                const float* Rbuf, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                int n_lo, int n_hi, hipStream_t stream);   // runs only if n_lo <= count < n_hi

// Q = A^T A in float64 (m x m, leading dimension ldq), from the padded float32 atoms.
hipError_t launch_gram_table(const float* At, int64_t lda, int m, int kpad, double* Q, int64_t ldq,
                             hipStream_t stream);

// The same product with bfloat16 operands (raw 16-bit storage), float32 accumulation.  Variants 8 and
// up read the dictionary from Apk, its copy in the matrix instruction's fragment order
// (launch_pack_bf16, packed_bf16_elems uint16 values); the others from At.
size_t packed_bf16_elems(int m, int kpad);
hipError_t launch_pack_bf16(const uint16_t* A16, int64_t lda, int m, int kpad, uint16_t* Apk, hipStream_t stream);
hipError_t launch_corr_gemm_bf16(int variant, const uint16_t* At, const uint16_t* Apk, int64_t lda, int m, int kpad,
                                 const uint16_t* Rbuf, int64_t ldr, const int* act,
                                 const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                 int n_lo, int n_hi, hipStream_t stream);

// The same product with e4m3 operands (raw bytes), per-atom and per-signal power-of-two scales
// applied in the epilogue: G = (A8 R8^T) * ascale[j] * rscale[signal].  kpad % 128 == 0.
hipError_t launch_corr_gemm_fp8(int variant, const uint8_t* A8, int64_t lda, int m, int kpad,
                                const uint8_t* R8, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                int n_lo, int n_hi, const float* ascale, const float* rscale, hipStream_t stream);

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
    int* clear_count;      // set to 0 by workgroup 0 before anything else (or null)
    // float32 band (0 = off): signals whose stop needs the exact re-score are appended (their rows)
    const double* rr2; double band; int* cert_list; int* n_cert;
};
hipError_t launch_select(const SelectArgs& a, hipStream_t stream);

// Certification of the natural stop under the float32 product (select.hip): for running signals whose
// selection admitted nothing, the atoms whose float32 |g~| lies within eps_i = band sqrt(rr2[sig]) of
// lambda are re-scored exactly (float32 data, float64 sums); exact violators are admitted (sel, nsel),
// otherwise vmax becomes the exact maximum over them.
struct CertifyArgs {
    const float* G; int64_t ldg; int m;     // the float32 product, one row per running signal
    const int* act; const int* n_act_dev; int p_grid;
    const double* lam; const double* rr2;   // lambda_i and ||xi_i||^2
    double band;                            // eps_i = band ||xi_i||
    const uint32_t* excl; int words;        // I bitmaps
    const float* At; int64_t lda; int n;    // float32 atoms
    const float* R; int64_t ldr;            // float32 residuals (row per signal)
    int k; const int* nI; int max_active;
    int* sel; int selcap; int* nsel; float* vmax;
    const int* cert_list; const int* n_cert;   // the rows the selection listed
};
hipError_t launch_certify(const CertifyArgs& a, hipStream_t stream);

// Reduced-precision screening (screen.hip).
struct ScreenArgs {
    const float* G; int64_t ldg; int m;
    const int* act; const int* n_act_dev; int p_grid;
    const double* lam; double lam_rel;       // lam_rel > 0: first pass of the relative rule
    const double* rnorm; const double* dxnorm;   // band eps_i = band_x rnorm[sig] + band_dx dxnorm[sig]
    double band_x, band_dx;
    const uint32_t* excl; int words;
    int k; const int* nI; int max_active;
    int* cand; int candcap; int* ncand;
    int* clear_count;                         // set to 0 by workgroup 0 before anything else (or null)
};
struct RescoreArgs {
    const float* At; int64_t lda; int kpad;  // float32 atoms
    const float* R; int64_t ldr;             // float32 residuals
    const float* G; int64_t ldg;             // screening product (row per running signal)
    const double* rnorm; const double* dxnorm; double band_x, band_dx;   // the band
    const int* act; const int* n_act_dev; int p_grid;
    const int* cand; int candcap; int candcap_lds; const int* ncand;
    double* lam; double lam_rel;
    int k; const int* nI; int max_active;
    int* sel; int selcap; int* nsel; float* vmax; int* status;
    // Two-pass use: a pass with spill_row set leaves the signals whose candidates exceed candcap_lds
    // (but fit candcap) undecided and records spill_row[sig] = its row + 1 (0 for every other running
    // signal); a pass over those signals with row_of = spill_row reads the product row recorded there.
    int* spill_row; const int* row_of;
    int* spill_act; int* n_spill;   // first pass: the left-over signals are appended here (n_spill starts at 0)
};
// e4m3 ranking (screen.hip): exact re-score of the candidates that the e4m3 product ranked highest,
// admission of the exact violators among them, and the list of signals left for a certified pass.
struct Rank8Args {
    const float* At; int64_t lda; int kpad;  // float32 atoms
    const float* R; int64_t ldr;             // float32 residuals
    const int* act; const int* n_act_dev; int p_grid;
    const int* cand; int candcap; const int* ncand;   // top |g~| outside I per signal
    const double* lam;
    int k; const int* nI; int max_active;
    int* sel; int selcap; int* nsel; float* vmax;
    int* cert;                               // [p] 1: no exact violator among the candidates
    int* cert_act; int* n_cert;              // those signals, appended in any order (n_cert starts at 0)
};
hipError_t launch_rank8(const Rank8Args& a, hipStream_t stream);
// A8[j] = e4m3(a_j / ascale[j]), ascale[j] the power of two that brings max |a_j| to at most 448.
hipError_t launch_atoms_fp8(const float* At, int64_t lda, int kpad, uint8_t* A8, float* ascale, int m,
                            hipStream_t stream);
hipError_t launch_to_bf16(const float* src, int64_t lds, uint16_t* dst, int64_t ldd, int rows, int cols,
                          hipStream_t stream);
// norms[3 m]: ||a_j||, ||bf16(a_j)|| and ||bf16(a_j) - a_j||, each rounded up
hipError_t launch_atom_norms(const float* At, int64_t lda, int n, float* norms, int m, hipStream_t stream);
hipError_t launch_screen(const ScreenArgs& a, hipStream_t stream);
hipError_t launch_rescore(const RescoreArgs& a, hipStream_t stream);

// float32 -> OCP e4m3 (bias 7, largest finite 448, no infinities), round to nearest, ties to even,
// saturating at +-448; NaN -> 0x7F.  Normal codes (|x| >= 2^-6) keep 3 mantissa bits, subnormal
// codes are multiples of 2^-9 (code 8 = 2^-6, the smallest normal, so the two ranges meet).
__host__ __device__ inline uint8_t fp8_e4m3(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint8_t sgn = (uint8_t)((u >> 24) & 0x80u);
    const uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return 0x7F;
    if (a >= 0x3c800000u) {                          // |x| >= 2^-6
        const uint32_t b = a + 0x7ffffu + ((a >> 20) & 1u);
        const int e = (int)(b >> 23) - 127;
        const uint32_t q = (b >> 20) & 7u;
        if (e > 8 || (e == 8 && q > 6)) return sgn | 0x7E;
        return sgn | (uint8_t)(((e + 7) << 3) | (int)q);
    }
    const float q = __builtin_rintf(__builtin_bit_cast(float, a) * 512.0f);   // exact scaling by 2^9
    return sgn | (uint8_t)q;
}

// Smallest power of two s with maxabs / s <= 448 (1 for maxabs == 0): x / s is exact and fits e4m3.
__host__ __device__ inline float fp8_pow2_scale(float maxabs)
{
    if (!(maxabs > 0.f) || !(maxabs < 3.0e38f)) return 1.f;
    int e;
    const float f = __builtin_frexpf(maxabs / 448.0f, &e);   // maxabs / 448 = f 2^e, f in [0.5, 1)
    return __builtin_ldexpf(1.0f, f == 0.5f ? e - 1 : e);
}

// Round-to-nearest-even float32 -> bfloat16 (raw bits).
__device__ inline uint16_t bf16_round(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x0040u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The float32 value of bfloat16 bits.
__device__ inline float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace bmpl
