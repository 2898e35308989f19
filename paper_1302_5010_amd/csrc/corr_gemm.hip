// Batched correlation G = A^T Xi on MFMA (float32).
//
// One outer iteration of the batched pursuit needs g_i = A^T xi_i for every
// running signal i: the full matrix-vector product of the worst-case analysis
// (Algorithm 1, step 3), done for all signals at once.  It is a dense
// contraction over the signal length n, so it runs on the matrix cores:
// M = running signals, N = atoms, K = n, both operands K-contiguous (the
// dictionary is stored atom by atom, residuals signal by signal).
//
// Tiling (gfx950, wave64): a workgroup computes a BM (signals) x BN (atoms)
// tile; each wave a WM x WN sub-tile as (WM/32) x (WN/32) blocks of
// v_mfma_f32_32x32x2f32.  K is consumed BK = 32 at a time through two LDS
// buffers (one barrier per stage); the next K-slice is prefetched into
// registers while the current one feeds the matrix cores.  Within each 8-wide
// k block, lane half h supplies k = 8b + 4h + t at step t, so every LDS
// fragment read is one 16-byte ds_read per 4 MFMAs (the summation order over k
// is immaterial to the contraction).
//
// Output: G[a*ldg + j], a = compact index of the running signal, j = atom.  The
// MFMA's row index carries the signal and its lane index the atom, so each
// accumulator register stores 32 consecutive atoms of one signal per
// half-wave (coalesced 128-byte stores).
//
// Several tile shapes are instantiated; the host picks one per launch from the
// number of running signals (autotuned, see bmpl_autotune).
#include "bmpl_internal.h"

namespace bmpl {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Each LDS stage holds 128 bytes of k per row: 32 float32 or 64 bfloat16 values, read back as
// one 16-byte fragment per lane per 8 (float32) or 16 (bfloat16) k values.
constexpr int ROW_BYTES = 128;
constexpr int LDS_ROW = ROW_BYTES + 16;   // bytes per LDS row (16-byte aligned, staggers banks)

template <int BM, int BN, int WM, int WN>
struct Shape {
    static constexpr int WAVES = (BM / WM) * (BN / WN);
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int TI = WM / 32;                 // MFMA blocks per wave, signal direction
    static constexpr int TJ = WN / 32;                 // atom direction
    static constexpr int LR = BM * 8 / THREADS;        // 16-byte loads per thread, residual tile
    static constexpr int LA = BN * 8 / THREADS;        // dictionary tile
    static_assert(LR * THREADS == BM * 8 && LA * THREADS == BN * 8, "tile/thread mismatch");
};

template <class E, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((Shape<BM, BN, WM, WN>::THREADS)) void corr_gemm_kernel(
    const E* __restrict__ At, int64_t lda, int m, int kpad,
    const E* __restrict__ Rbuf, int64_t ldr, const int* __restrict__ act,
    const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G, int64_t ldg, int tiles_n, int zero_row,
    int n_lo, int n_hi)
{
    using S = Shape<BM, BN, WM, WN>;
    constexpr int BK = ROW_BYTES / (int)sizeof(E);   // k per stage
    constexpr int VE = 16 / (int)sizeof(E);          // k per 16-byte chunk
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
    if (n_act < n_lo || n_act >= n_hi) return;   // another tile shape serves this running count
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so give each XCD a
    // contiguous run of tiles (atom tiles outer, signal tiles inner) to share A rows in its L2.
    const int nwg = gridDim.x;
    const int wid = blockIdx.x;
    int tile;
    {
        const int per = nwg / 8, rem = nwg % 8, xcd = wid % 8, loc = wid / 8;
        tile = (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
    }
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tm = tile % tiles_m;          // signal tile
    const int tn = tile / tiles_m;          // atom tile
    if (tn >= tiles_n) return;
    const int sig0 = tm * BM;
    const int atom0 = tn * BN;
    if (sig0 >= n_act) return;

    __shared__ __attribute__((aligned(16))) char sR[2][BM * LDS_ROW];
    __shared__ __attribute__((aligned(16))) char sA[2][BN * LDS_ROW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // Global -> register staging (element offsets from the kernel-argument base pointers, so the
    // loads stay global and the staging registers are never spilled).  Rows past the end point at
    // an all-zero row (row `zero_row` of the residuals, row m of the dictionary), so every load is
    // unconditional and is consumed only by the LDS store at the end of the stage.
    const int c4 = tid & 7;                   // which float4 of the 32-wide k slice
    const int r0 = tid >> 3;                  // first row; rows r0 + (THREADS/8) q
    constexpr int RSTEP = S::THREADS / 8;
    int64_t oR[S::LR], oA[S::LA];
    bool vR[S::LR], vA[S::LA];   // row in range (only used to pick the zero row)
#pragma unroll
    for (int q = 0; q < S::LR; ++q) {
        const int a = sig0 + r0 + RSTEP * q;
        vR[q] = a < n_act;
        const int s = vR[q] ? (act ? act[a] : a) : zero_row;
        oR[q] = (int64_t)s * ldr + VE * c4;
    }
#pragma unroll
    for (int q = 0; q < S::LA; ++q) {
        const int j = atom0 + r0 + RSTEP * q;
        vA[q] = j < m;
        oA[q] = (int64_t)(vA[q] ? j : m) * lda + VE * c4;
    }
    float4 gR[S::LR], gA[S::LA];
#define CORR_LOAD_SLICE(k0)                                                                                 \
    do {                                                                                                    \
        _Pragma("unroll") for (int q = 0; q < S::LR; ++q)                                                  \
            gR[q] = *reinterpret_cast<const float4*>(Rbuf + oR[q] + (k0));                                  \
        _Pragma("unroll") for (int q = 0; q < S::LA; ++q)                                                  \
            gA[q] = *reinterpret_cast<const float4*>(At + oA[q] + (k0));                                    \
    } while (0)
#define CORR_STORE_SLICE(buf)                                                                               \
    do {                                                                                                    \
        _Pragma("unroll") for (int q = 0; q < S::LR; ++q)                                                  \
            *reinterpret_cast<float4*>(&sR[buf][(r0 + RSTEP * q) * LDS_ROW + 16 * c4]) = gR[q];            \
        _Pragma("unroll") for (int q = 0; q < S::LA; ++q)                                                  \
            *reinterpret_cast<float4*>(&sA[buf][(r0 + RSTEP * q) * LDS_ROW + 16 * c4]) = gA[q];            \
    } while (0)

    floatx16 acc[S::TI][S::TJ];
#pragma unroll
    for (int i = 0; i < S::TI; ++i)
#pragma unroll
        for (int j = 0; j < S::TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    constexpr int WAVES_M = BM / WM;
    const int ws = (wave % WAVES_M) * WM;   // wave's signal offset in the tile
    const int wa = (wave / WAVES_M) * WN;   // wave's atom offset in the tile
    const int l32 = lane & 31;
    const int h = lane >> 5;

    CORR_LOAD_SLICE(0);
    CORR_STORE_SLICE(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kpad; k0 += BK) {
        // prefetch the next slice (the last iteration re-reads the final slice; its copy is never used)
        const int kn = k0 + BK < kpad ? k0 + BK : k0;
        CORR_LOAD_SLICE(kn);
        asm volatile("" ::: "memory");       // issue the prefetch before the matrix work
        const char* cR = sR[cur];
        const char* cA = sA[cur];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {       // 4 x 16-byte chunks per lane half per stage
            float4 fr[S::TI], fa[S::TJ];
#pragma unroll
            for (int i = 0; i < S::TI; ++i)
                fr[i] = *reinterpret_cast<const float4*>(&cR[(ws + 32 * i + l32) * LDS_ROW + kb * 32 + 16 * h]);
#pragma unroll
            for (int j = 0; j < S::TJ; ++j)
                fa[j] = *reinterpret_cast<const float4*>(&cA[(wa + 32 * j + l32) * LDS_ROW + kb * 32 + 16 * h]);
            if constexpr (sizeof(E) == 2) {
                // bfloat16: one v_mfma_f32_32x32x16_bf16 per block; lane half h supplies 8 consecutive k
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fr[i]), __builtin_bit_cast(bf16x8, fa[j]), acc[i][j], 0, 0, 0);
            } else {
                // float32: four v_mfma_f32_32x32x2f32 per block, k step outermost so consecutive MFMAs
                // write different accumulators
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].x, fa[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].y, fa[j].y, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].z, fa[j].z, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].w, fa[j].w, acc[i][j], 0, 0, 0);
            }
        }
        asm volatile("" ::: "memory");       // and consume it only after
        CORR_STORE_SLICE(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

#undef CORR_LOAD_SLICE
#undef CORR_STORE_SLICE

    // D[row][col] of a 32x32 block (both instructions): lane l, register r -> row 8(r/4) + 4(l/32) + r%4,
    // col l%32.
#pragma unroll
    for (int i = 0; i < S::TI; ++i)
#pragma unroll
        for (int j = 0; j < S::TJ; ++j) {
            const int atom = atom0 + wa + 32 * j + l32;
            if (atom >= m) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = sig0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (a < n_act) G[(int64_t)a * ldg + atom] = acc[i][j][r];
            }
        }
}

template <class E, int BM, int BN, int WM, int WN>
hipError_t launch_shape(const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr,
                        const int* act, const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                        int n_lo, int n_hi, hipStream_t stream)
{
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((corr_gemm_kernel<E, BM, BN, WM, WN>), dim3((unsigned)nwg),
                       dim3(Shape<BM, BN, WM, WN>::THREADS), 0, stream, At, lda, m, kpad, Rbuf, ldr, act,
                       n_act_dev, p_grid, G, ldg, tiles_n, zero_row, n_lo, n_hi);
    return hipGetLastError();
}

template <class E>
hipError_t launch_variant(int variant, const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr,
                          const int* act, const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                          int n_lo, int n_hi, hipStream_t stream)
{
    if (p_grid <= 0 || m <= 0) return hipSuccess;
    if (kpad % (ROW_BYTES / (int)sizeof(E))) return hipErrorInvalidValue;
    switch (variant) {
    case 0: return launch_shape<E, 128, 128, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    case 1: return launch_shape<E, 128, 256, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    case 2: return launch_shape<E, 256, 128, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    case 3: return launch_shape<E, 64, 128, 32, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    case 4: return launch_shape<E, 32, 64, 32, 32>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    case 5: return launch_shape<E, 64, 64, 32, 32>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

const char* corr_shape_name(int v)
{
    switch (v) {
    case 0: return "128x128 (4 waves of 64x64)";
    case 1: return "128x256 (8 waves of 64x64)";
    case 2: return "256x128 (8 waves of 64x64)";
    case 3: return "64x128 (4 waves of 32x64)";
    case 4: return "32x64 (2 waves of 32x32)";
    case 5: return "64x64 (4 waves of 32x32)";
    default: return "?";
    }
}

hipError_t launch_corr_gemm_f32(int variant, const float* At, int64_t lda, int m, int kpad,
                                const float* Rbuf, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                int n_lo, int n_hi, hipStream_t stream)
{
    return launch_variant<float>(variant, At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row,
                                 n_lo, n_hi, stream);
}

hipError_t launch_corr_gemm_bf16(int variant, const uint16_t* At, int64_t lda, int m, int kpad,
                                 const uint16_t* Rbuf, int64_t ldr, const int* act,
                                 const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                 int n_lo, int n_hi, hipStream_t stream)
{
    return launch_variant<__bf16>(variant, reinterpret_cast<const __bf16*>(At), lda, m, kpad,
                                  reinterpret_cast<const __bf16*>(Rbuf), ldr, act, n_act_dev, p_grid, G, ldg,
                                  zero_row, n_lo, n_hi, stream);
}

}  // namespace bmpl
