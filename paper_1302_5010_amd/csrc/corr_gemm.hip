// Batched correlation G = A^T Xi on MFMA (float32).
//
// One outer iteration of the batched pursuit needs g_i = A^T xi_i for every
// running signal i: the full matrix-vector product of the worst-case analysis
// (Algorithm 1, step 3), done for all signals at once.  It is a dense
// contraction over the signal length n, so it runs on the matrix cores:
// M = running signals, N = atoms, K = n, both operands K-contiguous (the
// dictionary is stored atom by atom, residuals signal by signal).
//
// The K loop is the shared double-buffered MFMA tile loop of gemm_tile.h.
//
// Output: G[a*ldg + j], a = compact index of the running signal, j = atom.  The
// MFMA's row index carries the signal and its lane index the atom, so each
// accumulator register stores 32 consecutive atoms of one signal per
// half-wave (coalesced 128-byte stores).
//
// Several tile shapes are instantiated; the host picks one per launch from the
// number of running signals (autotuned, see bmpl_autotune).  The large-wave shapes
// (128 x 128 and 64 x 128 per wave) issue more matrix instructions per LDS fragment
// read, which the short bfloat16 and e4m3 instructions need.
#include <algorithm>

#include "bmpl_internal.h"
#include "gemm_tile.h"

namespace bmpl {
namespace {

// Store a finished tile: D[row][col] of a 32x32 block (both instructions): lane l, register r -> row
// 8(r/4) + 4(l/32) + r%4, col l%32.  e4m3 operands carry power-of-two scales: one per atom, one per signal.
template <class E, int TI, int TJ>
__device__ __forceinline__ void store_tile(const floatx16 (&acc)[TI][TJ], int sig0, int ws, int atom0, int wa, int l32,
                                           int h, int m, int n_act, const int* __restrict__ act, float* __restrict__ G,
                                           int64_t ldg, const float* __restrict__ ascale, const float* __restrict__ rscale)
{
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int atom = atom0 + wa + 32 * j + l32;
            if (atom >= m) continue;
            const float sa = sizeof(E) == 1 ? ascale[atom] : 1.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = sig0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (a < n_act) {
                    if constexpr (sizeof(E) == 1)
                        G[(int64_t)a * ldg + atom] = acc[i][j][r] * sa * rscale[act ? act[a] : a];
                    else
                        G[(int64_t)a * ldg + atom] = acc[i][j][r];
                }
            }
        }
}

template <class E, int BM, int BN, int WM, int WN, int DEPTH>
__global__ __launch_bounds__((TileShape<BM, BN, WM, WN>::THREADS)) void corr_gemm_kernel(
    const E* __restrict__ At, int64_t lda, int m, int kpad,
    const E* __restrict__ Rbuf, int64_t ldr, const int* __restrict__ act,
    const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G, int64_t ldg, int tiles_n, int zero_row,
    int n_lo, int n_hi, const float* __restrict__ ascale, const float* __restrict__ rscale)
{
    using S = TileShape<BM, BN, WM, WN>;
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
    if (n_act < n_lo || n_act >= n_hi) return;   // another tile shape serves this running count
    // Only the signal tiles that hold running signals are numbered (the grid is sized for p_grid, the
    // count at capture time), so the working tiles are dealt evenly to the XCDs at every running count.
    const int tiles_m = ((n_act < p_grid ? n_act : p_grid) + BM - 1) / BM;
    const int nwg = tiles_m * tiles_n;
    if ((int)blockIdx.x >= nwg) return;
    const int tile = xcd_tile_index(blockIdx.x, nwg);
    int tm, tn;                             // signal tile, atom tile (grouped order, see grouped_tile)
    grouped_tile<8>(tile, tiles_m, tiles_n, tm, tn);
    if (tn >= tiles_n) return;
    const int sig0 = tm * BM;
    const int atom0 = tn * BN;
    if (sig0 >= n_act) return;

    __shared__ __attribute__((aligned(16))) TileLds<BM, BN> lds;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int VE = 16 / (int)sizeof(E);          // k per 16-byte chunk

    // Rows past the end point at an all-zero row (row `zero_row` of the residuals, row m of
    // the dictionary), so every staging load is unconditional.
    const int c4 = tile_c4(tid);
    const int r0 = tile_r0(tid);
    int64_t oR[S::LX], oA[S::LW];
#pragma unroll
    for (int q = 0; q < S::LX; ++q) {
        const int a = sig0 + r0 + S::RSTEP * q;
        const int s = a < n_act ? (act ? act[a] : a) : zero_row;
        oR[q] = (int64_t)s * ldr + VE * c4;
    }
#pragma unroll
    for (int q = 0; q < S::LW; ++q) {
        const int j = atom0 + r0 + S::RSTEP * q;
        oA[q] = (int64_t)(j < m ? j : m) * lda + VE * c4;
    }
    const int ws = (wave % S::WAVES_M) * WM;   // wave's signal offset in the tile
    const int wa = (wave / S::WAVES_M) * WN;   // wave's atom offset in the tile
    const int l32 = lane & 31;
    const int h = lane >> 5;
    floatx16 acc[S::TI][S::TJ];
    mfma_tile_loop<E, BM, BN, WM, WN, DEPTH>(Rbuf, oR, At, oA, kpad, lds, ws, wa, acc);

    store_tile<E, S::TI, S::TJ>(acc, sig0, ws, atom0, wa, l32, h, m, n_act, act, G, ldg, ascale, rscale);
}

// The same product with both operand tiles copied straight into swizzled LDS buffers (mfma_tile_loop_dma).
template <class E, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((TileShape<BM, BN, WM, WN>::THREADS)) void corr_gemm_dma_kernel(
    const E* __restrict__ At, int64_t lda, int m, int kpad,
    const E* __restrict__ Rbuf, int64_t ldr, const int* __restrict__ act,
    const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G, int64_t ldg, int tiles_n, int zero_row,
    int n_lo, int n_hi, const float* __restrict__ ascale, const float* __restrict__ rscale)
{
    using S = TileShape<BM, BN, WM, WN>;
    using D = DmaShape<BM, BN, WM, WN>;
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
    if (n_act < n_lo || n_act >= n_hi) return;   // another tile shape serves this running count
    const int tiles_m = ((n_act < p_grid ? n_act : p_grid) + BM - 1) / BM;   // as in corr_gemm_kernel
    const int nwg = tiles_m * tiles_n;
    if ((int)blockIdx.x >= nwg) return;
    const int tile = xcd_tile_index(blockIdx.x, nwg);
    int tm, tn;
    grouped_tile<8>(tile, tiles_m, tiles_n, tm, tn);
    if (tn >= tiles_n) return;
    const int sig0 = tm * BM;
    const int atom0 = tn * BN;
    if (sig0 >= n_act) return;

    __shared__ __attribute__((aligned(1024))) DmaLds<BM, BN> lds;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int VE = 16 / (int)sizeof(E);          // k per 16-byte chunk
    // rows past the end read an all-zero row (row zero_row of the residuals, row m of the dictionary)
    int64_t oR[D::GX], oA[D::GW];
#pragma unroll
    for (int i = 0; i < D::GX; ++i) {
        const int g = wave + S::WAVES * i;
        const int a = sig0 + dma_row(g, lane);
        const int sg = a < n_act ? (act ? act[a] : a) : zero_row;
        oR[i] = (int64_t)sg * ldr + VE * dma_chunk(g, lane);
    }
#pragma unroll
    for (int i = 0; i < D::GW; ++i) {
        const int g = wave + S::WAVES * i;
        const int j = atom0 + dma_row(g, lane);
        oA[i] = (int64_t)(j < m ? j : m) * lda + VE * dma_chunk(g, lane);
    }
    const int ws = (wave % S::WAVES_M) * WM;
    const int wa = (wave / S::WAVES_M) * WN;
    const int l32 = lane & 31;
    const int h = lane >> 5;
    floatx16 acc[S::TI][S::TJ];
    mfma_tile_loop_dma<E, BM, BN, WM, WN>(Rbuf, oR, At, oA, kpad, lds, ws, wa, acc);
    store_tile<E, S::TI, S::TJ>(acc, sig0, ws, atom0, wa, l32, h, m, n_act, act, G, ldg, ascale, rscale);
}

// ---------------------------------------------------------------------------------------------------
// bfloat16 product with the dictionary operand read straight from global memory into registers.
//
// The dictionary is fixed for a context, so its bfloat16 copy is also stored in the matrix
// instruction's fragment order (pack_bf16_fragments_kernel): for a block of 32 atoms and a chunk of 16
// k, the 64 lanes' 16-byte B fragments are one contiguous kilobyte (lane l: atom 32 jb + l % 32,
// k = 16 c + 8 (l / 32) .. + 8).  A wave loads its fragments with fully coalesced 16-byte loads, a
// whole stage (four chunks) ahead, and only the residual tile goes through LDS; this removes the
// dictionary's LDS stores and fragment reads, which bound the all-LDS loop for 16-bit operands.
// Atoms are padded to a multiple of 256 with zero fragments, so no load is predicated.
// ---------------------------------------------------------------------------------------------------
constexpr int PACK_ATOMS = 256;   // atom padding of the packed copy

__global__ __launch_bounds__(256) void pack_bf16_fragments_kernel(const uint16_t* __restrict__ A16, int64_t lda,
                                                                  int m, int kpad, uint4* __restrict__ Apk,
                                                                  int m_pad)
{
    const int nkc = kpad / 16;
    const int64_t total = (int64_t)(m_pad / 32) * nkc * 64;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int lane = (int)(e & 63);
        const int64_t fc = e >> 6;             // fragment index = jb * nkc + c
        const int c = (int)(fc % nkc);
        const int jb = (int)(fc / nkc);
        const int atom = 32 * jb + (lane & 31);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (atom < m) v = *reinterpret_cast<const uint4*>(A16 + (int64_t)atom * lda + 16 * c + 8 * (lane >> 5));
        Apk[e] = v;
    }
}

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((TileShape<BM, BN, WM, WN>::THREADS)) void corr_gemm_direct_kernel(
    const uint4* __restrict__ Apk, int m, int kpad, const __bf16* __restrict__ Rbuf, int64_t ldr,
    const int* __restrict__ act, const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G,
    int64_t ldg, int tiles_n, int zero_row, int n_lo, int n_hi)
{
    using S = TileShape<BM, BN, WM, WN>;
    constexpr int TI = S::TI, TJ = S::TJ;
    constexpr int LR = BM * 8 / S::THREADS;            // 16-byte residual loads per thread and stage
    static_assert(LR * S::THREADS == BM * 8, "residual staging");
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
    if (n_act < n_lo || n_act >= n_hi) return;   // another tile shape serves this running count
    const int tiles_m = ((n_act < p_grid ? n_act : p_grid) + BM - 1) / BM;   // as in corr_gemm_kernel
    const int nwg = tiles_m * tiles_n;
    if ((int)blockIdx.x >= nwg) return;
    const int tile = xcd_tile_index(blockIdx.x, nwg);
    int tm, tn;
    grouped_tile<8>(tile, tiles_m, tiles_n, tm, tn);
    if (tn >= tiles_n) return;
    const int sig0 = tm * BM;
    const int atom0 = tn * BN;
    if (sig0 >= n_act) return;

    __shared__ __attribute__((aligned(16))) char ldsR[2][BM * TILE_LDS_ROW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int c4 = tile_c4(tid);
    const int r0 = tile_r0(tid);
    int64_t oR[LR];
#pragma unroll
    for (int q = 0; q < LR; ++q) {
        const int a = sig0 + r0 + S::RSTEP * q;
        const int sg = a < n_act ? (act ? act[a] : a) : zero_row;
        oR[q] = (int64_t)sg * ldr + 8 * c4;
    }
    const int ws = (wave % S::WAVES_M) * WM;
    const int wa = (wave / S::WAVES_M) * WN;
    const int l32 = lane & 31;
    const int h = lane >> 5;
    const int nkc = kpad / 16;
    const uint4* aP[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) aP[j] = Apk + ((int64_t)((atom0 + wa) / 32 + j) * nkc) * 64 + lane;

    floatx16 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    float4 gR[LR];
    uint4 aC[4][TJ], aN[4][TJ];
#pragma unroll
    for (int q = 0; q < LR; ++q) gR[q] = *reinterpret_cast<const float4*>(Rbuf + oR[q]);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int j = 0; j < TJ; ++j) aC[kb][j] = aP[j][64 * kb];
#pragma unroll
    for (int q = 0; q < LR; ++q)
        *reinterpret_cast<float4*>(&ldsR[0][(r0 + S::RSTEP * q) * TILE_LDS_ROW + 16 * c4]) = gR[q];
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kpad; k0 += 64) {
        // next stage: residual slice into registers, dictionary fragments (the last stage re-reads itself)
        const int kn = k0 + 64 < kpad ? k0 + 64 : k0;
        const int cn = kn / 16;
#pragma unroll
        for (int q = 0; q < LR; ++q) gR[q] = *reinterpret_cast<const float4*>(Rbuf + oR[q] + kn);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < TJ; ++j) aN[kb][j] = aP[j][64 * (cn + kb)];
        asm volatile("" ::: "memory");
        const char* cR = ldsR[cur];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            float4 fx[TI];
#pragma unroll
            for (int i = 0; i < TI; ++i)
                fx[i] = *reinterpret_cast<const float4*>(&cR[(ws + 32 * i + l32) * TILE_LDS_ROW + kb * 32 + 16 * h]);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fx[i]),
                                                                       __builtin_bit_cast(bf16x8, aC[kb][j]),
                                                                       acc[i][j], 0, 0, 0);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < LR; ++q) {
            staged(gR[q]);   // see gemm_tile.h: keeps the residual load a stage ahead
            *reinterpret_cast<float4*>(&ldsR[cur ^ 1][(r0 + S::RSTEP * q) * TILE_LDS_ROW + 16 * c4]) = gR[q];
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < TJ; ++j) aC[kb][j] = aN[kb][j];
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int atom = atom0 + wa + 32 * j + l32;
            if (atom >= m) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = sig0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (a < n_act) G[(int64_t)a * ldg + atom] = acc[i][j][r];
            }
        }
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_direct(const uint16_t* Apk, int m, int kpad, const uint16_t* Rbuf, int64_t ldr, const int* act,
                         const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row, int n_lo, int n_hi,
                         hipStream_t stream)
{
    static_assert(PACK_ATOMS % BN == 0, "atom tiles must lie inside the packed padding");
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((corr_gemm_direct_kernel<BM, BN, WM, WN>), dim3((unsigned)nwg),
                       dim3(TileShape<BM, BN, WM, WN>::THREADS), 0, stream, reinterpret_cast<const uint4*>(Apk), m,
                       kpad, reinterpret_cast<const __bf16*>(Rbuf), ldr, act, n_act_dev, p_grid, G, ldg, tiles_n,
                       zero_row, n_lo, n_hi);
    return hipGetLastError();
}

template <class E, int BM, int BN, int WM, int WN, int DEPTH = 1>
hipError_t launch_shape(const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr,
                        const int* act, const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                        int n_lo, int n_hi, const float* ascale, const float* rscale, hipStream_t stream)
{
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((corr_gemm_kernel<E, BM, BN, WM, WN, DEPTH>), dim3((unsigned)nwg),
                       dim3(TileShape<BM, BN, WM, WN>::THREADS), 0, stream, At, lda, m, kpad, Rbuf, ldr, act,
                       n_act_dev, p_grid, G, ldg, tiles_n, zero_row, n_lo, n_hi, ascale, rscale);
    return hipGetLastError();
}

template <class E, int BM, int BN, int WM, int WN>
hipError_t launch_dma(const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr, const int* act,
                      const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row, int n_lo, int n_hi,
                      const float* ascale, const float* rscale, hipStream_t stream)
{
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((corr_gemm_dma_kernel<E, BM, BN, WM, WN>), dim3((unsigned)nwg),
                       dim3(TileShape<BM, BN, WM, WN>::THREADS), 0, stream, At, lda, m, kpad, Rbuf, ldr, act,
                       n_act_dev, p_grid, G, ldg, tiles_n, zero_row, n_lo, n_hi, ascale, rscale);
    return hipGetLastError();
}

template <class E>
hipError_t launch_variant(int variant, const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr,
                          const int* act, const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                          int n_lo, int n_hi, hipStream_t stream, const float* ascale = nullptr,
                          const float* rscale = nullptr)
{
    if (p_grid <= 0 || m <= 0) return hipSuccess;
    if (kpad % (TILE_ROW_BYTES / (int)sizeof(E))) return hipErrorInvalidValue;
    // float32 stages of the shapes with registers to spare load two stages ahead (faster: 604 -> 514 us
    // for the 256 x 128 tile at 1024 signals); 16- and 8-bit stages measured slower that way
    constexpr int DEEP = sizeof(E) == 4 ? 2 : 1;
    switch (variant) {
    case 0: return launch_shape<E, 128, 128, 64, 64, DEEP>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 1: return launch_shape<E, 256, 256, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 2: return launch_shape<E, 256, 128, 64, 64, DEEP>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 3: return launch_shape<E, 64, 128, 32, 64, DEEP>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 4: return launch_shape<E, 32, 64, 32, 32, DEEP>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 5: return launch_shape<E, 64, 64, 32, 32, DEEP>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 6: return launch_shape<E, 256, 256, 128, 128>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 7: return launch_shape<E, 256, 256, 128, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 11: return launch_dma<E, 256, 256, 128, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 12: return launch_dma<E, 256, 256, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 13: return launch_dma<E, 128, 128, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 14: return launch_dma<E, 256, 256, 128, 128>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

const char* corr_shape_name(int v)
{
    switch (v) {
    case 8: return "256x256 (8 waves of 128x64), dictionary fragments from global memory";
    case 9: return "128x256 (8 waves of 64x64), dictionary fragments from global memory";
    case 10: return "256x128 (4 waves of 128x64), dictionary fragments from global memory";
    case 0: return "128x128 (4 waves of 64x64)";
    case 1: return "256x256 (16 waves of 64x64)";
    case 2: return "256x128 (8 waves of 64x64)";
    case 3: return "64x128 (4 waves of 32x64)";
    case 4: return "32x64 (2 waves of 32x32)";
    case 5: return "64x64 (4 waves of 32x32)";
    case 6: return "256x256 (4 waves of 128x128)";
    case 7: return "256x256 (8 waves of 128x64)";
    case 11: return "256x256 (8 waves of 128x64), operand tiles copied straight into LDS";
    case 12: return "256x256 (16 waves of 64x64), operand tiles copied straight into LDS";
    case 13: return "128x128 (4 waves of 64x64), operand tiles copied straight into LDS";
    case 14: return "256x256 (4 waves of 128x128), operand tiles copied straight into LDS";
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

hipError_t launch_corr_gemm_fp8(int variant, const uint8_t* A8, int64_t lda, int m, int kpad,
                                const uint8_t* R8, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                int n_lo, int n_hi, const float* ascale, const float* rscale, hipStream_t stream)
{
    if (!ascale || !rscale) return hipErrorInvalidValue;
    return launch_variant<uint8_t>(variant, A8, lda, m, kpad, R8, ldr, act, n_act_dev, p_grid, G, ldg, zero_row,
                                   n_lo, n_hi, stream, ascale, rscale);
}

size_t packed_bf16_elems(int m, int kpad)
{
    return (size_t)((m + PACK_ATOMS - 1) / PACK_ATOMS * PACK_ATOMS) * (size_t)kpad;
}

hipError_t launch_pack_bf16(const uint16_t* A16, int64_t lda, int m, int kpad, uint16_t* Apk, hipStream_t stream)
{
    if (kpad % 64) return hipErrorInvalidValue;
    const int m_pad = (m + PACK_ATOMS - 1) / PACK_ATOMS * PACK_ATOMS;
    const int64_t total = (int64_t)(m_pad / 32) * (kpad / 16) * 64;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(pack_bf16_fragments_kernel, dim3(grid), dim3(256), 0, stream, A16, lda, m, kpad,
                       reinterpret_cast<uint4*>(Apk), m_pad);
    return hipGetLastError();
}

hipError_t launch_corr_gemm_bf16(int variant, const uint16_t* At, const uint16_t* Apk, int64_t lda, int m, int kpad,
                                 const uint16_t* Rbuf, int64_t ldr, const int* act,
                                 const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                                 int n_lo, int n_hi, hipStream_t stream)
{
    if (variant >= 8 && variant <= 10) {
        if (!Apk || p_grid <= 0 || m <= 0) return Apk ? hipSuccess : hipErrorInvalidValue;
        if (kpad % 64) return hipErrorInvalidValue;
        switch (variant) {
        case 8: return launch_direct<256, 256, 128, 64>(Apk, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
        case 9: return launch_direct<128, 256, 64, 64>(Apk, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
        case 10: return launch_direct<256, 128, 128, 64>(Apk, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, stream);
        default: return hipErrorInvalidValue;
        }
    }
    return launch_variant<__bf16>(variant, reinterpret_cast<const __bf16*>(At), lda, m, kpad,
                                  reinterpret_cast<const __bf16*>(Rbuf), ldr, act, n_act_dev, p_grid, G, ldg,
                                  zero_row, n_lo, n_hi, stream);
}

}  // namespace bmpl
