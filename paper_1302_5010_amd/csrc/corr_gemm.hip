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
#include "bmpl_internal.h"
#include "gemm_tile.h"

namespace bmpl {
namespace {

template <class E, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((TileShape<BM, BN, WM, WN>::THREADS)) void corr_gemm_kernel(
    const E* __restrict__ At, int64_t lda, int m, int kpad,
    const E* __restrict__ Rbuf, int64_t ldr, const int* __restrict__ act,
    const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G, int64_t ldg, int tiles_n, int zero_row,
    int n_lo, int n_hi, const float* __restrict__ ascale, const float* __restrict__ rscale)
{
    using S = TileShape<BM, BN, WM, WN>;
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
    if (n_act < n_lo || n_act >= n_hi) return;   // another tile shape serves this running count
    const int tile = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tm = tile % tiles_m;          // signal tile (signal tiles inner: an XCD's run shares atom rows)
    const int tn = tile / tiles_m;          // atom tile
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
    mfma_tile_loop<E, BM, BN, WM, WN>(Rbuf, oR, At, oA, kpad, lds, ws, wa, acc);

    // D[row][col] of a 32x32 block (both instructions): lane l, register r -> row 8(r/4) + 4(l/32) + r%4,
    // col l%32.
    if constexpr (sizeof(E) == 1) {
        // e4m3 operands carry power-of-two scales: one per atom, one per signal
#pragma unroll
        for (int i = 0; i < S::TI; ++i)
#pragma unroll
            for (int j = 0; j < S::TJ; ++j) {
                const int atom = atom0 + wa + 32 * j + l32;
                if (atom >= m) continue;
                const float sa = ascale[atom];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int a = sig0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                    if (a < n_act) G[(int64_t)a * ldg + atom] = acc[i][j][r] * sa * rscale[act ? act[a] : a];
                }
            }
    } else {
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
}

template <class E, int BM, int BN, int WM, int WN>
hipError_t launch_shape(const E* At, int64_t lda, int m, int kpad, const E* Rbuf, int64_t ldr,
                        const int* act, const int* n_act_dev, int p_grid, float* G, int64_t ldg, int zero_row,
                        int n_lo, int n_hi, const float* ascale, const float* rscale, hipStream_t stream)
{
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((corr_gemm_kernel<E, BM, BN, WM, WN>), dim3((unsigned)nwg),
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
    switch (variant) {
    case 0: return launch_shape<E, 128, 128, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 1: return launch_shape<E, 256, 256, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 2: return launch_shape<E, 256, 128, 64, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 3: return launch_shape<E, 64, 128, 32, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 4: return launch_shape<E, 32, 64, 32, 32>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 5: return launch_shape<E, 64, 64, 32, 32>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 6: return launch_shape<E, 256, 256, 128, 128>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    case 7: return launch_shape<E, 256, 256, 128, 64>(At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, zero_row, n_lo, n_hi, ascale, rscale, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

const char* corr_shape_name(int v)
{
    switch (v) {
    case 0: return "128x128 (4 waves of 64x64)";
    case 1: return "256x256 (16 waves of 64x64)";
    case 2: return "256x128 (8 waves of 64x64)";
    case 3: return "64x128 (4 waves of 32x64)";
    case 4: return "32x64 (2 waves of 32x32)";
    case 5: return "64x64 (4 waves of 32x32)";
    case 6: return "256x256 (4 waves of 128x128)";
    case 7: return "256x256 (8 waves of 128x64)";
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
