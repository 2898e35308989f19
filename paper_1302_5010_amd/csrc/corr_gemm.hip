// Batched correlation G = A^T Xi on MFMA (float32).
//
// One outer iteration of the batched pursuit needs g_i = A^T xi_i for every
// running signal i: the full matrix-vector product of the worst-case analysis
// (Algorithm 1, step 3), done for all signals at once.  It is a dense
// contraction over the signal length n, so it runs on the matrix cores:
// M = running signals, N = atoms, K = n, both operands K-contiguous (the
// dictionary is stored atom by atom, residuals signal by signal).
//
// Tiling (gfx950, wave64): a 256-thread workgroup computes a 128 (signals) x
// 128 (atoms) tile; each wave a 64 x 64 sub-tile as 2 x 2 v_mfma_f32_32x32x2f32
// blocks (64 accumulator registers).  K is consumed 32 at a time through LDS;
// the next K-slice is prefetched into registers while the current one is used.
// Within each 8-wide k block, lane half h supplies k = 8b + 4h + t at step t, so
// every LDS fragment read is one 16-byte ds_read per 4 MFMAs (the summation
// order over k is immaterial to the contraction).
//
// Output: G[a*ldg + j], a = compact index of the running signal, j = atom.  The
// MFMA's row index carries the signal and its column (lane) index the atom, so
// each accumulator register stores 32 consecutive atoms of one signal per
// half-wave (coalesced 128-byte stores).
#include "bmpl_internal.h"

namespace bmpl {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128;   // signals per workgroup tile
constexpr int BN = 128;   // atoms per workgroup tile
constexpr int BK = 32;    // k per LDS stage
constexpr int LDS_STRIDE = BK + 4;   // floats per LDS row (16-byte aligned, staggers banks)

__global__ __launch_bounds__(256) void corr_gemm_f32_kernel(
    const float* __restrict__ At, int64_t lda, int m, int kpad,
    const float* __restrict__ Rbuf, int64_t ldr, const int* __restrict__ act,
    const int* __restrict__ n_act_dev, int p_grid, float* __restrict__ G, int64_t ldg,
    int tiles_n)
{
    const int n_act = n_act_dev ? *n_act_dev : p_grid;
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

    __shared__ float sR[BM * LDS_STRIDE];
    __shared__ float sA[BN * LDS_STRIDE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // Global -> register staging: 4 float4 per operand per thread.
    const int c4 = tid & 7;       // which float4 of the 32-wide k slice
    const int r0 = tid >> 3;      // row 0..31, +32q
    const float* pR[4];
    const float* pA[4];
    bool vR[4], vA[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int a = sig0 + r0 + 32 * q;
        vR[q] = a < n_act;
        int s = vR[q] ? (act ? act[a] : a) : 0;
        pR[q] = Rbuf + (int64_t)s * ldr + 4 * c4;
        int j = atom0 + r0 + 32 * q;
        vA[q] = j < m;
        pA[q] = At + (int64_t)(vA[q] ? j : 0) * lda + 4 * c4;
    }
    float4 gR[4], gA[4];
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    auto load_slice = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            gR[q] = vR[q] ? *reinterpret_cast<const float4*>(pR[q] + k0) : zero4;
            gA[q] = vA[q] ? *reinterpret_cast<const float4*>(pA[q] + k0) : zero4;
        }
    };
    auto store_slice = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<float4*>(&sR[(r0 + 32 * q) * LDS_STRIDE + 4 * c4]) = gR[q];
            *reinterpret_cast<float4*>(&sA[(r0 + 32 * q) * LDS_STRIDE + 4 * c4]) = gA[q];
        }
    };

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int ws = (wave & 1) * 64;    // wave's signal offset in the tile
    const int wa = (wave >> 1) * 64;   // wave's atom offset in the tile
    const int l32 = lane & 31;
    const int h = lane >> 5;

    load_slice(0);
    store_slice();
    __syncthreads();
    for (int k0 = 0; k0 < kpad; k0 += BK) {
        const bool more = k0 + BK < kpad;
        if (more) load_slice(k0 + BK);
#pragma unroll
        for (int kb = 0; kb < BK / 8; ++kb) {
            float4 fr[2], fa[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                fr[i] = *reinterpret_cast<const float4*>(&sR[(ws + 32 * i + l32) * LDS_STRIDE + kb * 8 + 4 * h]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fa[j] = *reinterpret_cast<const float4*>(&sA[(wa + 32 * j + l32) * LDS_STRIDE + kb * 8 + 4 * h]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].x, fa[j].x, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].y, fa[j].y, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].z, fa[j].z, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fr[i].w, fa[j].w, acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
        if (more) {
            store_slice();
            __syncthreads();
        }
    }

    // D[row][col] of a 32x32x2 block: lane l, register r -> row 8(r/4) + 4(l/32) + r%4, col l%32.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int atom = atom0 + wa + 32 * j + l32;
            if (atom >= m) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = sig0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (a < n_act) G[(int64_t)a * ldg + atom] = acc[i][j][r];
            }
        }
}

}  // namespace

hipError_t launch_corr_gemm_f32(const float* At, int64_t lda, int m, int kpad,
                                const float* Rbuf, int64_t ldr, const int* act,
                                const int* n_act_dev, int p_grid, float* G, int64_t ldg,
                                hipStream_t stream)
{
    if (p_grid <= 0 || m <= 0) return hipSuccess;
    const int tiles_m = (p_grid + BM - 1) / BM;
    const int tiles_n = (m + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(corr_gemm_f32_kernel, dim3((unsigned)nwg), dim3(256), 0, stream,
                       At, lda, m, kpad, Rbuf, ldr, act, n_act_dev, p_grid, G, ldg, tiles_n);
    return hipGetLastError();
}

}  // namespace bmpl
