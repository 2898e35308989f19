// Gram table Q = A^T A in float64 (the precomputed Q of Section III, Eq. (12)).
//
// The batch mode of the paper precomputes Q once per dictionary and amortises
// it over all signals (Remark 1).  Here Q serves the master problem: the Gram
// rows G_{J,I} of the atoms entering an active set become gathers from Q
// instead of n-long float64 dot products per pair.  Entries are accumulated in
// float64 from the float32 atoms (every product is exact in float64), so they
// equal the directly computed Gram entries up to summation order.
//
// A dense symmetric rank-n update on the float64 matrix cores:
// v_mfma_f64_16x16x4f64, 128 x 128 output tiles per 256-thread workgroup (each
// wave 64 x 64 = 4 x 4 blocks), K staged through LDS 16 at a time with the
// float32 -> float64 conversion done once at staging.  Only tiles on or below
// the diagonal are computed; each entry on or below the diagonal is written to
// both triangles, so Q is exactly symmetric.
#include "bmpl_internal.h"

namespace bmpl {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int TB = 128;          // tile edge
constexpr int KB = 16;           // k per LDS stage
constexpr int LS = KB + 1;       // LDS row stride (doubles)

__global__ __launch_bounds__(256) void gram_table_kernel(const float* __restrict__ At, int64_t lda, int m,
                                                         int kpad, double* __restrict__ Q, int64_t ldq, int T)
{
    // blockIdx.x enumerates lower-triangle tiles (ti >= tj) row by row.
    const int64_t b = blockIdx.x;
    int ti = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) / 2.0);
    while ((int64_t)ti * (ti + 1) / 2 > b) --ti;
    while ((int64_t)(ti + 1) * (ti + 2) / 2 <= b) ++ti;
    const int tj = (int)(b - (int64_t)ti * (ti + 1) / 2);
    if (ti >= T || tj > ti) return;
    const int i0 = ti * TB, j0 = tj * TB;

    __shared__ double sI[TB * LS];
    __shared__ double sJ[TB * LS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;

    doublex4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = doublex4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < kpad; k0 += KB) {
        // stage 128 atoms x 16 k of each operand: 2048 values, 8 per thread
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int r = e >> 4, kk = e & 15;
            const int ai = i0 + r, aj = j0 + r;
            const int k = k0 + kk;
            sI[r * LS + kk] = (ai < m && k < kpad) ? (double)At[(int64_t)ai * lda + k] : 0.0;
            sJ[r * LS + kk] = (aj < m && k < kpad) ? (double)At[(int64_t)aj * lda + k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KB; ks += 4) {
            double fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = sI[(wi + 16 * a + (lane & 15)) * LS + ks + (lane >> 4)];
#pragma unroll
            for (int c = 0; c < 4; ++c) fb[c] = sJ[(wj + 16 * c + (lane & 15)) * LS + ks + (lane >> 4)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[c], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
    }
    // D of a float64 16x16x4 block: lane l, element r -> row l/16 + 4r, column l%16.
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wi + 16 * a + (lane >> 4) + 4 * r;
                const int gj = j0 + wj + 16 * c + (lane & 15);
                if (gi < m && gj < m && !(ti == tj && gi < gj)) {
                    Q[(int64_t)gi * ldq + gj] = acc[a][c][r];
                    Q[(int64_t)gj * ldq + gi] = acc[a][c][r];
                }
            }
}

}  // namespace

hipError_t launch_gram_table(const float* At, int64_t lda, int m, int kpad, double* Q, int64_t ldq,
                             hipStream_t stream)
{
    const int T = (m + TB - 1) / TB;
    const int64_t nblk = (int64_t)T * (T + 1) / 2;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gram_table_kernel, dim3((unsigned)nblk), dim3(256), 0, stream, At, lda, m, kpad, Q, ldq, T);
    return hipGetLastError();
}

}  // namespace bmpl
