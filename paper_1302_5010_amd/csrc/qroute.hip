// The correlation of Section III's batch mode (Eq. (12)): with beta = A^T b kept
// from the start and the precomputed Q = A^T A (Remark 1),
//     g = A^T (b - A x) = beta - Q_{:,S} x_S,
// so an outer iteration streams |S| rows of Q per signal instead of multiplying
// A^T by the residual.  Both kernels accumulate in float64 from float32 atoms and
// signals (beta) and from the float64 Q and x.
//
// atb_f64_kernel: beta[i][j] = a_j^T b_i for all signals and atoms, a 64 x 64
//   output tile (signals x atoms) per workgroup, operands staged through LDS.
// q_corr_kernel: per running signal and chunk of 1024 atoms, the support's
//   (atom, x) pairs staged in LDS, then g_j = beta_j - sum_k x_k Q[atom_k][j]
//   with threads along j (each Q row read coalesced), stored as float32 for the
//   selection.
#include "bmpl_internal.h"
#include "qroute.h"

namespace bmpl {
namespace {

__global__ __launch_bounds__(256) void atb_f64_kernel(const float* __restrict__ At, int64_t lda, int m,
                                                      const float* __restrict__ Bw, int64_t ldb, int p, int n,
                                                      double* __restrict__ beta, int64_t ldbeta)
{
    __shared__ float sB[16][64];
    __shared__ float sA[16][64];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, kk = e & 15, rr = e >> 4;   // 64 rows x 16 k per operand
            const int k = k0 + kk;
            sB[kk][rr] = (i0 + rr < p && k < n) ? Bw[(int64_t)(i0 + rr) * ldb + k] : 0.f;
            sA[kk][rr] = (j0 + rr < m && k < n) ? At[(int64_t)(j0 + rr) * lda + k] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double bv[4], av[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) { bv[a] = sB[kk][4 * ty + a]; av[a] = sA[kk][4 * tx + a]; }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(bv[a], av[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + 4 * ty + a;
        if (i >= p) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + 4 * tx + b;
            if (j < m) beta[(int64_t)i * ldbeta + j] = acc[a][b];
        }
    }
}

constexpr int QCHUNK = 1024;       // atoms per workgroup (4 per thread)
constexpr int QSTAGE = 512;        // support entries staged in LDS at a time

__global__ __launch_bounds__(256) void q_corr_kernel(QCorrArgs a)
{
    __shared__ int s_atom[QSTAGE];
    __shared__ double s_x[QSTAGE];
    const int n_act = *a.n_act_dev;
    const int row = blockIdx.y;
    if (row >= n_act) return;
    const int sig = a.act[row];
    const int j0 = blockIdx.x * QCHUNK;
    const int tid = threadIdx.x;
    const Workspace& w = a.w;
    const int nS = w.blk[sig] ? w.nS[sig] : 0;
    const SlotBlock b = slot_block(w.blk[sig], w.cap[sig], w.n);   // only read when nS > 0
    double g[QCHUNK / 256];
#pragma unroll
    for (int t = 0; t < QCHUNK / 256; ++t) {
        const int j = j0 + tid + 256 * t;
        g[t] = j < w.m ? a.beta[(int64_t)sig * a.ldbeta + j] : 0.0;
    }
    for (int k0 = 0; k0 < nS; k0 += QSTAGE) {
        const int nk = nS - k0 < QSTAGE ? nS - k0 : QSTAGE;
        __syncthreads();
        for (int k = tid; k < nk; k += 256) {
            const int u = b.sord[k0 + k];
            s_atom[k] = b.atom[u];
            s_x[k] = b.x[u];
        }
        __syncthreads();
        int k = 0;
        if (j0 + QCHUNK <= w.m) {
            // a chunk inside the row: four rows of Q (sixteen loads per thread) requested together; a
            // guarded load compiles to a branch that waits for its data, one row after another
            for (; k + 4 <= nk; k += 4) {
                double qv[4][QCHUNK / 256];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double* qrow = a.Q + (int64_t)s_atom[k + e] * a.ldq + j0 + tid;
#pragma unroll
                    for (int t = 0; t < QCHUNK / 256; ++t) qv[e][t] = qrow[256 * t];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double xk = s_x[k + e];
#pragma unroll
                    for (int t = 0; t < QCHUNK / 256; ++t) g[t] -= xk * qv[e][t];
                }
            }
        }
        for (; k < nk; ++k) {
            const double xk = s_x[k];
            const double* qrow = a.Q + (int64_t)s_atom[k] * a.ldq;
#pragma unroll
            for (int t = 0; t < QCHUNK / 256; ++t) {
                const int j = j0 + tid + 256 * t;
                if (j < w.m) g[t] -= xk * qrow[j];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < QCHUNK / 256; ++t) {
        const int j = j0 + tid + 256 * t;
        if (j < w.m) a.G[(int64_t)row * a.ldg + j] = (float)g[t];
    }
}

}  // namespace

hipError_t launch_atb_f64(const float* At, int64_t lda, int m, const float* Bw, int64_t ldb, int p, int n,
                          double* beta, int64_t ldbeta, hipStream_t s)
{
    if (p <= 0 || m <= 0) return hipSuccess;
    dim3 grid((m + 63) / 64, (p + 63) / 64);
    hipLaunchKernelGGL(atb_f64_kernel, grid, dim3(256), 0, s, At, lda, m, Bw, ldb, p, n, beta, ldbeta);
    return hipGetLastError();
}

hipError_t launch_q_corr(const QCorrArgs& a, hipStream_t s)
{
    if (a.p_grid <= 0) return hipSuccess;
    dim3 grid((a.w.m + QCHUNK - 1) / QCHUNK, a.p_grid);
    hipLaunchKernelGGL(q_corr_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace bmpl
