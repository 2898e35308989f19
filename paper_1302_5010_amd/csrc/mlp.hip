// Kernels of the learned support proposal: a small network that scores every
// atom for a signal so that the pursuit can start from a good active set
// (the warm start of Algorithm 1, step 5, taken from outside the method; the
// natural stopping condition, Eq. (9), still certifies the result).
//
//   embedding   z = (A P)^T b, then scaled to unit root-mean-square
//   network     h1 = gelu(W1 z + b1), h2 = gelu(W2 h1 + b2), s = W3 h2 + b3
//   loss        binary cross-entropy with logits, positive-class weight w
//   training    gradients by the chain rule, Adam with float32 master weights
//   proposal    the k largest scores per signal (radix select, ties to the lower index)
//
// Precision: weights and activations in bfloat16 for the matrix products,
// float32 accumulation, float32 pre-activations, logits, gradients and
// optimiser state.  All products C = X W^T run on the shared MFMA tile loop
// with both operands K-contiguous; the backward products that contract over
// the batch or the output width use bfloat16 transposes made for them.
#include <float.h>

#include <algorithm>

#include "bmpl_internal.h"
#include "gemm_tile.h"
#include "mlp.h"

namespace bmpl {
namespace {

__device__ inline float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float gelu_f(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }

__device__ inline float gelu_prime_f(float u)
{
    return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

// ---------------------------------------------------------------------------
// Epilogues of C = X W^T: called once per output element (row r of X, row c of W).
// ---------------------------------------------------------------------------
struct EpiStore {            // C[r][c] = v (+ bias[c])
    float* C; int64_t ldc; const float* bias;
    __device__ void operator()(int r, int c, float v) const
    {
        C[(int64_t)r * ldc + c] = bias ? v + bias[c] : v;
    }
};
struct EpiBiasGelu {         // u = v + bias[c]; U[r][c] = u (if kept); H[r][c] = bf16(gelu(u))
    const float* bias; float* U; int64_t ldu; uint16_t* H; int64_t ldh;
    __device__ void operator()(int r, int c, float v) const
    {
        const float u = v + bias[c];
        if (U) U[(int64_t)r * ldu + c] = u;
        H[(int64_t)r * ldh + c] = bf16_round(gelu_f(u));
    }
};
struct EpiGeluBack {         // d = v * gelu'(U[r][c]); D[r][c] = d; D16[r][c] = bf16(d)
    const float* U; int64_t ldu; float* D; int64_t ldd; uint16_t* D16; int64_t ld16;
    __device__ void operator()(int r, int c, float v) const
    {
        const float d = v * gelu_prime_f(U[(int64_t)r * ldu + c]);
        D[(int64_t)r * ldd + c] = d;
        D16[(int64_t)r * ld16 + c] = bf16_round(d);
    }
};

// C[r][c] = sum_k X[r][k] W[c][k] for r < M, c < N; kpad % 64 == 0 and both operands hold
// zeros in columns past the true contraction length.  Rows past M (N) re-read row M-1 (N-1);
// their results are never stored.
template <int BM, int BN, int WM, int WN, class Epi>
__global__ __launch_bounds__((TileShape<BM, BN, WM, WN>::THREADS)) void mlp_gemm_kernel(
    const __bf16* __restrict__ X, int64_t ldx, int M, const __bf16* __restrict__ W, int64_t ldw, int N, int kpad,
    int tiles_m, int tiles_n, Epi epi)
{
    using S = TileShape<BM, BN, WM, WN>;
    const int tile = xcd_tile_index(blockIdx.x, gridDim.x);
    int tm, tn;                              // grouped order: an XCD's concurrent tiles share X and W rows
    grouped_tile<8>(tile, tiles_m, tiles_n, tm, tn);
    if (tn >= tiles_n) return;
    const int row0 = tm * BM, col0 = tn * BN;

    __shared__ __attribute__((aligned(16))) TileLds<BM, BN> lds;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int c4 = tile_c4(tid);
    const int r0 = tile_r0(tid);
    int64_t oX[S::LX], oW[S::LW];
#pragma unroll
    for (int q = 0; q < S::LX; ++q) {
        const int r = row0 + r0 + S::RSTEP * q;
        oX[q] = (int64_t)(r < M ? r : M - 1) * ldx + 8 * c4;
    }
#pragma unroll
    for (int q = 0; q < S::LW; ++q) {
        const int c = col0 + r0 + S::RSTEP * q;
        oW[q] = (int64_t)(c < N ? c : N - 1) * ldw + 8 * c4;
    }
    const int ws = (wave % S::WAVES_M) * WM;
    const int wa = (wave / S::WAVES_M) * WN;
    floatx16 acc[S::TI][S::TJ];
    mfma_tile_loop<__bf16, BM, BN, WM, WN>(X, oX, W, oW, kpad, lds, ws, wa, acc);

    const int l32 = lane & 31;
    const int h = lane >> 5;
#pragma unroll
    for (int i = 0; i < S::TI; ++i)
#pragma unroll
        for (int j = 0; j < S::TJ; ++j) {
            const int c = col0 + wa + 32 * j + l32;
            if (c >= N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + ws + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (row < M) epi(row, c, acc[i][j][r]);
            }
        }
}

template <int BM, int BN, int WM, int WN, class Epi>
hipError_t launch_gemm_shape(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                             const Epi& epi, hipStream_t s)
{
    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    const int64_t nwg = (int64_t)tiles_m * tiles_n;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mlp_gemm_kernel<BM, BN, WM, WN, Epi>), dim3((unsigned)nwg),
                       dim3(TileShape<BM, BN, WM, WN>::THREADS), 0, s, reinterpret_cast<const __bf16*>(X), ldx, M,
                       reinterpret_cast<const __bf16*>(W), ldw, N, kpad, tiles_m, tiles_n, epi);
    return hipGetLastError();
}

template <class Epi>
hipError_t launch_gemm(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                       const Epi& epi, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (kpad <= 0 || kpad % 64 || ldx % 8 || ldw % 8 || ldx < kpad || ldw < kpad) return hipErrorInvalidValue;
    // very large outputs (four or more rounds of 256 x 256 tiles on 256 CUs): eight 128 x 64 waves per
    // tile; large ones: 128 x 128 tiles of four 64 x 64 waves; small ones: 64 x 64 tiles of 32 x 32 waves
    if ((int64_t)((M + 255) / 256) * ((N + 255) / 256) >= 1024)
        return launch_gemm_shape<256, 256, 128, 64>(X, ldx, M, W, ldw, N, kpad, epi, s);
    if ((int64_t)((M + 127) / 128) * ((N + 127) / 128) >= 512)
        return launch_gemm_shape<128, 128, 64, 64>(X, ldx, M, W, ldw, N, kpad, epi, s);
    return launch_gemm_shape<64, 64, 32, 32>(X, ldx, M, W, ldw, N, kpad, epi, s);
}

// ---------------------------------------------------------------------------
// (A P)^T: APt[c][i] = sum_j P[j][c] A[j][i] in float32, written as bfloat16 [d][npad]
// (zeros past n).  A one-time precomputation: a plain 64 x 64 LDS-tiled product.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ At, int64_t lda, int n, int m,
                                                      const float* __restrict__ P, int d, uint16_t* __restrict__ APt,
                                                      int npad)
{
    __shared__ float sP[16][64];
    __shared__ float sA[16][64];
    const int c0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    float acc[4][4] = {};
    for (int j0 = 0; j0 < m; j0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, jj = e >> 6, cc = e & 63;
            const int j = j0 + jj;
            sP[jj][cc] = (j < m && c0 + cc < d) ? P[(int64_t)j * d + c0 + cc] : 0.f;
            sA[jj][cc] = (j < m && i0 + cc < n) ? At[(int64_t)j * lda + i0 + cc] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            float pv[4], av[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) { pv[a] = sP[jj][4 * ty + a]; av[a] = sA[jj][4 * tx + a]; }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(pv[a], av[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int c = c0 + 4 * ty + a;
        if (c >= d) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + 4 * tx + b;
            if (i < npad) APt[(int64_t)c * npad + i] = i < n ? bf16_round(acc[a][b]) : (uint16_t)0;
        }
    }
}

// Signals to bfloat16 rows [p][npad], zeros past n.
__global__ __launch_bounds__(256) void signals_bf16_kernel(const float* __restrict__ B, int64_t ldb, int n,
                                                           uint16_t* __restrict__ B16, int npad)
{
    const int r = blockIdx.x;
    for (int i = threadIdx.x; i < npad; i += 256)
        B16[(int64_t)r * npad + i] = i < n ? bf16_round(B[(int64_t)r * ldb + i]) : (uint16_t)0;
}

// X0[r] = bf16(Z[r] * sqrt(d) / ||Z[r]||) (a zero row stays zero); optionally X0 widened to Zout.
__global__ __launch_bounds__(256) void embed_norm_kernel(const float* __restrict__ Z, int d,
                                                         uint16_t* __restrict__ X0, float* __restrict__ Zout,
                                                         int64_t ldz_out)
{
    __shared__ double red[4];
    const int r = blockIdx.x;
    const float* z = Z + (int64_t)r * d;
    double s = 0.0;
    for (int c = threadIdx.x; c < d; c += 256) s += (double)z[c] * z[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    const double nrm = sqrt(red[0] + red[1] + red[2] + red[3]);
    const float scale = nrm > 0.0 ? (float)(sqrt((double)d) / nrm) : 0.f;
    for (int c = threadIdx.x; c < d; c += 256) {
        const uint16_t v = bf16_round(z[c] * scale);
        X0[(int64_t)r * d + c] = v;
        if (Zout) Zout[(int64_t)r * ldz_out + c] = bf16_to_f(v);
    }
}

// Weighted binary cross-entropy with logits, one workgroup per signal.  In place:
// S[r][j] (logit) becomes dl/ds divided by the batch size; D16 gets its bfloat16 copy with zeros
// in columns m..mpad-1; rowloss[r] = sum_j l(s_j, y_j).  Targets y_j = 1 for the atoms listed in
// supp[r][0..len[r]).
constexpr int BCE_MAX_WORDS = 4096;    // m <= 131072
__global__ __launch_bounds__(256) void bce_grad_kernel(float* __restrict__ S, int64_t lds,
                                                       uint16_t* __restrict__ D16, int64_t ld16, int m, int mpad,
                                                       const int* __restrict__ supp, int64_t ld_supp,
                                                       const int* __restrict__ supp_len, float pos_w, float inv_batch,
                                                       float* __restrict__ rowloss)
{
    __shared__ uint32_t bits[BCE_MAX_WORDS];
    __shared__ double red[4];
    const int r = blockIdx.x;
    const int words = (m + 31) >> 5;
    for (int w = threadIdx.x; w < words; w += 256) bits[w] = 0u;
    __syncthreads();
    const int len = min(supp_len[r], (int)ld_supp);
    for (int t = threadIdx.x; t < len; t += 256) {
        const int j = supp[(int64_t)r * ld_supp + t];
        if (j >= 0 && j < m) atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    double part = 0.0;
    float* s = S + (int64_t)r * lds;
    for (int j = threadIdx.x; j < mpad; j += 256) {
        if (j >= m) { D16[(int64_t)r * ld16 + j] = 0; continue; }
        const float x = s[j];
        const bool y = (bits[j >> 5] >> (j & 31)) & 1u;
        const float e = expf(-fabsf(x));
        const float sp_pos = fmaxf(x, 0.f) + log1pf(e);     // log(1 + e^x)
        const float sp_neg = fmaxf(-x, 0.f) + log1pf(e);    // log(1 + e^-x)
        part += y ? (double)pos_w * sp_neg : (double)sp_pos;
        const float sig = x >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
        const float g = (y ? sig * pos_w - pos_w : sig) * inv_batch;
        s[j] = g;
        D16[(int64_t)r * ld16 + j] = bf16_round(g);
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) rowloss[r] = (float)(red[0] + red[1] + red[2] + red[3]);
}

// loss = sum_r rowloss[r] / rows (one workgroup).
__global__ __launch_bounds__(256) void loss_sum_kernel(const float* __restrict__ rowloss, int rows, double* loss)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += 256) s += rowloss[r];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *loss = (red[0] + red[1] + red[2] + red[3]) / rows;
}

// out[c] = sum_{r < rows} in[r][c]  (bias gradients).
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ in, int64_t ld, int rows, int cols,
                                                     float* __restrict__ out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += in[(int64_t)r * ld + c];
    out[c] = (float)s;
}

// out[c][r] = in[r][c] for c < cols, r < rows; out[c][r] = 0 for rows <= r < ldo (ldo % 64 == 0).
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t* __restrict__ in, int64_t ldi, int rows,
                                                             int cols, uint16_t* __restrict__ out, int64_t ldo)
{
    __shared__ uint16_t t[64][66];
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int q = ty; q < 64; q += 4) {
        const int r = r0 + q, c = c0 + tx;
        t[q][tx] = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
        const int c = c0 + q, r = r0 + tx;
        if (c < cols && r < ldo) out[(int64_t)c * ldo + r] = t[tx][q];
    }
}

// Adam with bias correction (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t); refreshes the bfloat16 copy.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ P, float* __restrict__ m1,
                                                   float* __restrict__ m2, const float* __restrict__ g,
                                                   uint16_t* __restrict__ P16, int64_t count, float lr, float beta1,
                                                   float beta2, float eps, float bc1, float bc2)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float a = beta1 * m1[i] + (1.f - beta1) * gi;
        const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float v = P[i] - lr * (a / bc1) / (sqrtf(b / bc2) + eps);
        P[i] = v;
        P16[i] = bf16_round(v);
    }
}

__global__ __launch_bounds__(256) void params_bf16_kernel(const float* __restrict__ P, uint16_t* __restrict__ P16,
                                                          int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        P16[i] = bf16_round(P[i]);
}

// ---------------------------------------------------------------------------
// Top-k per row (k <= 256), ties to the lower index, output ascending by atom index,
// padded with -1 when the row is shorter than k.  One workgroup per row.
//   1. Each thread keeps the two largest order keys of its entries; the k-th largest of
//      those 512 keys, T, is at most the row's k-th largest key (they are distinct
//      entries of the row), so every entry of the top k has a key >= T.
//   2. Each wave compacts, in index order, the entries of its quarter of the row with a
//      key >= T (typically a few hundred in all) into LDS as (key, index) pairs.
//   3. A bitonic sort orders the candidates by key, then lower index; the first k are
//      the answer, whose indices a second bitonic sort puts in ascending order.
// If a quarter holds more candidates than its LDS share (many equal keys), the row is
// done by an exact radix select over the keys in global memory instead.
// ---------------------------------------------------------------------------
__device__ inline uint32_t order_key(float x)
{
    if (x != x) return 0u;                     // NaN ranks below everything
    uint32_t u = __float_as_uint(x == 0.f ? 0.f : x);   // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exclusive prefix count of `flag` over the workgroup (256 threads) and the total.
__device__ inline int block_excl_count(bool flag, int* s_wave, int& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t bal = __ballot(flag);
    const int within = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    return before + within;
}

// In-place bitonic sort of N (a power of two) LDS elements by 256 threads, descending or ascending.
template <class T, int N, bool DESC>
__device__ inline void bitonic_sort(T* v)
{
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < N / 2; t += 256) {
                const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));   // stride is a power of two
                const int j = i + stride;
                const bool first_up = ((i & size) == 0) == DESC;   // this block ends in the final order
                const T x = v[i], y = v[j];
                if (first_up ? (x < y) : (x > y)) { v[i] = y; v[j] = x; }
            }
            __syncthreads();
        }
    }
}

constexpr int TOPK_CAP = 2048;   // candidates per row in LDS, a quarter per wave

__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ S, int64_t lds, int L, int k,
                                                   int* __restrict__ out, int64_t ldo)
{
    __shared__ uint32_t s_t[512];
    __shared__ uint64_t s_c[TOPK_CAP];
    __shared__ int s_sel[256];
    __shared__ int s_over;
    __shared__ int hist[256];
    __shared__ int s_digit, s_need;
    __shared__ int s_wave[4];
    const int row = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float* s = S + (int64_t)row * lds;
    int* o = out + (int64_t)row * ldo;
    const int kk = k < L ? k : L;

    // 1. per-thread two largest keys, then their kk-th largest over the workgroup.  A thread's eight loads
    //    are unconditional whenever every thread's lie inside the row (a guarded load compiles to a branch
    //    that waits for its data, so the loads would run one after another).
    uint32_t t1 = 0u, t2 = 0u;
    for (int j0 = tid; j0 < L; j0 += 256 * 8) {
        uint32_t key[8];
        if (j0 - tid + 256 * 8 <= L) {
#pragma unroll
            for (int e = 0; e < 8; ++e) key[e] = order_key(s[j0 + 256 * e]);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = j0 + 256 * e;
                key[e] = j < L ? order_key(s[j]) : 0u;
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t u = key[e];
            if (u > t1) { t2 = t1; t1 = u; } else if (u > t2) { t2 = u; }
        }
    }
    s_t[2 * tid] = t1;
    s_t[2 * tid + 1] = t2;
    if (tid == 0) s_over = 0;
    __syncthreads();
    bitonic_sort<uint32_t, 512, true>(s_t);
    const uint32_t T = kk > 0 ? s_t[kk - 1] : 0xFFFFFFFFu;

    // 2. per-wave ordered compaction of the keys >= T over the wave's quarter of the row
    constexpr int CW = TOPK_CAP / 4;
    const int q4 = (L + 3) / 4;
    const int lo = wave * q4, hi = lo + q4 < L ? lo + q4 : L;
    int cnt = 0;
    uint64_t* mine = s_c + wave * CW;
    for (int b0 = lo; b0 < hi; b0 += 64 * 4) {
        uint32_t key[4];
        if (b0 + 64 * 4 <= hi) {   // the whole step inside the quarter (the same for the whole wave)
#pragma unroll
            for (int e = 0; e < 4; ++e) key[e] = order_key(s[b0 + 64 * e + lane]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = b0 + 64 * e + lane;
                key[e] = j < hi ? order_key(s[j]) : 0u;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = b0 + 64 * e + lane;
            const bool take = j < hi && key[e] >= T && kk > 0;
            const uint64_t bal = __ballot(take);
            const int pos = cnt + __popcll(bal & ((1ull << lane) - 1ull));
            if (take && pos < CW) mine[pos] = ((uint64_t)key[e] << 32) | (uint64_t)(~(uint32_t)j);
            cnt += __popcll(bal);
        }
    }
    if (cnt > CW && lane == 0) s_over = 1;
    for (int q = cnt + lane; q < CW; q += 64) mine[q] = 0ull;   // below every real (key, index) pair
    __syncthreads();

    if (!s_over) {
        // 3. gather the four quarters' candidates to the front (through registers: the moves overlap),
        //    order them, take the first kk, list their indices ascending
        if (lane == 0) s_wave[wave] = cnt;
        __syncthreads();
        const int off = (wave > 0 ? s_wave[0] : 0) + (wave > 1 ? s_wave[1] : 0) + (wave > 2 ? s_wave[2] : 0);
        const int c = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        uint64_t mv[CW / 64];
#pragma unroll
        for (int q = 0; q < CW / 64; ++q) mv[q] = mine[lane + 64 * q];
        __syncthreads();
        int N = 256;
        while (N < c) N <<= 1;
#pragma unroll
        for (int q = 0; q < CW / 64; ++q) {
            const int e = lane + 64 * q;
            if (e < cnt) s_c[off + e] = mv[q];
        }
        for (int e = c + tid; e < N; e += 256) s_c[e] = 0ull;
        __syncthreads();
        if (N == 256) bitonic_sort<uint64_t, 256, true>(s_c);
        else if (N == 512) bitonic_sort<uint64_t, 512, true>(s_c);
        else if (N == 1024) bitonic_sort<uint64_t, 1024, true>(s_c);
        else bitonic_sort<uint64_t, TOPK_CAP, true>(s_c);
        s_sel[tid] = tid < kk ? (int)(~(uint32_t)(s_c[tid] & 0xFFFFFFFFull)) : 0x7FFFFFFF;
        __syncthreads();
        bitonic_sort<int, 256, false>(s_sel);
        if (tid < k) o[tid] = tid < kk ? s_sel[tid] : -1;
        return;
    }

    // Fallback: exact radix select over the keys in global memory.  Four 8-bit passes find the
    // kk-th largest key P and how many keys equal to P to take; a final pass compacts in index order.
    uint32_t prefix = 0u, mask = 0u;
    int need = kk;
    if (need > 0) {
        for (int shift = 24; shift >= 0; shift -= 8) {
            hist[tid] = 0;
            __syncthreads();
            for (int j = tid; j < L; j += 256) {
                const uint32_t u = order_key(s[j]);
                if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int above = 0, d = 255;
                for (; d > 0; --d) {
                    if (above + hist[d] >= need) break;
                    above += hist[d];
                }
                s_digit = d;
                s_need = need - above;
            }
            __syncthreads();
            prefix |= (uint32_t)s_digit << shift;
            mask |= 0xFFu << shift;
            need = s_need;
            __syncthreads();
        }
    }
    // keys > prefix are all taken; `need` keys equal to prefix, the lowest indices first
    int base_out = 0, base_tie = 0;
    for (int c0 = 0; c0 < L && kk > 0; c0 += 256) {
        const int j = c0 + tid;
        const uint32_t u = j < L ? order_key(s[j]) : 0u;
        const bool gt = j < L && u > prefix;
        const bool eq = j < L && u == prefix;
        int tot_eq, tot_sel;
        const int tie_rank = base_tie + block_excl_count(eq, s_wave, tot_eq);
        const bool sel = gt || (eq && tie_rank < need);
        const int pos = base_out + block_excl_count(sel, s_wave, tot_sel);
        if (sel) o[pos] = j;
        base_tie += tot_eq;
        base_out += tot_sel;
    }
    for (int q = base_out + tid; q < k; q += 256) o[q] = -1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t mlp_project(const float* At, int64_t lda, int n, int m, const float* P, int d, uint16_t* APt, int npad,
                       hipStream_t s)
{
    dim3 grid((npad + 63) / 64, (d + 63) / 64);
    hipLaunchKernelGGL(project_kernel, grid, dim3(256), 0, s, At, lda, n, m, P, d, APt, npad);
    return hipGetLastError();
}

hipError_t mlp_signals_bf16(const float* B, int64_t ldb, int n, int p, uint16_t* B16, int npad, hipStream_t s)
{
    if (p <= 0) return hipSuccess;
    hipLaunchKernelGGL(signals_bf16_kernel, dim3(p), dim3(256), 0, s, B, ldb, n, B16, npad);
    return hipGetLastError();
}

hipError_t mlp_gemm_store(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                          float* C, int64_t ldc, const float* bias, hipStream_t s)
{
    return launch_gemm(X, ldx, M, W, ldw, N, kpad, EpiStore{C, ldc, bias}, s);
}

hipError_t mlp_gemm_bias_gelu(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                              const float* bias, float* U, int64_t ldu, uint16_t* H, int64_t ldh, hipStream_t s)
{
    return launch_gemm(X, ldx, M, W, ldw, N, kpad, EpiBiasGelu{bias, U, ldu, H, ldh}, s);
}

hipError_t mlp_gemm_gelu_back(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                              const float* U, int64_t ldu, float* D, int64_t ldd, uint16_t* D16, int64_t ld16,
                              hipStream_t s)
{
    return launch_gemm(X, ldx, M, W, ldw, N, kpad, EpiGeluBack{U, ldu, D, ldd, D16, ld16}, s);
}

hipError_t mlp_embed_norm(const float* Z, int d, int p, uint16_t* X0, float* Zout, int64_t ldz_out, hipStream_t s)
{
    if (p <= 0) return hipSuccess;
    hipLaunchKernelGGL(embed_norm_kernel, dim3(p), dim3(256), 0, s, Z, d, X0, Zout, ldz_out);
    return hipGetLastError();
}

hipError_t mlp_bce_grad(float* S, int64_t lds, uint16_t* D16, int64_t ld16, int m, int mpad, int rows,
                        const int* supp, int64_t ld_supp, const int* supp_len, float pos_w, float* rowloss,
                        double* loss, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if ((m + 31) / 32 > BCE_MAX_WORDS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bce_grad_kernel, dim3(rows), dim3(256), 0, s, S, lds, D16, ld16, m, mpad, supp, ld_supp,
                       supp_len, pos_w, 1.0f / rows, rowloss);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, rowloss, rows, loss);
    return hipGetLastError();
}

hipError_t mlp_colsum(const float* in, int64_t ld, int rows, int cols, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, in, ld, rows, cols, out);
    return hipGetLastError();
}

hipError_t mlp_transpose(const uint16_t* in, int64_t ldi, int rows, int cols, uint16_t* out, int64_t ldo,
                         hipStream_t s)
{
    if (ldo % 64 || ldo < rows) return hipErrorInvalidValue;
    dim3 grid((unsigned)(ldo / 64), (cols + 63) / 64);
    hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(256), 0, s, in, ldi, rows, cols, out, ldo);
    return hipGetLastError();
}

hipError_t mlp_adam(float* P, float* m1, float* m2, const float* g, uint16_t* P16, int64_t count, float lr,
                    float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, m1, m2, g, P16, count, lr, beta1,
                       beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t mlp_params_bf16(const float* P, uint16_t* P16, int64_t count, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(params_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, P16, count);
    return hipGetLastError();
}

hipError_t mlp_topk(const float* S, int64_t lds, int rows, int L, int k, int* out, int64_t ldo, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (k < 1 || k > 256 || L < 1 || ldo < k) return hipErrorInvalidValue;
    if ((size_t)L * 4 > TOPK_MAX_LDS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(topk_kernel, dim3(rows), dim3(256), 0, s, S, lds, L, k, out, ldo);
    return hipGetLastError();
}

}  // namespace bmpl
