// Reduced-precision screening of the worst-case analysis (Algorithm 1, step 3).
//
// With a bfloat16 correlation product g~ = bf16(A)^T bf16(xi) (float32
// accumulation) every entry is within a certified band of the float32 value.
// With a^ = bf16(a_j), da = a^ - a_j, x^ = bf16(xi), dx = x^ - xi, the products
// a^_k x^_k are exact in float32 and
//     a^ . x^ - a_j . xi = a^ . dx + da . xi             (exactly),
// so by Cauchy-Schwarz, with the float32 accumulation's n 2^-24 sum |a^_k x^_k|,
//     |g~_j - g_j| <= ||a^|| ||dx|| + ||da|| ||xi|| + n 2^-24 ||a^|| (||xi|| + ||dx||)
//                  <= eps_i = band_x ||xi_i|| + band_dx ||dx_i||
// with the maxima of ||a^|| and ||da|| over the atoms (set up once) and ||dx_i||
// measured where the residual is rounded.  Rounding errors of random data are
// about a third of their worst case, so this is two to three times narrower than
// the worst-case 2^-7 max_j ||a_j|| ||xi_i||.  The screen keeps every atom whose band
// could reach the selection threshold, the candidates are re-scored exactly
// (float32 data, float64 accumulation), and only re-scored values decide which
// atoms enter I and whether the natural stopping condition Eq. (9) holds.  So
// the selected atoms are exactly the float32 top-rho violators and the stop is
// certified, as with the float32 product.
//
// Candidate rule for signal i (atoms outside I, L_j = |g~_j| - eps, U_j = |g~_j| + eps):
//   tau = rho-th largest L_j (or -inf), thr = max(lambda, tau);  C = { j : U_j > thr }.
// Every true top-rho violator lies in C (its |g_j| is at least tau and above lambda), and
// when tau <= lambda every possible violator does.  For the relative lambda rule on the
// first pass, lambda is replaced by the lower bound c (max|g~| - eps) and C also holds every
// atom that may attain max_j |g_j| (U_j >= max|g~| - eps), so the exact maximum sets lambda.
#include <float.h>
#include <limits.h>
#include <stdint.h>

#include "../../include/bmpl.h"
#include "bmpl_internal.h"
#include "wave_ops.h"

namespace bmpl {
namespace {

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ src, int64_t lds,
                                                      uint16_t* __restrict__ dst, int64_t ldd, int rows, int cols)
{
    const int r = blockIdx.x;
    if (r >= rows) return;
    for (int c = threadIdx.x; c < cols; c += 256) dst[(int64_t)r * ldd + c] = bf16_round(src[(int64_t)r * lds + c]);
}

// ||a_j||, ||bf16(a_j)|| and ||bf16(a_j) - a_j|| into norms[j], norms[m + j], norms[2m + j], rounded up.
__global__ __launch_bounds__(256) void atom_norm_kernel(const float* __restrict__ At, int64_t lda, int n,
                                                        float* __restrict__ norms, int m)
{
    __shared__ double red[3][4];
    const int j = blockIdx.x;
    if (j >= m) return;
    double s = 0.0, sh = 0.0, sd = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const float f = At[(int64_t)j * lda + k];
        const float h = bf16_value(bf16_round(f));
        const double v = f, vh = h, d = (double)h - (double)f;
        s += v * v;
        sh += vh * vh;
        sd += d * d;
    }
    s = wave_sum(s);
    sh = wave_sum(sh);
    sd = wave_sum(sd);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = sh;
        red[2][threadIdx.x >> 6] = sd;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double* r = red[threadIdx.x];
        norms[(int64_t)threadIdx.x * m + j] = (float)sqrt(r[0] + r[1] + r[2] + r[3]) * (1.0f + 1e-6f);
    }
}

// x . y over n4 float4 (float32 data, float64 accumulation) by one wave; every lane gets the sum.
// Six 16-byte loads of x per lane are in flight before the first is used (eight would cost the
// re-score kernel a quarter of its workgroups per CU).
__device__ inline double wave_dot_f64(const float4* __restrict__ x, const float4* __restrict__ y, int n4, int lane)
{
    constexpr int CH = 8;   // eight float4 per lane in flight (n = 2048: one step), four workgroups per CU
    double acc = 0.0;
    for (int q0 = lane; q0 < n4; q0 += 64 * CH) {
        float4 fx[CH];
        if (q0 - lane + 64 * CH <= n4) {   // the whole step inside the vectors (the same for the whole wave):
#pragma unroll                             // no branch, so the loads are all in flight at once
            for (int e = 0; e < CH; ++e) fx[e] = x[q0 + 64 * e];
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const float4 fy = y[q0 + 64 * e];
                acc += (double)fx[e].x * fy.x + (double)fx[e].y * fy.y + (double)fx[e].z * fy.z +
                       (double)fx[e].w * fy.w;
            }
            continue;
        }
        // the tail: clamped indices, so these loads too are issued together (a guarded load compiles to
        // a branch whose end waits for it); chunks past the end count zero
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = q0 + 64 * e;
            fx[e] = x[q < n4 ? q : n4 - 1];
        }
#pragma unroll
        for (int e = 0; e < CH; ++e) {    // y is read as the sums need it (LDS in the re-score)
            const int q = q0 + 64 * e;
            const float4 fy = y[q < n4 ? q : n4 - 1];
            const double d = (double)fx[e].x * fy.x + (double)fx[e].y * fy.y + (double)fx[e].z * fy.z +
                             (double)fx[e].w * fy.w;
            acc += q < n4 ? d : 0.0;
        }
    }
    return wave_sum(acc);
}

// The candidate rule by sweeps over the row (used when many equal values overflow the candidate buffer
// of screen_select_kernel): the thread maxima, then per-thread lists of the entries at or above their
// k-th largest, then the candidates.
template <int KMAX>
__device__ void screen_sweeps(const ScreenArgs& a, int row, int sig, int k, float eps)
{
    __shared__ float s_top[4][KMAX];
    __shared__ float s_red[8];
    __shared__ int s_cnt;
    const float* g = a.G + (int64_t)row * a.ldg;
    const uint32_t* ex = a.excl ? a.excl + (int64_t)sig * a.words : nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Pass 1: the k largest |g~| outside I (values only) and the largest |g~| overall, in two sweeps:
    // each thread's maximum first (the k-th largest of the 256 thread maxima bounds the k-th largest
    // entry from below), then per-thread sorted lists of only the entries at or above that bound.
    const bool vec4 = ((a.ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.G) & 15) == 0);
    const int m4 = vec4 ? (a.m & ~3) : 0;
    // visit(|g~_j|, outside I) for every atom, in increasing j per thread
    auto scan = [&](auto&& visit) {
        constexpr int CH = 8;   // loads per thread issued before the first is used
        for (int base = 4 * tid; base < m4; base += 1024 * CH) {
            float4 f[CH];
            uint32_t word[CH];
            row_chunks<CH>(g, ex, base - 4 * tid, m4, 0u, f, word);   // 4 atoms share one word
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                if (base + 1024 * q >= m4) break;
                visit(fabsf(f[q].x), !(word[q] & 1u));
                visit(fabsf(f[q].y), !(word[q] & 2u));
                visit(fabsf(f[q].z), !(word[q] & 4u));
                visit(fabsf(f[q].w), !(word[q] & 8u));
            }
        }
        for (int j = m4 + tid; j < a.m; j += 256)
            visit(fabsf(g[j]), !(ex && ((ex[j >> 5] >> (j & 31)) & 1u)));
    };
    float gall = 0.f, tmax = -1.f;
    scan([&](float v, bool out) {
        gall = fmaxf(gall, v);
        if (out) tmax = fmaxf(tmax, v);
    });
    {
        float cur = tmax;
        for (int r = 0; r < k; ++r) {
            const float b = wave_max(cur);
            if (lane == 0) s_top[wave][r] = b;
            const unsigned long long owners = __ballot(cur == b);
            if (lane == __ffsll((long long)owners) - 1) cur = -2.f;   // pop one holder
        }
    }
    __syncthreads();
    if (tid == 0) {
        float T = INFINITY;
        int p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        for (int r = 0; r < k; ++r) {
            const float v0 = p0 < k ? s_top[0][p0] : -3.f, v1 = p1 < k ? s_top[1][p1] : -3.f;
            const float v2 = p2 < k ? s_top[2][p2] : -3.f, v3 = p3 < k ? s_top[3][p3] : -3.f;
            const float b = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
            T = b;
            if (b == v0) ++p0; else if (b == v1) ++p1; else if (b == v2) ++p2; else ++p3;
        }
        s_red[4] = T;
    }
    __syncthreads();
    const float T = s_red[4];
    __syncthreads();
    float top[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) top[q] = -1.f;
    auto consider = [&](float v, bool out) {
        if (!out || !(v >= T) || !(v > top[KMAX - 1])) return;
        float cv = v;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            const bool sw = cv > top[q];
            const float t = top[q];
            top[q] = sw ? cv : t;
            cv = sw ? t : cv;
        }
    };
    if (T <= FLT_MAX) scan(consider);
    gall = wave_max(gall);
    // wave merge of the per-thread lists: k rounds of a wave max on the heads
    for (int r = 0; r < k; ++r) {
        const float b = wave_max(top[0]);
        if (lane == 0) s_top[wave][r] = b;
        // the first lane holding the head value pops it
        const unsigned long long owners = __ballot(top[0] == b);
        if (owners && lane == __ffsll((long long)owners) - 1) {
#pragma unroll
            for (int q = 0; q < KMAX - 1; ++q) top[q] = top[q + 1];
            top[KMAX - 1] = -1.f;
        }
    }
    if (lane == 0) s_red[wave] = gall;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    // k-th largest over the four wave lists
    float kth = -1.f;
    if (k > 0) {
        int p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        for (int r = 0; r < k; ++r) {
            const float v0 = p0 < k ? s_top[0][p0] : -1.f, v1 = p1 < k ? s_top[1][p1] : -1.f;
            const float v2 = p2 < k ? s_top[2][p2] : -1.f, v3 = p3 < k ? s_top[3][p3] : -1.f;
            const float b = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
            kth = b;
            if (b == v0) ++p0; else if (b == v1) ++p1; else if (b == v2) ++p2; else ++p3;
        }
    }
    const float gmax = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
    const double lam_lo = a.lam_rel > 0.0 ? a.lam_rel * ((double)gmax - eps) : a.lam[sig];
    const double tau = kth >= 0.f ? (double)kth - eps : -1.0;
    const double thr = lam_lo > tau ? lam_lo : tau;
    const double thr_max = a.lam_rel > 0.0 ? (double)gmax - eps : DBL_MAX;   // U_j >= this: may attain the max

    // Pass 2: collect the candidates.
    int* cand = a.cand + (int64_t)sig * a.candcap;
    constexpr int CH = 8;   // loads per thread issued before the first is used
    for (int b0 = 0; b0 < a.m; b0 += 256 * CH) {
        float v[CH];
        uint32_t word[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int j = b0 + 256 * q + tid;
            const bool in = j < a.m;
            v[q] = in ? fabsf(g[j]) : 0.f;
            word[q] = (ex && in) ? ex[j >> 5] : 0u;
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int j = b0 + 256 * q + tid;
            bool take = false;
            if (j < a.m && !((word[q] >> (j & 31)) & 1u)) {
                const double u = (double)v[q] + eps;
                take = (u > thr) || (u >= thr_max);
            }
            const unsigned long long bal = __ballot(take);
            int base = 0;
            if (lane == 0 && bal) base = atomicAdd(&s_cnt, __popcll(bal));
            base = __shfl(base, 0);
            if (take) {
                const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
                if (pos < a.candcap) cand[pos] = j;
            }
        }
    }
    __syncthreads();
    if (tid == 0) a.ncand[sig] = s_cnt;
}

// Candidates of one signal from a single read of its row.  Each thread's first eight float4 stay in
// registers; the k-th largest T of the threads' maxima over them (outside I) bounds the k-th largest
// |g~| outside I from below, so tau = that value - eps >= T - eps, and every candidate (U_j > thr >= tau,
// or U_j >= max|g~| - eps >= T - eps) has |g~_j| + eps >= T - eps; with a fixed lambda it also has
// |g~_j| + eps > lambda.  The entries that pass these tests (computed in the same double arithmetic as the
// rule itself) are appended to an LDS buffer as the row streams in.  The buffer holds every entry at or
// above the k-th largest whenever it holds k entries, so the k-th largest, tau and thr follow from it, and
// the candidates are the buffered entries that pass the rule.  When it holds fewer than k (fixed lambda),
// the k-th largest has U <= lambda, so tau <= lambda = thr.  A buffer overflow falls back to the sweeps.
template <int KMAX>
__global__ __launch_bounds__(256) void screen_select_kernel(ScreenArgs a)
{
    constexpr int CH = 8;       // float4 per thread held in registers
    constexpr int CAP = 2048;   // buffered entries
    __shared__ float s_cv[CAP];
    __shared__ int s_ci[CAP];
    __shared__ float s_tw[4 * KMAX];
    __shared__ float s_r[4];
    __shared__ float s_T, s_kth;
    __shared__ int s_n, s_cnt;
    if (a.clear_count && blockIdx.x == 0 && threadIdx.x == 0) *a.clear_count = 0;   // the re-score's spill list
    const int n_act = a.n_act_dev ? *a.n_act_dev : a.p_grid;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act ? a.act[row] : row;
    const float* g = a.G + (int64_t)row * a.ldg;
    const uint32_t* ex = a.excl ? a.excl + (int64_t)sig * a.words : nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float eps = (float)(a.band_x * a.rnorm[sig] + a.band_dx * a.dxnorm[sig]);

    int k = a.k;
    if (a.nI && a.max_active > 0) {
        const int room = a.max_active - a.nI[sig];
        k = room < k ? (room > 0 ? room : 0) : k;
    }
    const bool rel = a.lam_rel > 0.0;
    const bool vec4 = ((a.ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.G) & 15) == 0);
    const int m4 = vec4 ? (a.m & ~3) : 0;

    float4 f0[CH];
    uint32_t w0[CH];     // bit set: in I or past the row
    row_chunks<CH>(g, ex, 0, m4, 0xFu, f0, w0);
    // The rest of the row streams in chunks of CS float4 per thread, each chunk's loads issued one chunk
    // ahead (the first before the bound is computed), so a workgroup waits for memory about once.
    constexpr int CS = 4;
    float4 fa[CS];
    uint32_t wa[CS];
    auto load_chunk = [&](int base0, float4 (&f)[CS], uint32_t (&word)[CS]) {
        row_chunks<CS>(g, ex, base0, m4, 0xFu, f, word);
    };
    load_chunk(1024 * CH, fa, wa);
    float gall = 0.f, tmax = -1.f;   // largest |g~| over every atom; over the registered atoms outside I
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        gall = fmaxf(gall, fmaxf(fmaxf(fabsf(f0[q].x), fabsf(f0[q].y)), fmaxf(fabsf(f0[q].z), fabsf(f0[q].w))));
        if (!(w0[q] & 1u)) tmax = fmaxf(tmax, fabsf(f0[q].x));
        if (!(w0[q] & 2u)) tmax = fmaxf(tmax, fabsf(f0[q].y));
        if (!(w0[q] & 4u)) tmax = fmaxf(tmax, fabsf(f0[q].z));
        if (!(w0[q] & 8u)) tmax = fmaxf(tmax, fabsf(f0[q].w));
    }
    {
        float cur = tmax;
        for (int r = 0; r < k; ++r) {
            const float b = wave_max(cur);
            if (lane == 0) s_tw[wave * KMAX + r] = b;
            const unsigned long long owners = __ballot(cur == b);
            if (lane == __ffsll((long long)owners) - 1) cur = -2.f;   // pop one holder
        }
    }
    if (tid == 0) { s_n = 0; s_T = INFINITY; }
    __syncthreads();
    if (tid < 4 * k) {   // T = the k-th largest of the 4k listed maxima (equal values write the same T)
        const int tw = tid / k;
        const float v = s_tw[tw * KMAX + (tid - tw * k)];
        int gt = 0, ge = 0;
        for (int w2 = 0; w2 < 4; ++w2)
            for (int r = 0; r < k; ++r) {
                const float w = s_tw[w2 * KMAX + r];
                gt += w > v;
                ge += w >= v;
            }
        if (gt < k && ge >= k) s_T = v;
    }
    __syncthreads();
    // admission test on u = |g~| + eps: u >= T - eps (k > 0), and u > lambda for a fixed lambda
    const double pre = k > 0 ? (double)s_T - eps : -DBL_MAX;
    const double lam_fix = rel ? -DBL_MAX : a.lam[sig];
    auto ok = [&](float v) {
        const double u = (double)v + eps;
        return u >= pre && u > lam_fix;
    };
    auto take = [&](bool t, int j, float v) {   // called by the whole wave
        const unsigned long long bal = __ballot(t);
        if (!bal) return;
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_n, __popcll(bal));
        base = __shfl(base, 0);
        const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
        if (t && pos < CAP) { s_cv[pos] = v; s_ci[pos] = j; }
    };
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int j0 = 4 * tid + 1024 * q;
        take(!(w0[q] & 1u) && ok(fabsf(f0[q].x)), j0, fabsf(f0[q].x));
        take(!(w0[q] & 2u) && ok(fabsf(f0[q].y)), j0 + 1, fabsf(f0[q].y));
        take(!(w0[q] & 4u) && ok(fabsf(f0[q].z)), j0 + 2, fabsf(f0[q].z));
        take(!(w0[q] & 8u) && ok(fabsf(f0[q].w)), j0 + 3, fabsf(f0[q].w));
    }
    for (int base0 = 1024 * CH; base0 < m4; base0 += 1024 * CS) {   // the same trip count in every lane
        const int base = base0 + 4 * tid;
        float4 fb[CS];
        uint32_t wb[CS];
        load_chunk(base0 + 1024 * CS, fb, wb);   // the next chunk (past the row: zeros, no load)
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const int j0 = base + 1024 * q;
            const float v0 = fabsf(fa[q].x), v1 = fabsf(fa[q].y), v2 = fabsf(fa[q].z), v3 = fabsf(fa[q].w);
            gall = fmaxf(gall, fmaxf(fmaxf(v0, v1), fmaxf(v2, v3)));
            take(!(wa[q] & 1u) && ok(v0), j0, v0);
            take(!(wa[q] & 2u) && ok(v1), j0 + 1, v1);
            take(!(wa[q] & 4u) && ok(v2), j0 + 2, v2);
            take(!(wa[q] & 8u) && ok(v3), j0 + 3, v3);
        }
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            fa[q] = fb[q];
            wa[q] = wb[q];
        }
    }
    for (int j0 = m4; j0 < a.m; j0 += 256) {
        const int j = j0 + tid;
        const bool in = j < a.m;
        const float v = in ? fabsf(g[j]) : 0.f;
        gall = fmaxf(gall, v);
        const bool out = in && !(ex && ((ex[j >> 5] >> (j & 31)) & 1u));
        take(out && ok(v), j, v);
    }
    gall = wave_max(gall);
    if (lane == 0) s_r[wave] = gall;
    if (tid == 0) { s_cnt = 0; s_kth = -1.f; }
    __syncthreads();
    const int nc = s_n;
    if (nc > CAP) {
        screen_sweeps<KMAX>(a, row, sig, k, eps);
        return;
    }
    const float gmax = fmaxf(fmaxf(s_r[0], s_r[1]), fmaxf(s_r[2], s_r[3]));
    if (k > 0 && nc >= k) {
        if (nc <= 2 * 256) {
            // k-th largest buffered value: the entry with fewer than k larger values and at least k at or above
            for (int e = tid; e < nc; e += 256) {
                const float v = s_cv[e];
                int gt = 0, ge = 0;
                for (int d = 0; d < nc; ++d) {
                    const float w = s_cv[d];
                    gt += w > v;
                    ge += w >= v;
                }
                if (gt < k && ge >= k) s_kth = v;   // every writer stores the same value
            }
        } else {
            int N = 64;
            while (N < nc) N <<= 1;
            for (int e = nc + tid; e < N; e += 256) { s_cv[e] = -1.f; s_ci[e] = -1; }
            __syncthreads();
            for (int size = 2; size <= N; size <<= 1)       // descending by value (the indices ride along)
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    for (int t = tid; t < N / 2; t += 256) {
                        const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1)), j = i + stride;
                        const float vi = s_cv[i], vj = s_cv[j];
                        if (((i & size) == 0) ? (vi < vj) : (vi > vj)) {
                            const int ii = s_ci[i];
                            s_cv[i] = vj; s_cv[j] = vi;
                            s_ci[i] = s_ci[j]; s_ci[j] = ii;
                        }
                    }
                    __syncthreads();
                }
            if (tid == 0) s_kth = s_cv[k - 1];
        }
    }
    __syncthreads();
    const float kth = s_kth;
    const double lam_lo = rel ? a.lam_rel * ((double)gmax - eps) : a.lam[sig];
    const double tau = kth >= 0.f ? (double)kth - eps : -1.0;
    const double thr = lam_lo > tau ? lam_lo : tau;
    const double thr_max = rel ? (double)gmax - eps : DBL_MAX;   // U_j >= this: may attain the max
    int* cand = a.cand + (int64_t)sig * a.candcap;
    for (int e0 = 0; e0 < nc; e0 += 256) {
        const int e = e0 + tid;
        bool t = false;
        if (e < nc) {
            const double u = (double)s_cv[e] + eps;
            t = (u > thr) || (u >= thr_max);
        }
        const unsigned long long bal = __ballot(t);
        int base = 0;
        if (lane == 0 && bal) base = atomicAdd(&s_cnt, __popcll(bal));
        base = __shfl(base, 0);
        if (t) {
            const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
            if (pos < a.candcap) cand[pos] = s_ci[e];
        }
    }
    __syncthreads();
    if (tid == 0) a.ncand[sig] = s_cnt;
}

// Exact re-score of the candidates (float32 data, float64 accumulation), then the
// selection itself.  Scored in two stages: first the k candidates with the largest
// |g~| (their k-th exact value v_k bounds the true k-th largest from below), then only
// the candidates whose band still reaches max(lambda, v_k); the rest cannot enter the
// top k nor violate.  The residual is staged in LDS once per signal.
__global__ __launch_bounds__(256) void rescore_kernel(RescoreArgs a)
{
    extern __shared__ __align__(16) double s_dyn[];
    __shared__ double red[8];
    __shared__ int s_lim;
    const int n_act = a.n_act_dev ? *a.n_act_dev : a.p_grid;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act ? a.act[row] : row;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nc_all = a.ncand[sig];
    if (a.spill_row) {   // first of two passes: more candidates than this pass's LDS holds are left over
        const bool over_lds = nc_all > a.candcap_lds && nc_all <= a.candcap;
        if (tid == 0) {
            a.spill_row[sig] = over_lds ? row + 1 : 0;
            if (over_lds) a.spill_act[atomicAdd(a.n_spill, 1)] = sig;
        }
        if (over_lds) return;
    }
    const bool overflow = nc_all > a.candcap || nc_all > a.candcap_lds;
    const int nc = overflow ? 0 : nc_all;
    const int* cand = a.cand + (int64_t)sig * a.candcap;
    const float* r = a.R + (int64_t)sig * a.ldr;
    const float* gt = a.G + (int64_t)(a.row_of ? a.row_of[sig] - 1 : row) * a.ldg;
    double* s_val = s_dyn;                                       // [candcap_lds] exact |g|, -1 = unscored
    float* s_gt = reinterpret_cast<float*>(s_dyn + a.candcap_lds);   // [candcap_lds] |g~|
    float* s_r = s_gt + a.candcap_lds;                           // [kpad] residual
    const double eps = a.band_x * a.rnorm[sig] + a.band_dx * a.dxnorm[sig];

    int k = a.k;
    if (a.nI && a.max_active > 0) {
        const int room = a.max_active - a.nI[sig];
        k = room < k ? (room > 0 ? room : 0) : k;
    }
    if ((a.kpad & 3) == 0 && (a.ldr & 3) == 0 && (reinterpret_cast<uintptr_t>(a.R) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(s_r) & 15) == 0) {
        // the residual in two batches of float4 loads per thread at most (n <= 2048: one round trip)
        const float4* r4 = reinterpret_cast<const float4*>(r);
        float4* s_r4 = reinterpret_cast<float4*>(s_r);
        const int n4 = a.kpad / 4;
        for (int q0 = tid; q0 < n4; q0 += 2 * 256) {
            const float4 v0 = r4[q0];
            const float4 v1 = q0 + 256 < n4 ? r4[q0 + 256] : make_float4(0.f, 0.f, 0.f, 0.f);
            s_r4[q0] = v0;
            if (q0 + 256 < n4) s_r4[q0 + 256] = v1;
        }
    } else {
        for (int q = tid; q < a.kpad; q += 256) s_r[q] = r[q];
    }
    for (int c = tid; c < nc; c += 256) {
        s_val[c] = -1.0;
        s_gt[c] = fabsf(gt[cand[c]]);
    }
    __syncthreads();
    auto score = [&](int c) {     // by one wave; returns in every lane
        const float4* aj = reinterpret_cast<const float4*>(a.At + (int64_t)cand[c] * a.lda);
        return fabs(wave_dot_f64(aj, reinterpret_cast<const float4*>(s_r), a.kpad / 4, lane));
    };
    // Stage 1: the candidates ranked among the first k by |g~| (ties to the lower atom).
    for (int c = wave; c < nc; c += 4) {
        const float v = s_gt[c];
        const int j = cand[c];
        int rank = 0;
        for (int d = lane; d < nc; d += 64) {
            const float w = s_gt[d];
            rank += (w > v || (w == v && cand[d] < j)) ? 1 : 0;
        }
        rank = wave_sum(rank);
        if (rank < (k > 0 ? k : 1)) {
            const double e = score(c);
            if (lane == 0) s_val[c] = e;
        }
    }
    __syncthreads();
    // v_k (k-th largest exact value so far) and the largest exact value so far.
    if (tid == 0) { red[0] = -1.0; red[1] = 0.0; }
    __syncthreads();
    double e1 = 0.0;
    for (int c = tid; c < nc; c += 256) {
        const double v = s_val[c];
        if (v < 0.0) continue;
        e1 = fmax(e1, v);
        int gt = 0, ge = 0;
        for (int d = 0; d < nc; ++d) {
            const double w = s_val[d];
            gt += w > v;
            ge += w >= v;
        }
        if (k > 0 && gt < k && ge >= k) red[0] = v;   // every writer stores the same value
    }
    e1 = wave_max(e1);
    __syncthreads();
    if (lane == 0) red[2 + wave] = e1;   // red[0] = v_k, red[2..5] = per-wave maxima
    __syncthreads();
    const double vk = red[0];
    e1 = fmax(fmax(red[2], red[3]), fmax(red[4], red[5]));
    __syncthreads();
    const bool rel = a.lam_rel > 0.0;
    const double lam_lo = rel ? a.lam_rel * e1 : a.lam[sig];    // lambda >= this (the max is >= e1)
    const double thr = lam_lo > vk ? lam_lo : vk;
    // Stage 2: every remaining candidate whose band reaches thr (or, for the relative rule, the max).
    for (int c = wave; c < nc; c += 4) {
        if (s_val[c] >= 0.0) continue;
        const double u = (double)s_gt[c] + eps;
        if (!(u > thr) && !(rel && u >= e1)) continue;
        const double e = score(c);
        if (lane == 0) s_val[c] = e;
    }
    __syncthreads();
    double mx = 0.0;
    for (int c = tid; c < nc; c += 256) mx = fmax(mx, s_val[c]);
    mx = wave_max(mx);
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    double lam = a.lam[sig];
    if (rel) {
        lam = a.lam_rel * mx;
        if (tid == 0) a.lam[sig] = lam;
    }
    __syncthreads();
    // rank the violators: larger |g| first, ties to the lower atom index
    int cnt = 0;
    for (int c = tid; c < nc; c += 256) {
        const double v = s_val[c];
        if (!(v > lam)) continue;
        const int j = cand[c];
        int rank = 0;
        for (int d = 0; d < nc; ++d) {
            const double w = s_val[d];
            if (w > lam && (w > v || (w == v && cand[d] < j))) ++rank;
        }
        if (rank < k) a.sel[(int64_t)sig * a.selcap + rank] = j;
        ++cnt;
    }
    cnt = wave_sum(cnt);
    if (lane == 0) red[wave] = (double)cnt;
    __syncthreads();
    if (tid == 0) {
        int nv = (int)(red[0] + red[1] + red[2] + red[3]);
        nv = nv < k ? nv : k;
        a.nsel[sig] = nv;
        float vm = (float)mx;
        if (nv == 0 && (double)vm > lam) vm = nextafterf(vm, 0.f);   // keep the float copy <= lambda
        a.vmax[sig] = vm;
        if (overflow) {
            a.nsel[sig] = 0;
            a.vmax[sig] = FLT_MAX;
            a.status[sig] |= BMPL_SIG_INEXACT;
        }
        s_lim = a.nsel[sig];
    }
    __syncthreads();
    for (int q = s_lim + tid; q < a.selcap && q < k; q += 256) a.sel[(int64_t)sig * a.selcap + q] = -1;
}

// ---------------------------------------------------------------------------
// e4m3 ranking.  The e4m3 product only orders the atoms: its error (about 2^-3 of
// ||a|| ||xi||, far wider than bfloat16's) is too large to certify anything.  The
// highest-ranked candidates are re-scored exactly (float32 data, float64 sums); the
// exact violators among them, largest first (ties to the lower index), are admitted,
// at most k.  A signal with no exact violator among its candidates may have converged
// or may hide violators the ranking missed: it is flagged for the certified pass.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void rank8_kernel(Rank8Args a)
{
    constexpr int CMAX = 64;
    __shared__ double s_val[CMAX];
    __shared__ int s_idx[CMAX];
    const int n_act = a.n_act_dev ? *a.n_act_dev : a.p_grid;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act ? a.act[row] : row;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nc = min(a.ncand[sig], min(a.candcap, CMAX));
    const float* r = a.R + (int64_t)sig * a.ldr;
    for (int c = wave; c < nc; c += 4) {
        const int j = a.cand[(int64_t)sig * a.candcap + c];
        const float4* aj = reinterpret_cast<const float4*>(a.At + (int64_t)j * a.lda);
        const double acc = wave_dot_f64(aj, reinterpret_cast<const float4*>(r), a.kpad / 4, lane);
        if (lane == 0) { s_val[c] = fabs(acc); s_idx[c] = j; }
    }
    __syncthreads();
    int k = a.k;
    if (a.nI && a.max_active > 0) {
        const int room = a.max_active - a.nI[sig];
        k = room < k ? (room > 0 ? room : 0) : k;
    }
    const double lam = a.lam[sig];
    int nsel = 0;
    double vmx = 0.0;
    for (int c = 0; c < nc; ++c) {             // every thread, small loops: counts and the maximum
        vmx = fmax(vmx, s_val[c]);
        nsel += s_val[c] > lam;
    }
    nsel = nsel < k ? nsel : k;
    if (tid < nc && s_val[tid] > lam) {
        const double v = s_val[tid];
        const int j = s_idx[tid];
        int rank = 0;
        for (int c = 0; c < nc; ++c)
            rank += s_val[c] > lam && (s_val[c] > v || (s_val[c] == v && s_idx[c] < j));
        if (rank < k) a.sel[(int64_t)sig * a.selcap + rank] = j;
    }
    if (tid == 0) {
        a.nsel[sig] = nsel;
        a.vmax[sig] = (float)vmx;
        a.cert[sig] = nsel == 0 ? 1 : 0;
        if (nsel == 0 && a.cert_act) a.cert_act[atomicAdd(a.n_cert, 1)] = sig;
    }
}

__global__ __launch_bounds__(256) void atoms_fp8_kernel(const float* __restrict__ At, int64_t lda, int kpad,
                                                        uint8_t* __restrict__ A8, float* __restrict__ ascale, int m)
{
    __shared__ float red[4];
    const int j = blockIdx.x;
    if (j >= m) return;
    const float* a = At + (int64_t)j * lda;
    float mx = 0.f;
    for (int k = threadIdx.x; k < kpad; k += 256) mx = fmaxf(mx, fabsf(a[k]));
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    const float s = fp8_pow2_scale(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
    const float inv = 1.0f / s;        // exact: s is a power of two
    for (int k = threadIdx.x; k < kpad; k += 256) A8[(int64_t)j * kpad + k] = fp8_e4m3(a[k] * inv);
    if (threadIdx.x == 0) ascale[j] = s;
}

}  // namespace

hipError_t launch_to_bf16(const float* src, int64_t lds, uint16_t* dst, int64_t ldd, int rows, int cols,
                          hipStream_t stream)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(rows), dim3(256), 0, stream, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_atom_norms(const float* At, int64_t lda, int n, float* norms, int m, hipStream_t stream)
{
    hipLaunchKernelGGL(atom_norm_kernel, dim3(m), dim3(256), 0, stream, At, lda, n, norms, m);
    return hipGetLastError();
}

hipError_t launch_screen(const ScreenArgs& a, hipStream_t stream)
{
    if (a.p_grid <= 0) return hipSuccess;
    if (a.k < 0 || a.k > 64) return hipErrorInvalidValue;
    if (a.k <= 16)
        hipLaunchKernelGGL(screen_select_kernel<16>, dim3(a.p_grid), dim3(256), 0, stream, a);
    else if (a.k <= 32)
        hipLaunchKernelGGL(screen_select_kernel<32>, dim3(a.p_grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(screen_select_kernel<64>, dim3(a.p_grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_rescore(const RescoreArgs& a, hipStream_t stream)
{
    if (a.p_grid <= 0) return hipSuccess;
    const size_t lds = (size_t)a.candcap_lds * (sizeof(double) + sizeof(float)) + (size_t)a.kpad * sizeof(float);
    hipLaunchKernelGGL(rescore_kernel, dim3(a.p_grid), dim3(256), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_rank8(const Rank8Args& a, hipStream_t stream)
{
    if (a.p_grid <= 0) return hipSuccess;
    if (a.kpad % 4 || a.lda % 4 || a.ldr % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rank8_kernel, dim3(a.p_grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_atoms_fp8(const float* At, int64_t lda, int kpad, uint8_t* A8, float* ascale, int m,
                            hipStream_t stream)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(atoms_fp8_kernel, dim3(m), dim3(256), 0, stream, At, lda, kpad, A8, ascale, m);
    return hipGetLastError();
}

}  // namespace bmpl
