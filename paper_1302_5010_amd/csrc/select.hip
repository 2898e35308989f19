// Worst-case analysis (Algorithm 1, step 3): per running signal, pick the atoms
// outside the active set I with the largest |g_j| that violate |g_j| > lambda
// (the natural stopping condition, Eq. (9), fails exactly for these), at most k
// of them, largest first, ties to the lower atom index.
//
// One 256-thread workgroup per signal reads its row of correlations once
// (coalesced).  Each thread's first eight 16-byte loads stay in registers; the
// k-th largest of the threads' maxima over them bounds the row's k-th largest from
// below, so when each thread then keeps a sorted top-KMAX list in registers, of the
// registered entries and of the rest of the row as it streams in, only entries at
// or above that bound are inserted (few, so the list insertions stay rare).  Each wave then
// merges its 64 lists with k rounds of a wave-wide argmax on the list heads
// (cross-lane shuffles, no LDS); the four wave lists are ranked in LDS.
// On the first pass of the relative lambda rule the row maximum is reduced first
// and lambda_i = c * ||A^T b_i||_inf is set from it (Section IV-A).
#include <float.h>
#include <limits.h>
#include <stdint.h>

#include "bmpl_internal.h"

namespace bmpl {
namespace {

__device__ inline bool better(float v, int i, float w, int j)
{
    return v > w || (v == w && i < j);
}

template <int KMAX>
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a)
{
    const int n_act = a.n_act_dev ? *a.n_act_dev : a.p_grid;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act ? a.act[row] : row;
    const float* g = a.G + (int64_t)row * a.ldg;
    const uint32_t* ex = a.excl ? a.excl + (int64_t)sig * a.words : nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ float s_red[4];
    __shared__ float s_val[4 * KMAX];
    __shared__ int s_idx[4 * KMAX];
    __shared__ double s_lam;

    // Per-signal cap on the number of atoms admitted this pass.
    int k = a.k;
    if (a.nI && a.max_active > 0) {
        int room = a.max_active - a.nI[sig];
        k = room < k ? (room > 0 ? room : 0) : k;
    }

    // Rows are read as float4 when the layout allows it (the internal buffers always do).
    const bool vec4 = ((a.ldg & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.G) & 15) == 0);
    const int m4 = vec4 ? (a.m & ~3) : 0;

    // Pass 1 (relative lambda rule only): lambda_i = c * max_j |g_j|.
    if (a.lam_rel > 0.0) {
        float mx = 0.f;
#pragma unroll 4
        for (int j0 = 4 * tid; j0 < m4; j0 += 1024) {
            const float4 f = *reinterpret_cast<const float4*>(g + j0);
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(f.x), fabsf(f.y)), fmaxf(fabsf(f.z), fabsf(f.w))));
        }
        for (int j = m4 + tid; j < a.m; j += 256) mx = fmaxf(mx, fabsf(g[j]));
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        if (lane == 0) s_red[wave] = mx;
        __syncthreads();
        if (tid == 0) {
            float v = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
            a.lam[sig] = a.lam_rel * (double)v;
        }
        __syncthreads();
    }
    if (tid == 0) s_lam = a.lam[sig];
    __syncthreads();
    const double lam = s_lam;
    // (double)v > lam  <=>  v > lamf for every float v, with lamf the largest float <= lam
    float lamf = (float)lam;
    if ((double)lamf > lam) lamf = nextafterf(lamf, -INFINITY);

    // Each thread's first CH float4 of the row stay in registers; the rest is streamed once later.
    constexpr int CH = 8;
    float4 f0[CH];
    uint32_t w0[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int j0 = 4 * tid + 1024 * q;
        const bool in = j0 < m4;
        f0[q] = in ? *reinterpret_cast<const float4*>(g + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
        w0[q] = (ex && in) ? (ex[j0 >> 5] >> (j0 & 31)) : 0xFu;   // 4 atoms share one word; 0xF: absent
    }
    // The k-th largest of the 256 threads' maxima over their registered entries is at most the k-th
    // largest |g_j| of the row (they are k distinct entries of it), so only entries >= T can be among
    // the k largest: the insertions below skip the rest.
    float tmax = -1.f;
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        if (!(w0[q] & 1u)) tmax = fmaxf(tmax, fabsf(f0[q].x));
        if (!(w0[q] & 2u)) tmax = fmaxf(tmax, fabsf(f0[q].y));
        if (!(w0[q] & 4u)) tmax = fmaxf(tmax, fabsf(f0[q].z));
        if (!(w0[q] & 8u)) tmax = fmaxf(tmax, fabsf(f0[q].w));
    }
    float vmx = fmaxf(tmax, 0.f);
    {
        float cur = tmax;
        for (int r = 0; r < k; ++r) {
            float b = cur;
            for (int o = 32; o > 0; o >>= 1) b = fmaxf(b, __shfl_xor(b, o));
            if (lane == 0) s_val[wave * KMAX + r] = b;
            const unsigned long long owners = __ballot(cur == b);
            if (lane == __ffsll((long long)owners) - 1) cur = -2.f;   // pop one holder
        }
    }
    __syncthreads();
    if (tid == 0) {
        float T = INFINITY;                        // k = 0: nothing is admitted
        int p0 = 0, p1 = 0, p2 = 0, p3 = 0;        // merge the four descending wave lists
        for (int r = 0; r < k; ++r) {
            const float v0 = p0 < k ? s_val[p0] : -3.f, v1 = p1 < k ? s_val[KMAX + p1] : -3.f;
            const float v2 = p2 < k ? s_val[2 * KMAX + p2] : -3.f, v3 = p3 < k ? s_val[3 * KMAX + p3] : -3.f;
            const float bv = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
            T = bv;
            if (bv == v0) ++p0; else if (bv == v1) ++p1; else if (bv == v2) ++p2; else ++p3;
        }
        s_red[0] = T;
    }
    __syncthreads();
    const float T = s_red[0];
    __syncthreads();

    // Pass B: per-thread sorted top-KMAX lists of the entries >= T that violate.
    float val[KMAX];
    int idx[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) { val[q] = -1.f; idx[q] = INT_MAX; }
    auto consider = [&](int j, float v) {
        if (!(v > lamf) || !(v >= T) || !(v > val[KMAX - 1])) return;
        float cv = v;
        int ci = j;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {   // stable insertion: equal values keep lower index first
            bool sw = cv > val[q];
            float tv = val[q];
            int ti = idx[q];
            val[q] = sw ? cv : tv;
            idx[q] = sw ? ci : ti;
            cv = sw ? tv : cv;
            ci = sw ? ti : ci;
        }
    };
    // the registered entries, then the rest of the row in one stream (vmax over every entry outside I)
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int j0 = 4 * tid + 1024 * q;
        if (!(w0[q] & 1u)) consider(j0, fabsf(f0[q].x));
        if (!(w0[q] & 2u)) consider(j0 + 1, fabsf(f0[q].y));
        if (!(w0[q] & 4u)) consider(j0 + 2, fabsf(f0[q].z));
        if (!(w0[q] & 8u)) consider(j0 + 3, fabsf(f0[q].w));
    }
    auto visit = [&](int j, float v) {
        vmx = fmaxf(vmx, v);
        consider(j, v);
    };
    constexpr int CS = 4;   // float4 loads per thread in flight in the stream
    for (int base = 4 * tid + 1024 * CH; base < m4; base += 1024 * CS) {
        float4 f[CS];
        uint32_t word[CS];
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const int j0 = base + 1024 * q;
            const bool in = j0 < m4;
            f[q] = in ? *reinterpret_cast<const float4*>(g + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
            word[q] = (ex && in) ? (ex[j0 >> 5] >> (j0 & 31)) : 0u;
        }
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const int j0 = base + 1024 * q;
            if (j0 >= m4) break;
            if (!(word[q] & 1u)) visit(j0, fabsf(f[q].x));
            if (!(word[q] & 2u)) visit(j0 + 1, fabsf(f[q].y));
            if (!(word[q] & 4u)) visit(j0 + 2, fabsf(f[q].z));
            if (!(word[q] & 8u)) visit(j0 + 3, fabsf(f[q].w));
        }
    }
    for (int j = m4 + tid; j < a.m; j += 256) {
        if (ex && ((ex[j >> 5] >> (j & 31)) & 1u)) continue;
        visit(j, fabsf(g[j]));
    }
    // vmax over the signal (outside I)
    for (int o = 32; o > 0; o >>= 1) vmx = fmaxf(vmx, __shfl_xor(vmx, o));
    __syncthreads();
    if (lane == 0) s_red[wave] = vmx;

    // Wave merge: k rounds of argmax over the 64 list heads.
    for (int r = 0; r < k; ++r) {
        float bv = val[0];
        int bi = idx[0];
        for (int o = 32; o > 0; o >>= 1) {
            float ov = __shfl_xor(bv, o);
            int oi = __shfl_xor(bi, o);
            if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { s_val[wave * KMAX + r] = bv; s_idx[wave * KMAX + r] = bi; }
        if (bv < 0.f) {
            for (int rr = r + 1; rr < k && lane == 0; ++rr) { s_val[wave * KMAX + rr] = -1.f; s_idx[wave * KMAX + rr] = INT_MAX; }
            break;
        }
        if (idx[0] == bi) {   // the winning lane pops its head
#pragma unroll
            for (int q = 0; q < KMAX - 1; ++q) { val[q] = val[q + 1]; idx[q] = idx[q + 1]; }
            val[KMAX - 1] = -1.f;
            idx[KMAX - 1] = INT_MAX;
        }
    }
    __syncthreads();
    // Rank the 4k wave candidates; candidate c lands at its rank if < k.
    int cnt = 0;
    if (tid < 4 * k) {
        const int w = tid / k, r = tid % k;
        const float v = s_val[w * KMAX + r];
        const int i = s_idx[w * KMAX + r];
        if (v >= 0.f) {
            int rank = 0;
            for (int c = 0; c < 4 * k; ++c) {
                const float ov = s_val[(c / k) * KMAX + c % k];
                const int oi = s_idx[(c / k) * KMAX + c % k];
                if (ov >= 0.f && better(ov, oi, v, i)) ++rank;
            }
            if (rank < k) a.sel[(int64_t)sig * a.selcap + rank] = i;
        }
    }
    // count = number of valid candidates, capped at k
    if (tid == 0) {
        for (int c = 0; c < 4 * k; ++c) cnt += s_val[(c / k) * KMAX + c % k] >= 0.f;
        cnt = cnt < k ? cnt : k;
        a.nsel[sig] = cnt;
        a.vmax[sig] = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
    }
    __syncthreads();
    if (tid == 0) { s_red[0] = (float)a.nsel[sig]; }
    __syncthreads();
    const int nsel = (int)s_red[0];
    for (int q = nsel + tid; q < a.selcap && q < k; q += 256) a.sel[(int64_t)sig * a.selcap + q] = -1;
}

}  // namespace

hipError_t launch_select(const SelectArgs& a, hipStream_t stream)
{
    if (a.p_grid <= 0) return hipSuccess;
    if (a.k <= 0 || a.k > 64 || a.k > a.selcap) return hipErrorInvalidValue;
    if (a.k <= 16)
        hipLaunchKernelGGL(select_kernel<16>, dim3(a.p_grid), dim3(256), 0, stream, a);
    else if (a.k <= 32)
        hipLaunchKernelGGL(select_kernel<32>, dim3(a.p_grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(select_kernel<64>, dim3(a.p_grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace bmpl
