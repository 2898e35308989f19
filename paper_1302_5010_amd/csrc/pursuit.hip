// Per-signal kernels of the batched pursuit: set-up, the stop/compaction step,
// the master problem on the ragged active sets, and result packing.
//
// Master problem (Eq. (7)): min_x lambda ||x||_1 + 1/2 ||b - A x||^2 with
// x = 0 outside the active set I.  The paper runs proximal gradient on it; here
// it is solved exactly, warm-started from the previous outer iteration
// (Algorithm 1, step 4), by a sign-fixed active-set method on the support
// S subset of I:
//   * for a fixed support S and signs theta the minimiser is
//     x_S = G_SS^{-1} (c_S - lambda theta_S), with G = A_I^T A_I and c = A_I^T b;
//   * atoms of I \ S whose gradient c_u - G_uS x_S exceeds lambda in magnitude
//     enter S with the sign of that gradient;
//   * if the new minimiser flips the sign of a coordinate, the step stops at the
//     first zero crossing and that atom leaves S.
// The objective decreases strictly at every non-zero step, so the loop ends at
// the restricted optimum, the point proximal gradient converges to.
//
// G_II is accumulated in float64 from the float32 atoms (products exact, sums in
// float64) and kept packed per signal, grown by rows as atoms enter I (atoms
// never leave I).  G_SS is represented by its inverse Cholesky factor
// Rinv = L^{-1} (G_SS = L L^T, so G_SS^{-1} = Rinv^T Rinv): adding an atom is a
// Cholesky row append computed from Rinv^T (Rinv g), a solve is Rinv^T (Rinv w)
// (two matrix-vector products, or one pass over a factor in global memory), and
// removing position q is a Givens downdate of the rows below it.
//
// One 256-thread workgroup per signal; signals are independent.
#include <float.h>
#include <limits.h>

#include "../../include/bmpl.h"
#include "bmpl_internal.h"
#include "pursuit.h"
#include "wave_ops.h"

namespace bmpl {
namespace {

constexpr int NT = 256;
constexpr int NB = 16;      // new atoms per Gram pass
constexpr int CH = 64;      // k per Gram staging chunk (direct Gram rows)
constexpr int JADD = 32;    // most violators added to S per active-set step (the largest ones)
constexpr int JADD0 = 8;    // the width a signal starts with
constexpr int LAZY_MIN = 32;   // new slots in one pass above which the Gram matrix is kept lazily
// Exclusion flag of a slot left out of S for the rest of one pass (cleared at the write-back): an
// atom admitted alone whose sign-fixed coefficient came out with the wrong sign.  Alone, its exact
// coefficient is (|g_u| - lambda) / pivot^2 > 0, so the wrong sign means |g_u| exceeds lambda by
// less than the rounding of x*; it would be dropped with no step and admitted again at once.
constexpr unsigned char EX_PASS = 2;
constexpr int JB = SOLVE_JB;   // atoms per block factor append

__device__ inline double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// block_sum for a caller that has passed a barrier since the last read of red (saves the first one).
__device__ inline double block_sum_fenced(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__device__ inline double block_max(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// e4m3 copy of residual row `sig` (already written to R by this workgroup) with its power-of-two
// scale, for the e4m3 ranking product.
__device__ inline void write_residual_fp8(const Workspace& w, int sig, double* red)
{
    const float* R = w.R + (int64_t)sig * w.kpad;
    double mx = 0.0;
    for (int r = threadIdx.x; r < w.kpad; r += NT) mx = fmax(mx, (double)fabsf(R[r]));
    const float s = fp8_pow2_scale((float)block_max(mx, red));   // the barriers also publish R
    const float inv = 1.0f / s;
    uint8_t* R8 = w.R8 + (int64_t)sig * w.kpad;
    for (int r = threadIdx.x; r < w.kpad; r += NT) R8[r] = fp8_e4m3(R[r] * inv);
    if (threadIdx.x == 0) w.rscale8[sig] = s;
}

// (alpha, position) minimum, ties to the smaller position.
__device__ inline void block_argmin(double& a, int& q, double* red, int* redi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto take = [&](double oa, int oq) {
        if (oa < a || (oa == a && (unsigned)oq < (unsigned)q)) { a = oa; q = oq; }
    };
    take(lane_move<DPP_XOR1>(a), lane_move<DPP_XOR1>(q));
    take(lane_move<DPP_XOR2>(a), lane_move<DPP_XOR2>(q));
    take(lane_move<DPP_HALF_MIRROR>(a), lane_move<DPP_HALF_MIRROR>(q));
    take(lane_move<DPP_MIRROR>(a), lane_move<DPP_MIRROR>(q));
    take(lane_move<-1>(a), lane_move<-1>(q));
    {
        const double a0 = read_lane(a, 0), a1 = read_lane(a, 32);
        const int q0 = __builtin_amdgcn_readlane(q, 0), q1 = __builtin_amdgcn_readlane(q, 32);
        a = a0; q = q0;
        take(a1, q1);
    }
    __syncthreads();
    if (lane == 0) { red[wave] = a; redi[wave] = q; }
    __syncthreads();
    a = red[0];
    q = redi[0];
    for (int w = 1; w < 4; ++w)
        if (red[w] < a || (red[w] == a && (unsigned)redi[w] < (unsigned)q)) { a = red[w]; q = redi[w]; }
}

// A block of `sz` doubles from the arena (one thread calls it), or null when no chunk has room.  The
// offset `top` only grows (one fetch-and-add per request, so many workgroups allocate at once without
// retry loops); a range that would straddle the end of a chunk is abandoned and the request is made
// again, which lands past that end.  The chunk list is constant while kernels run.
__device__ double* arena_alloc(Arena* A, unsigned long long sz)
{
    const int nc = A->nchunks;
    for (int attempt = 0; attempt < 4; ++attempt) {
        const unsigned long long off = atomicAdd(&A->top, sz);
        int c = 0;
        while (c < nc && off >= A->start[c] + A->size[c]) ++c;
        if (c == nc) return nullptr;
        if (off + sz <= A->start[c] + A->size[c]) return A->base[c] + (off - A->start[c]);
    }
    return nullptr;
}

// The factor when it is held in LDS, addressed as LDS: the compiler then reads it with LDS
// instructions instead of generic (flat) ones, which wait on both memory counters.
typedef __attribute__((address_space(3))) double lds_double;
__device__ __forceinline__ lds_double* to_lds(double* p) { return (lds_double*)p; }
__device__ __forceinline__ const lds_double* to_lds(const double* p) { return (const lds_double*)p; }
// A factor known to be in global memory, addressed as global: loads then take a scalar base and a
// 32-bit lane offset instead of a 64-bit address per load.  p must be the same in every thread.
typedef __attribute__((address_space(1))) const double global_cdouble;
typedef __attribute__((address_space(1))) double global_double;
__device__ __forceinline__ global_cdouble* to_global(const double* p)
{
    // the same pointer in every thread: read it from the first lane so it stays in scalar registers
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (global_cdouble*)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ global_double* to_global(double* p)
{
    return (global_double*)const_cast<global_cdouble*>(to_global(static_cast<const double*>(p)));
}
__device__ __forceinline__ bool is_lds(const double* p)
{
    return __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(p));
}

// Per-signal working view inside the solve kernel.  G is global (row-major,
// stride K); the rest points into LDS or into the global homes.
struct Sig {
    int K;
    bool r_lds;           // R lives in LDS (latency-optimised loops) or in global memory (coalesced loops)
    double* G;            // G_II by slot
    double* R;            // Rinv, packed lower row-major by support position
    double* x;            // coefficient by slot
    double* c;            // a_u^T b by slot
    signed char* th;      // sign by slot, 0 = not in S
    unsigned char* ex;    // slot excluded from S
    int* so;              // slot of each support position
};

// z[i] = sum_{k <= i} R(i, k) w[k] for i < s with the factor in global memory: one row per wave at a
// time, lanes across the row (coalesced, eight loads in flight: clamped indices, so no load is guarded
// by a branch that would wait for it), a wave reduction per row.
__device__ inline void rows_matvec_global(const double* R, const double* w, double* z, int s)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < s; i += NT / 64) {
        const double* Ri = R + tri(i);
        double a0 = 0.0, a1 = 0.0;
        for (int k0 = lane; k0 <= i; k0 += 512) {
            double r[8], wv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + 64 * e <= i ? k0 + 64 * e : i;
                r[e] = Ri[k];
                wv[e] = w[k];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
                (e & 1 ? a1 : a0) += k0 + 64 * e <= i ? r[e] * wv[e] : 0.0;
        }
        const double acc = wave_sum(a0 + a1);
        if (lane == 0) z[i] = acc;
    }
}

// Lanes per row (or column) of an LDS-resident factor with s support positions: a short support
// leaves most threads idle, so P consecutive lanes share a row and the serial chain is s / P long.
__device__ inline int split_lanes(int s) { return s <= NT / 4 ? 4 : (s <= NT / 2 ? 2 : 1); }

// z[i] = sum_{k <= i} R(i, k) v[k] for i < s (packed lower factor in LDS), split_lanes(s) lanes per
// row combined by shuffles inside the group.  Returns this lane's share of sum_i z_i^2.
template <class VP>
__device__ inline double rows_matvec_lds_t(const lds_double* R, VP v, double* z, int s)
{
    const int P = split_lanes(s);
    const int sub = threadIdx.x & (P - 1);
    double part = 0.0;
    for (int i = threadIdx.x / P; i < s; i += NT / P) {   // the P lanes of a group share i
        const lds_double* Ri = R + tri(i);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int k = sub;
        for (; k + 3 * P <= i; k += 4 * P) {
            a0 += Ri[k] * v[k];
            a1 += Ri[k + P] * v[k + P];
            a2 += Ri[k + 2 * P] * v[k + 2 * P];
            a3 += Ri[k + 3 * P] * v[k + 3 * P];
        }
        for (; k <= i; k += P) a0 += Ri[k] * v[k];
        const double acc = group_sum((a0 + a1) + (a2 + a3), P);
        if (sub == 0) {
            z[i] = acc;
            part += acc * acc;
        }
    }
    return part;
}

__device__ inline double rows_matvec_lds(const double* Rg, const double* v, double* z, int s)
{
    // the vector too is addressed as LDS when it lives there (the usual case)
    if (__builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(v)))
        return rows_matvec_lds_t(to_lds(Rg), to_lds(v), z, s);
    return rows_matvec_lds_t(to_lds(Rg), v, z, s);
}

// out[k] = (sum_{i = k}^{s-1} v[i] R(i, k)) / div for k < s (packed lower factor in LDS),
// split_lanes(s) lanes per column.
template <class VP, class OP>
__device__ inline void cols_matvec_lds_t(const lds_double* R, VP v, OP out, int s, double div)
{
    const int P = split_lanes(s);
    const int sub = threadIdx.x & (P - 1);
    for (int k = threadIdx.x / P; k < s; k += NT / P) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = k + sub;
        for (; i + 3 * P < s; i += 4 * P) {
            a0 += v[i] * R[tri(i) + k];
            a1 += v[i + P] * R[tri(i + P) + k];
            a2 += v[i + 2 * P] * R[tri(i + 2 * P) + k];
            a3 += v[i + 3 * P] * R[tri(i + 3 * P) + k];
        }
        for (; i < s; i += P) a0 += v[i] * R[tri(i) + k];
        const double acc = group_sum((a0 + a1) + (a2 + a3), P);
        if (sub == 0) out[k] = acc / div;
    }
}

// out[k] = (sum_{i >= k} v[i] R(i, k)) / div for k < s (the factor in LDS), split_lanes(s) lanes per
// column; the vector and the output are addressed as LDS too when both live there.
__device__ inline void cols_matvec_lds(const double* R, const double* v, double* out, int s, double div)
{
    if (__builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(v)) &&
        __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(out)))
        cols_matvec_lds_t(to_lds(R), to_lds(v), to_lds(out), s, div);
    else
        cols_matvec_lds_t(to_lds(R), v, out, s, div);
}

// sum_{i = k}^{s-1} v[i] R(i, k) over column k of a packed lower factor.
__device__ inline double col_dot(const Sig& f, const double* v, int k, int s)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (f.r_lds) {
        const lds_double* R = to_lds(f.R);
        int i = k;
        int o = (int)(tri(k) + k);           // offset of R(i, k); the next row adds i + 1
        for (; i + 4 <= s; i += 4) {
            const int o1 = o + i + 1, o2 = o1 + i + 2, o3 = o2 + i + 3;
            a0 += v[i] * R[o];
            a1 += v[i + 1] * R[o1];
            a2 += v[i + 2] * R[o2];
            a3 += v[i + 3] * R[o3];
            o = o3 + i + 4;
        }
        for (; i < s; ++i) {
            a0 += v[i] * R[o];
            o += i + 1;
        }
    } else {
        // global factor: rows in lockstep across the wave so loads of one row coalesce; eight rows'
        // loads in flight (rows above k read row k instead and count zero, so no load is guarded)
        int i = k & ~63;
        for (; i + 8 <= s; i += 8) {
            double r[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) r[e] = f.R[tri(i + e >= k ? i + e : k) + k];
#pragma unroll
            for (int e = 0; e < 8; ++e) r[e] = i + e >= k ? r[e] : 0.0;
            a0 += v[i] * r[0] + v[i + 4] * r[4];
            a1 += v[i + 1] * r[1] + v[i + 5] * r[5];
            a2 += v[i + 2] * r[2] + v[i + 6] * r[6];
            a3 += v[i + 3] * r[3] + v[i + 7] * r[7];
        }
        for (; i < s; ++i)
            if (i >= k) a0 += v[i] * f.R[tri(i) + k];
    }
    return (a0 + a1) + (a2 + a3);
}

// Rinv^T (Rinv w) in one pass over a factor in global memory with s <= 1024 positions:
// z_i = sum_{k <= i} R(i, k) w[k] and out_k = sum_i z_i R(i, k) / div.  The columns are split over
// the waves (wave v owns the 64-column chunks v, v + 4, v + 8, v + 12, lane l column l of each), the
// rows taken in batches: a wave loads its chunks of the batch's rows (chunks past a row's diagonal
// are skipped by a test on the row index, a scalar branch that leaves the loads in flight; the chunk
// that holds the diagonal is read whole and masked, so every load of the wave shares one lane
// offset: it reads at most 63 entries past the factor's last one, which lie inside the signal's slot
// block, where the per-slot vectors follow the factor), forms its partial dot products, and the four
// waves' partials meet in LDS (double-buffered, one barrier per batch, added in wave order) to give
// z_i, which each lane folds into its columns' sums while the rows are still in registers.  A row
// below 512 has at most two chunks per wave, so batches there take 8 rows (4 beyond): up to sixteen
// loads per lane in flight in every batch.  One read of the factor, instead of a row pass
// and a column pass that waits for its loads row by row.  Every thread ends with the same sum of
// z_i^2; z_i goes to z[i] when z is not null.
//   append (gjj > 0): returns the pivot gjj - sum_i z_i^2; when it exceeds 1e-11 gjj, out receives
//     the new factor row (div = -sqrt(pivot)), else out is left alone.
//   solve (gjj = 0): div = 1; returns 0.
// Ends with a barrier when it writes out.
constexpr int FOLD_MAX = 1024;

// Rows [i_begin, i_end) of the one-pass product, RB at a time, each lane's chunks j < NJ.
template <int RB, int NJ>
__device__ inline void fold_rows(global_cdouble* R, int i_begin, int i_end, const double (&g)[4], double (&acc)[4],
                                 double& zz, int& buf, double* z, double (*part)[NT / 64][8])
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int i0 = i_begin; i0 < i_end; i0 += RB) {
        double r[RB][NJ];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int i = i0 + q < i_end ? i0 + q : i_end - 1;   // the same on every lane
            global_cdouble* Ri = R + tri(i);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int c0 = 64 * (wave + 4 * j);
                r[q][j] = c0 <= i ? Ri[c0 + lane] : 0.0;       // whole chunk, masked below
            }
        }
#pragma unroll
        for (int h = 0; h < (RB + 7) / 8; ++h) {
            double pq[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 8 * h; q < RB && q < 8 * h + 8; ++q) {
                double a = 0.0;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const int k = 64 * (wave + 4 * j) + lane;
                    r[q][j] = k <= i0 + q && i0 + q < i_end ? r[q][j] : 0.0;
                    a += r[q][j] * g[j];
                }
                pq[q - 8 * h] = a;
            }
            const double mine = wave_sum8(pq);   // lane l holds the wave's sum for row wave_sum8_index(l)
            if (lane < 8 && 8 * h + wave_sum8_index(lane) < RB) part[buf][wave][8 * h + wave_sum8_index(lane)] = mine;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const double zi = ((part[buf][0][q] + part[buf][1][q]) + part[buf][2][q]) + part[buf][3][q];
            zz += zi * zi;                       // zero past i_end
            if (z && threadIdx.x == 0 && i0 + q < i_end) z[i0 + q] = zi;
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[j] += zi * r[q][j];
        }
        buf ^= 1;
    }
}

__device__ inline double fold_pass_global(const double* R, const double* w, int s, double* out, double* z,
                                          double gjj)
{
    __shared__ double part_lds[2][NT / 64][8];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    s = __builtin_amdgcn_readfirstlane(s);      // the same in every thread: row indices stay scalar
    const int last = s > 0 ? s - 1 : 0;
    double g[4], acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 64 * (wave + 4 * j) + lane;
        g[j] = w[k < s ? k : last];
        acc[j] = 0.0;
    }
    double zz = 0.0;
    int buf = 0;
    global_cdouble* Rg = to_global(R);
    fold_rows<8, 2>(Rg, 0, s < 512 ? s : 512, g, acc, zz, buf, z, part_lds);
    fold_rows<4, 4>(Rg, 512, s, g, acc, zz, buf, z, part_lds);
    double div = 1.0, pivot = 0.0;
    if (gjj > 0.0) {
        pivot = gjj - zz;
        if (!(pivot > 1e-11 * gjj)) return pivot;
        div = -sqrt(pivot);
    }
    // (out's own memory: a generic store would hold up the barrier until it reaches global memory)
    if (is_lds(out)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 64 * (wave + 4 * j) + lane;
            if (k < s) to_lds(out)[k] = acc[j] / div;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 64 * (wave + 4 * j) + lane;
            if (k < s) to_global(out)[k] = acc[j] / div;
        }
    }
    __syncthreads();
    return pivot;
}

// Append slot j with sign th at support position s = nS (a Cholesky row append
// held as the inverse factor).  Returns false and excludes j if its Schur
// complement pivot vanishes, i.e. a_j is numerically in the span of A_S.
template <bool FOLD>
__device__ bool chol_append(Sig& v, int& nS, int j, signed char th, double* vw, double* vz, double* red,
                            uint64_t* cnt)
{
    const int s = nS;
    const int tid = threadIdx.x;
    const uint64_t t_in = cnt ? wall_clock64() : 0;
    if (cnt && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(cnt), 1ull);
    const double* Gj = v.G + (int64_t)j * v.K;
    __shared__ double s_gjj;
    // w = G(S, j): four positions per thread at once, slot numbers first and then the gathers (clamped
    // indices: a load behind a per-thread test would be waited for before the next one is issued)
    for (int k0 = tid; k0 < s; k0 += 4 * NT) {
        int sk[4];
        double gv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + NT * e;
            sk[e] = v.so[k < s ? k : s - 1];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) gv[e] = Gj[sk[e]];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (k0 + NT * e < s) vw[k0 + NT * e] = gv[e];
    }
    if (tid == 0) s_gjj = Gj[j];
    __syncthreads();
    double* Rs = v.R + tri(s);
    const double gjj = s_gjj;
    const bool fold = FOLD && !v.r_lds && s <= FOLD_MAX;   // one pass over a global factor
    double dd;
    if (fold) {
        dd = fold_pass_global(v.R, vw, s, Rs, nullptr, gjj);   // writes the new row if dd is a pivot
    } else {
        double part = 0.0;
        if (v.r_lds) {
            part = rows_matvec_lds(v.R, vw, vz, s);    // z = Rinv w
        } else {
            rows_matvec_global(v.R, vw, vz, s);
            __syncthreads();
            for (int i = tid; i < s; i += NT) part += vz[i] * vz[i];
        }
        dd = gjj - block_sum_fenced(part, red);   // the barrier after the gather fences red
    }
    if (!(dd > 1e-11 * gjj)) {
        if (tid == 0) { v.ex[j] = 1; v.th[j] = 0; v.x[j] = 0.0; }
        __syncthreads();
        if (cnt && tid == 0)   // cnt[-2]: ticks spent in appends (phase slot 4)
            atomicAdd(reinterpret_cast<unsigned long long*>(cnt - 2), (unsigned long long)(wall_clock64() - t_in));
        return false;
    }
    const double d = sqrt(dd);
    if (v.r_lds)                             // new row: -(z^T Rinv)_k / d
        cols_matvec_lds(v.R, vz, Rs, s, -d);
    else if (!fold)
        for (int k = tid; k < s; k += NT) Rs[k] = -col_dot(v, vz, k, s) / d;
    if (tid == 0) {
        Rs[s] = 1.0 / d;
        v.so[s] = j;
        v.th[j] = th;
    }
    nS = s + 1;
    __syncthreads();
    if (cnt && tid == 0)   // cnt[-2]: ticks spent in appends (phase slot 4)
        atomicAdd(reinterpret_cast<unsigned long long*>(cnt - 2), (unsigned long long)(wall_clock64() - t_in));
    return true;
}

// Append the slots list[0..J) (J <= JB), in list order, at support positions nS, nS + 1, ...
// as one block.  With s0 = nS, W = G(S, list) and Z = Rinv W (s0 x J), the Schur complement
// C = G(list, list) - Z^T Z is factored in list order with the single-append pivot rule (an atom
// whose pivot C_ee - |l_e|^2 falls to 1e-11 g_ee or below is excluded, as chol_append would), and
// the accepted atoms A get the inverse-factor rows [-L22^{-1} Z_A^T Rinv, L22^{-1}].  The same
// factor as J single appends in exact arithmetic, for two passes over Rinv instead of 2J.
// Signs come from vg (sign of the gradient) or, with vg == nullptr, from the slots' current theta.
// zs: LDS scratch of (s0 + 1) * JB doubles.
__device__ void chol_append_block(Sig& v, int& nS, const int* list, int J, const double* vg, double* zs,
                                  uint64_t* cnt)
{
    __shared__ double s_C[JB * JB];     // Schur complement (lower), then L22^{-1}
    __shared__ double s_L[JB * JB];     // L22, rows in accepted order
    __shared__ int s_acc[JB];
    __shared__ int s_na;
    const int s0 = nS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t t_in = cnt ? wall_clock64() : 0;
    if (cnt && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(cnt), (unsigned long long)J);

    // 1. W = G(S, list): row k = support position, JB columns, zero past J
    for (int t = tid; t < s0 * JB; t += NT) {
        const int k = t / JB, e = t - k * JB;
        zs[t] = e < J ? v.G[(int64_t)list[e] * v.K + v.so[k]] : 0.0;
    }
    __syncthreads();
    // 2. Z = Rinv W in place.  Rows from the bottom, one per wave per round; row i needs the W rows
    //    at or below it, so a round's rows are written only after every wave has read them.
    for (int top = s0 - 1; top >= 0; top -= NT / 64) {
        const int i = top - wave;
        double acc[JB];
#pragma unroll
        for (int e = 0; e < JB; ++e) acc[e] = 0.0;
        if (i >= 0) {
            const double* Ri = v.R + tri(i);
            for (int k = lane; k <= i; k += 512) {   // eight loads in flight per lane, the row's tail too
                double r[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) r[q] = Ri[k + 64 * q <= i ? k + 64 * q : i];   // clamped, unguarded
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (k + 64 * q > i) break;
                    const double* wk = zs + (k + 64 * q) * JB;
#pragma unroll
                    for (int e = 0; e < JB; ++e) acc[e] += r[q] * wk[e];
                }
            }
        }
        static_assert(JB == 8, "the eight-way wave sum");
        const double val = wave_sum8(acc);   // uniform per wave: every lane takes part
        __syncthreads();
        if (i >= 0 && lane < JB) zs[i * JB + wave_sum8_index(lane)] = val;
    }
    __syncthreads();
    // 3. C = G(list, list) - Z^T Z, lower triangle
    for (int t = tid; t < J * J; t += NT) {
        const int e = t / J, f = t - e * J;
        if (f > e) continue;
        double sum = 0.0;
        for (int i = 0; i < s0; ++i) sum += zs[i * JB + e] * zs[i * JB + f];
        s_C[e * JB + f] = v.G[(int64_t)list[e] * v.K + list[f]] - sum;
    }
    __syncthreads();
    // 4. Cholesky of C in list order with exclusion, then L22^{-1} into s_C (one thread, J <= JB)
    if (tid == 0) {
        int na = 0;
        for (int e = 0; e < J; ++e) {
            double dd = s_C[e * JB + e];
            for (int b = 0; b < na; ++b) {
                double x = s_C[e * JB + s_acc[b]];          // C(e, A_b), A_b < e
                for (int c = 0; c < b; ++c) x -= s_L[na * JB + c] * s_L[b * JB + c];
                x /= s_L[b * JB + b];
                s_L[na * JB + b] = x;
                dd -= x * x;
            }
            const int u = list[e];
            const double gjj = v.G[(int64_t)u * v.K + u];
            if (dd > 1e-11 * gjj) {
                s_L[na * JB + na] = sqrt(dd);
                s_acc[na++] = e;
            } else {
                v.ex[u] = 1; v.th[u] = 0; v.x[u] = 0.0;
            }
        }
        for (int a2 = 0; a2 < na; ++a2) {
            const double dinv = 1.0 / s_L[a2 * JB + a2];
            for (int b = 0; b < a2; ++b) {
                double x = 0.0;
                for (int c = b; c < a2; ++c) x += s_L[a2 * JB + c] * s_C[c * JB + b];
                s_C[a2 * JB + b] = -x * dinv;
            }
            s_C[a2 * JB + a2] = dinv;
        }
        s_na = na;
    }
    __syncthreads();
    const int na = s_na;
    if (na < J) {   // keep only the accepted columns of Z, in accepted order
        for (int i = tid; i < s0; i += NT) {
            double* zi = zs + i * JB;
            for (int b = 0; b < na; ++b) zi[b] = zi[s_acc[b]];
        }
        __syncthreads();
    }
    // 5. New rows: R(s0 + a, k) = -sum_{b <= a} L22^{-1}(a, b) M(b, k), M(b, k) = sum_{i >= k} Z(i, b) R(i, k).
    //    Threads own columns k; a wave's lanes walk the rows in lockstep so reads of one row coalesce.
    for (int kb = 0; kb < s0; kb += NT) {
        const int k = kb + tid;
        double acc[JB];
#pragma unroll
        for (int b = 0; b < JB; ++b) acc[b] = 0.0;
        int i = kb + wave * 64;
        for (; i + 8 <= s0; i += 8) {              // eight rows' loads in flight
            double r[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {   // clamped to row >= column and column < s0: always inside the factor
                const int kk = k < s0 ? k : s0 - 1;
                r[q] = v.R[tri(i + q >= kk ? i + q : kk) + kk];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = i + q >= k ? r[q] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double* zi = zs + (i + q) * JB;
#pragma unroll
                for (int b = 0; b < JB; ++b) acc[b] += r[q] * zi[b];
            }
        }
        for (; i < s0; ++i) {
            if (i >= k) {
                const double r = v.R[tri(i) + k];
                const double* zi = zs + i * JB;
#pragma unroll
                for (int b = 0; b < JB; ++b) acc[b] += r * zi[b];
            }
        }
        if (k < s0) {
#pragma unroll
            for (int a2 = 0; a2 < JB; ++a2) {
                if (a2 >= na) break;
                double val = 0.0;
#pragma unroll
                for (int b = 0; b <= a2; ++b) val += s_C[a2 * JB + b] * acc[b];
                v.R[tri(s0 + a2) + k] = -val;
            }
        }
    }
    for (int t = tid; t < na * JB; t += NT) {
        const int a2 = t / JB, b = t - a2 * JB;
        if (b <= a2) v.R[tri(s0 + a2) + s0 + b] = s_C[a2 * JB + b];
    }
    if (tid < na) {
        const int u = list[s_acc[tid]];
        v.so[s0 + tid] = u;
        v.th[u] = vg ? (vg[u] > 0.0 ? 1 : -1) : v.th[u];
    }
    nS = s0 + na;
    __syncthreads();
    if (cnt && tid == 0)   // cnt[-2]: ticks spent in appends (phase slot 4)
        atomicAdd(reinterpret_cast<unsigned long long*>(cnt - 2), (unsigned long long)(wall_clock64() - t_in));
}

// Append the slots list[0..nv) in order, in blocks of JB, stopping at nmax support positions
// (the remaining slots are excluded).
__device__ void append_list(Sig& v, int& nS, const int* list, int nv, const double* vg, int nmax, double* zs,
                            uint64_t* cnt)
{
    for (int e = 0; e < nv;) {
        if (nS >= nmax) {
            for (int t = threadIdx.x; t < nv - e; t += NT) v.ex[list[e + t]] = 1;
            __syncthreads();
            return;
        }
        int J = nv - e < JB ? nv - e : JB;
        J = J < nmax - nS ? J : nmax - nS;
        chol_append_block(v, nS, list + e, J, vg, zs, cnt);
        e += J;
    }
}

// Remove support position q from the inverse factor in O(|S|^2).  Moving column q of Rinv to the end
// only relabels G's order; Givens rotations of consecutive rows j, j + 1 (j = q .. s-2), each chosen to
// clear row j's entry in the moved column, then restore triangularity.  Rotations act on the left of
// Rinv, so Rinv^T Rinv = G^{-1} is unchanged for the remaining positions, and the leading
// (s-1) x (s-1) block is the new inverse factor (rows may change sign, which no product of the solver
// sees).  One barrier per row: row j's new values land where no later step reads, and the next step's
// writes (row j + 1) wait until every thread has read the old row j + 1.  The moved column's running
// entries live in `cbuf` (s doubles of scratch, each entry owned by one thread), so the downdate needs
// no per-thread arrays whatever |S| is.  The caller shifts the support order.
//
// zc (or null): the cached z = Rinv w of the sign-fixed solve (by position).  Rotating rows rotates z's
// entries the same way (the moved column's w entry moves with it, so every row's product with w is
// unchanged); thread 0 carries them along, and zc[s-1] receives the last (removed) row's value.  On
// return cbuf[0..s-2] holds that last row's entries.
//
// Up to DROP_COLS * 256 positions, each thread keeps its columns' running entries in registers and
// loads the next row's entries one iteration ahead, so the global factor's load latency overlaps the
// barrier; the next row is only read, never written, during an iteration, and the barrier per row keeps
// every read of a row before the iteration that writes it.  (The kernel capped at 128 registers uses a
// narrower register window: four columns, |S| <= 1024.)
template <int DROP_COLS>
__device__ void chol_drop(Sig& v, int s, int q, double* cbuf, double* zc)
{
    const int tid = threadIdx.x;
    if (s <= DROP_COLS * NT) {
        // Loads take clamped, always valid indices and the unused values are zeroed after them: a
        // guarded load compiles to a branch whose end waits for the data, so a thread's loads would run
        // one after another.
        double cv[DROP_COLS], nx[DROP_COLS];
        const bool has_next = q + 1 < s;
#pragma unroll
        for (int t = 0; t < DROP_COLS; ++t) {
            const int c = tid + NT * t;
            const int cq = c < q ? c : q;
            cv[t] = v.R[tri(q) + cq];
            if (has_next) nx[t] = v.R[tri(q + 1) + (c < q ? c : q + 1)];
        }
#pragma unroll
        for (int t = 0; t < DROP_COLS; ++t) {
            const int c = tid + NT * t;
            cv[t] = c < q ? cv[t] : 0.0;
            nx[t] = (has_next && c <= q) ? nx[t] : 0.0;
        }
        double last = v.R[tri(q) + q];
        double b = q + 1 < s ? v.R[tri(q + 1) + q] : 0.0;
        double zcar = (zc && tid == 0) ? zc[q] : 0.0;
        // every thread has its R(q, q) before the owner of column q rewrites row q in the first rotation
        __syncthreads();
        for (int j = q; j < s - 1; ++j) {
            // prefetch row j + 2 (the next iteration's row), columns shifted past the moved one
            double nn[DROP_COLS];
            const bool more = j + 2 < s;   // the same for every thread
            const double* r2 = v.R + tri(j + 2);
            double bn = 0.0;
            if (more) {
#pragma unroll
                for (int t = 0; t < DROP_COLS; ++t) {
                    const int c = tid + NT * t;
                    const int cc = c <= j + 1 ? c : j + 1;
                    nn[t] = r2[cc < q ? cc : cc + 1];
                }
                bn = r2[q];
#pragma unroll
                for (int t = 0; t < DROP_COLS; ++t) nn[t] = tid + NT * t <= j + 1 ? nn[t] : 0.0;
            } else {
#pragma unroll
                for (int t = 0; t < DROP_COLS; ++t) nn[t] = 0.0;
            }
            const double r = hypot(last, b);
            const double cs = r > 0.0 ? b / r : 1.0;
            const double sn = r > 0.0 ? -last / r : 0.0;
            double* out = v.R + tri(j);
#pragma unroll
            for (int t = 0; t < DROP_COLS; ++t) {
                const int c = tid + NT * t;
                if (c <= j) {                    // columns past j stay zero in the moved column
                    out[c] = cs * cv[t] + sn * nx[t];
                    cv[t] = -sn * cv[t] + cs * nx[t];
                }
                nx[t] = nn[t];
            }
            if (zc && tid == 0) {
                const double zn = zc[j + 1];
                zc[j] = cs * zcar + sn * zn;
                zcar = -sn * zcar + cs * zn;
            }
            last = r;
            b = bn;
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < DROP_COLS; ++t) {
            const int c = tid + NT * t;
            if (c < s) cbuf[c] = cv[t];
        }
        if (zc && tid == 0) zc[s - 1] = zcar;
        __syncthreads();
        return;
    }
    for (int c = tid; c < s; c += NT) cbuf[c] = c < q ? v.R[tri(q) + c] : 0.0;
    double last = v.R[tri(q) + q];
    double zcar = (zc && tid == 0) ? zc[q] : 0.0;
    __syncthreads();
    for (int j = q; j < s - 1; ++j) {
        const double* nx = v.R + tri(j + 1);
        const double b = nx[q];
        const double r = hypot(last, b);
        const double cs = r > 0.0 ? b / r : 1.0;
        const double sn = r > 0.0 ? -last / r : 0.0;
        double* out = v.R + tri(j);
        for (int c = tid; c <= j; c += NT) {     // columns past j stay zero in the moved column
            const double nxt = nx[c < q ? c : c + 1];
            const double cv = cbuf[c];
            out[c] = cs * cv + sn * nxt;
            cbuf[c] = -sn * cv + cs * nxt;
        }
        if (zc && tid == 0) {
            const double zn = zc[j + 1];
            zc[j] = cs * zcar + sn * zn;
            zcar = -sn * zcar + cs * zn;
        }
        last = r;
        __syncthreads();
    }
    if (zc && tid == 0) zc[s - 1] = zcar;
    __syncthreads();
}

// chol_drop's register path for a factor in global memory (s <= 4 NT): the same rotations in the same
// order.  Every access names its memory (the factor as global from a scalar base, zc as LDS or global
// by ZK: 0 none, 1 LDS, 2 global): the generic accesses of chol_drop count against the LDS counter
// as well, so its barrier after each step waited for that step's global loads and stores to
// complete.  Here the barrier only orders the workgroup (its waves share one vector L1, which keeps
// their global accesses in order), and the next step's row and zc entry are in flight meanwhile:
// their loads take clamped indices and are not masked (a masked load, or one behind a branch, makes
// the wave wait for it at once), into two buffers that take turns.  Entries past a row's end are
// never used: step j uses row j + 1 in columns c <= j only, and rows past s - 1 (read as row s - 1)
// are never used.  Row r is read two steps before step r rewrites it, with a barrier after every step.
template <int ZK>
__device__ void chol_drop_global_t(Sig& v, int s, int q, double* cbuf, double* zc)
{
    constexpr int DC = 4;
    const int tid = threadIdx.x;
    s = __builtin_amdgcn_readfirstlane(s);
    q = __builtin_amdgcn_readfirstlane(q);
    global_double* R = to_global(v.R);
    // row r >= q + 1 with column q moved out (entry c from column c if c < q, else c + 1; clamped
    // into the row), and bq = R(r, q)
    auto load_row = [&](int r, double (&o)[DC], double& bq) {
        r = r < s ? r : s - 1;
        global_double* Rr = R + tri(r);
#pragma unroll
        for (int t = 0; t < DC; ++t) {
            const int c = tid + NT * t;
            const int cc = c <= r - 1 ? c : r - 1;
            o[t] = Rr[cc < q ? cc : cc + 1];
        }
        bq = Rr[q];
    };
    auto load_z = [&](int r) -> double {
        r = r < s ? r : s - 1;
        if (ZK == 1) return to_lds(zc)[r];
        if (ZK == 2) return to_global(zc)[r];
        return 0.0;
    };
    double cv[DC], ra[DC], rb[DC];
    {
        global_double* Rq = R + tri(q);
#pragma unroll
        for (int t = 0; t < DC; ++t) {
            const int c = tid + NT * t;
            cv[t] = Rq[c < q ? c : q];
        }
#pragma unroll
        for (int t = 0; t < DC; ++t) cv[t] = tid + NT * t < q ? cv[t] : 0.0;
    }
    double ba = 0.0, bb = 0.0;
    if (q + 1 < s) load_row(q + 1, ra, ba);
    double za = load_z(q + 1), zb = 0.0;
    double last = R[tri(q) + q];
    double zcar = load_z(q);
    // every thread has its R(q, q) before the owner of column q rewrites row q in the first rotation
    __syncthreads();
    // Step j rotates with row j + 1 (in X) and loads row j + 2 into Z, the buffer step j - 1 used; the
    // two buffers take turns by name (a copy of a register that a load is still filling would wait
    // for the load).
    auto step = [&](int j, const double (&X)[DC], double bX, double zX, double (&Z)[DC], double& bZ, double& zZ) {
        load_row(j + 2, Z, bZ);
        zZ = load_z(j + 2);
        const double r = hypot(last, bX);
        const double cs = r > 0.0 ? bX / r : 1.0;
        const double sn = r > 0.0 ? -last / r : 0.0;
        global_double* out = R + tri(j);
#pragma unroll
        for (int t = 0; t < DC; ++t) {
            const int c = tid + NT * t;
            if (c <= j) {                    // columns past j stay zero in the moved column
                out[c] = cs * cv[t] + sn * X[t];
                cv[t] = -sn * cv[t] + cs * X[t];
            }
        }
        if (ZK != 0) {
            const double zj = cs * zcar + sn * zX;
            zcar = -sn * zcar + cs * zX;
            if (tid == 0) {
                if (ZK == 1) to_lds(zc)[j] = zj;
                else to_global(zc)[j] = zj;
            }
        }
        last = r;
        __syncthreads();
    };
    for (int j = q; j < s - 1; j += 2) {
        step(j, ra, ba, za, rb, bb, zb);
        if (j + 1 >= s - 1) break;
        step(j + 1, rb, bb, zb, ra, ba, za);
    }
#pragma unroll
    for (int t = 0; t < DC; ++t) {
        const int c = tid + NT * t;
        if (c < s) cbuf[c] = cv[t];
    }
    if (ZK != 0 && tid == 0) {
        if (ZK == 1) to_lds(zc)[s - 1] = zcar;
        else to_global(zc)[s - 1] = zcar;
    }
    __syncthreads();
}

// chol_drop_global_t for a zc in global memory (the fold kernel's large supports)
__device__ inline void chol_drop_global(Sig& v, int s, int q, double* cbuf, double* zc)
{
    chol_drop_global_t<2>(v, s, q, cbuf, zc);
}

// The sign-fixed minimiser after support positions s0..s1-1 were appended to the factor, from the cached
// z = Rinv w and x* = Rinv^T z of the positions before: the new factor is Rinv with rows s0..s1-1 added
// (its earlier rows unchanged), and w only gains the entries of the new positions (a member's sign does
// not change while it stays in S), so z gains the new rows' products with w and x* gains those rows'
// contributions: O((s1 - s0) s1) work instead of two passes over the factor.  vw: scratch.
__device__ void xstar_after_append(const Sig& v, int s0, int s1, double lam, double* vw, double* vzc, double* vx,
                                   double* red)
{
    const int tid = threadIdx.x;
    for (int k = tid; k < s1; k += NT) {
        const int u = v.so[k];
        vw[k] = v.c[u] - lam * (double)v.th[u];
    }
    __syncthreads();
    for (int p = s0; p < s1; ++p) {
        const double* Rp = v.R + tri(p);
        double part = 0.0;
        for (int k = tid; k <= p; k += NT) part += Rp[k] * vw[k];
        const double zp = block_sum(part, red);
        if (tid == 0) vzc[p] = zp;
    }
    __syncthreads();
    for (int k = tid; k < s1; k += NT) {
        double acc = k < s0 ? vx[k] : 0.0;
        for (int p = k > s0 ? k : s0; p < s1; ++p) acc += v.R[tri(p) + k] * vzc[p];
        vx[k] = acc;
    }
    __syncthreads();
}

// x_S = Rinv^T Rinv (c_S - lambda theta_S) into vx[0..nS).
template <bool FOLD>
__device__ void sign_fixed_solve(const Sig& v, int nS, double lam, double* vw, double* vz, double* vx)
{
    const int tid = threadIdx.x;
    for (int k = tid; k < nS; k += NT) {
        const int u = v.so[k];
        vw[k] = v.c[u] - lam * (double)v.th[u];
    }
    __syncthreads();
    if (FOLD && !v.r_lds && nS <= FOLD_MAX) {   // one pass over a global factor
        fold_pass_global(v.R, vw, nS, vx, vz, 0.0);
        return;
    }
    if (v.r_lds) {
        rows_matvec_lds(v.R, vw, vz, nS);
    } else {
        rows_matvec_global(v.R, vw, vz, nS);
    }
    __syncthreads();
    if (v.r_lds)
        cols_matvec_lds(v.R, vz, vx, nS, 1.0);
    else
        for (int k = tid; k < nS; k += NT) vx[k] = col_dot(v, vz, k, nS);
    __syncthreads();
}

// g_u = c_u - G_uS x_S for the slots u < nI (all of them, or only those outside S
// that may still enter it).  A row of 16 lanes takes two slots at a time and splits their support
// entries (G is global, so a slot costs one round trip with its loads in flight rather than a chain of
// |S| / 8), then sums each row by DPP moves inside the row.  (Reading the rows contiguously over all
// slots of I against x by slot was measured slower on large active sets: |I| / |S| times the entries.)
// DEPTH support entries per lane and slot are in flight at once (8 in the kernel without a register cap).
template <int DEPTH>
__device__ void grad_slots(const Sig& v, int nI, int nS, double* vg, bool outside_only)
{
    constexpr int GL = 16, NG = NT / GL;
    const int sub = threadIdx.x & (GL - 1), grp = threadIdx.x / GL;
    for (int u0 = grp; u0 < nI; u0 += 2 * NG) {
        const int u1 = u0 + NG;
        const bool d0 = !(outside_only && (v.th[u0] != 0 || v.ex[u0]));
        const bool d1 = u1 < nI && !(outside_only && (v.th[u1] != 0 || v.ex[u1]));
        if (!d0 && !d1) continue;       // the same decision for the whole row of lanes
        const double* G0 = v.G + (int64_t)u0 * v.K;
        const double* G1 = v.G + (int64_t)(d1 ? u1 : u0) * v.K;
        double a0 = 0.0, a1 = 0.0;
        for (int k0 = sub; k0 < nS; k0 += GL * DEPTH) {
            double g0[DEPTH], g1[DEPTH], xv[DEPTH];
            // clamped positions: every load is issued (a guarded one would wait at its branch's end);
            // positions past nS count zero through xv
#pragma unroll
            for (int e = 0; e < DEPTH; ++e) {
                const int k = k0 + GL * e;
                const int sk = v.so[k < nS ? k : nS - 1];
                g0[e] = G0[sk];
                g1[e] = G1[sk];
                xv[e] = v.x[sk];
            }
#pragma unroll
            for (int e = 0; e < DEPTH; ++e) {
                const bool in = k0 + GL * e < nS;
                g0[e] = in && d0 ? g0[e] : 0.0;
                g1[e] = in && d1 ? g1[e] : 0.0;
                xv[e] = in ? xv[e] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < DEPTH; ++e) {
                a0 += g0[e] * xv[e];
                a1 += g1[e] * xv[e];
            }
        }
        a0 = row16_sum(a0);
        a1 = row16_sum(a1);
        if (sub == 0) {
            if (d0) vg[u0] = v.c[u0] - a0;
            if (d1) vg[u1] = v.c[u1] - a1;
        }
    }
    __syncthreads();
}

// Element i of a global array that a generic pointer (the same in every thread) points into.
template <class T>
__device__ __forceinline__ T gld(const T* p, int64_t i)
{
    typedef __attribute__((address_space(1))) const T gT;
    return reinterpret_cast<gT*>(const_cast<gT*>(reinterpret_cast<gT*>(to_global(reinterpret_cast<const double*>(p)))))[i];
}
template <class T>
__device__ __forceinline__ void gst(T* p, int64_t i, T x)
{
    typedef __attribute__((address_space(1))) T gT;
    reinterpret_cast<gT*>(to_global(reinterpret_cast<double*>(p)))[i] = x;
}

// grad_slots for the fold kernel with the per-slot vectors in global memory (|S| <= GF_MS NT,
// |I| <= GF_MU NT): the same gradients, organised around the dependent gather G(u, so[k]).  Every
// thread reads the slot and coefficient of its support positions (tid + NT m) once; the slots that
// need a gradient are listed in slot order (list: nI ints of global scratch, written through wave
// ballots); the list is taken GF_B slots at a time: one round trip gathers every thread's entries of
// those rows (the next batch's slot numbers already in flight), the partial sums meet in LDS
// (double-buffered, added in wave order) and thread i writes slot i's gradient.  grad_slots takes a
// slot's support entries 16 lanes at a time, a slot-number load and then the gathers for every 64
// entries, so its round trips grow with |S|.  Ends with a barrier.
constexpr int GF_MS = 4, GF_MU = 8, GF_B = 4;

__device__ void grad_fold(const Sig& v, int nI, int nS, double* vg, bool outside_only, int* list)
{
    __shared__ double part[2][NT / 64][GF_B];
    __shared__ int wcnt[NT / 64][GF_MU];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    nI = __builtin_amdgcn_readfirstlane(nI);
    nS = __builtin_amdgcn_readfirstlane(nS);
    if (nI == 0) {
        __syncthreads();
        return;
    }
    global_cdouble* G = to_global(v.G);
    const int64_t K = v.K;
    // this thread's support positions: slot and coefficient (zero past nS)
    int sk[GF_MS];
    double xs[GF_MS];
#pragma unroll
    for (int m = 0; m < GF_MS; ++m) {
        const int k = tid + NT * m;
        sk[m] = nS > 0 ? gld(v.so, k < nS ? k : nS - 1) : 0;
    }
#pragma unroll
    for (int m = 0; m < GF_MS; ++m) xs[m] = gld(v.x, sk[m]);
#pragma unroll
    for (int m = 0; m < GF_MS; ++m) xs[m] = tid + NT * m < nS ? xs[m] : 0.0;
    // the slots that need a gradient, listed in the order (m, wave, lane) = slot order
    unsigned need = 0;
#pragma unroll
    for (int m = 0; m < GF_MU; ++m) {
        const int u = tid + NT * m;
        const int uc = u < nI ? u : nI - 1;
        const signed char th = gld(v.th, uc);
        const unsigned char ex = gld(v.ex, uc);
        need |= (u < nI && (!outside_only || (th == 0 && !ex))) ? 1u << m : 0u;
    }
    unsigned long long bal[GF_MU];
#pragma unroll
    for (int m = 0; m < GF_MU; ++m) bal[m] = __ballot((need >> m) & 1);
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < GF_MU; ++m) wcnt[wave][m] = __popcll(bal[m]);
    }
    __syncthreads();
    int ncand = 0;
#pragma unroll
    for (int m = 0; m < GF_MU; ++m) {
        int off = ncand;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            off += w < wave ? wcnt[w][m] : 0;
            ncand += wcnt[w][m];
        }
        if ((need >> m) & 1) {
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(bal[m] >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)bal[m], 0));
            gst(list, off + rank, tid + NT * m);
        }
    }
    ncand = __builtin_amdgcn_readfirstlane(ncand);
    __syncthreads();
    int nx[GF_B];
#pragma unroll
    for (int i = 0; i < GF_B; ++i) nx[i] = gld(list, i < ncand ? i : ncand - 1);
    int buf = 0;
    for (int b = 0; b < ncand; b += GF_B) {
        int us[GF_B];
#pragma unroll
        for (int i = 0; i < GF_B; ++i) us[i] = __builtin_amdgcn_readfirstlane(nx[i]);
#pragma unroll
        for (int i = 0; i < GF_B; ++i) {
            const int e = b + GF_B + i;
            nx[i] = gld(list, e < ncand ? e : ncand - 1);
        }
        double cu[GF_B], gv[GF_B][GF_MS];
#pragma unroll
        for (int i = 0; i < GF_B; ++i) {
            cu[i] = gld(v.c, us[i]);
            global_cdouble* Gu = G + us[i] * K;
#pragma unroll
            for (int m = 0; m < GF_MS; ++m) gv[i][m] = Gu[sk[m]];
        }
        double pq[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < GF_B; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < GF_MS; ++m) acc += gv[i][m] * xs[m];
            pq[i] = acc;
        }
        const double mine = wave_sum8(pq);       // lane l holds the wave's sum for slot wave_sum8_index(l)
        if (lane < 8 && wave_sum8_index(lane) < GF_B) part[buf][wave][wave_sum8_index(lane)] = mine;
        __syncthreads();
        if (tid < GF_B && b + tid < ncand) {
            int u = us[0];
            double c = cu[0];
#pragma unroll
            for (int i = 1; i < GF_B; ++i) {
                u = tid == i ? us[i] : u;
                c = tid == i ? cu[i] : c;
            }
            const double sum = ((part[buf][0][tid] + part[buf][1][tid]) + part[buf][2][tid]) + part[buf][3][tid];
            gst(vg, u, c - sum);
        }
        buf ^= 1;
    }
    __syncthreads();
}

// Gram rows G(q, u) of the new slots q against every slot u, and c_q = a_q^T b,
// as n-long float64 dot products (used when no Gram table is available).  The
// new atoms are staged through LDS in chunks (s_new: CH x NB doubles of the launch's dynamic
// LDS, present only when there is no table); each thread owns one slot u.
static_assert(CH * NB * 8 == GRAM_STAGE_BYTES, "direct Gram staging size");
__device__ void gram_rows_direct(const SolveArgs& a, Sig& s, const int* g_atom, const float* bw, int nI0,
                                 int nnew, int nI, double* s_new)
{
    const int tid = threadIdx.x;
    const int kpad = a.w.kpad;
    const int K = s.K;
    for (int g0 = 0; g0 < nnew; g0 += NB) {
        const int nb = nnew - g0 < NB ? nnew - g0 : NB;
        for (int ub = 0; ub <= nI; ub += NT) {
            const int u = ub + tid;
            const bool live = u <= nI;
            const float* col = (u < nI) ? a.At + (int64_t)g_atom[u] * a.lda : bw;
            double acc[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) acc[t] = 0.0;
            for (int kc = 0; kc < kpad; kc += CH) {
                __syncthreads();
                for (int e = tid; e < nb * CH; e += NT) {
                    const int t = e / CH, kk = e % CH;
                    const int atom = g_atom[nI0 + g0 + t];
                    s_new[kk * NB + t] = (kc + kk < kpad) ? (double)a.At[(int64_t)atom * a.lda + kc + kk] : 0.0;
                }
                __syncthreads();
                if (live) {
                    const int kend = (kpad - kc) < CH ? (kpad - kc) : CH;
                    for (int kk = 0; kk < kend; kk += 4) {
                        const float4 f = *reinterpret_cast<const float4*>(col + kc + kk);
                        const double fv[4] = {(double)f.x, (double)f.y, (double)f.z, (double)f.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const double* sn = s_new + (kk + e) * NB;
#pragma unroll
                            for (int t = 0; t < NB; ++t)
                                if (t < nb) acc[t] += fv[e] * sn[t];
                        }
                    }
                }
            }
            if (live) {
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    if (t >= nb) break;
                    const int q = nI0 + g0 + t;
                    if (u == nI) {
                        s.c[q] = acc[t];
                    } else {
                        s.G[(int64_t)q * K + u] = acc[t];
                        s.G[(int64_t)u * K + q] = acc[t];
                    }
                }
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Set-up: copy b_i into the padded signal and residual buffers, ||b_i||^2,
// finiteness, lambda (absolute rule), and clear the per-signal state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a)
{
    const int sig = blockIdx.x;
    const Workspace& w = a.w;
    __shared__ double red[4];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const float* b = a.B + (int64_t)sig * a.ldb;
    float* Bw = a.Bw + (int64_t)sig * w.kpad;
    float* R = w.R + (int64_t)sig * w.kpad;
    double part = 0.0, dpart = 0.0;
    int bad = 0;
    for (int r = threadIdx.x; r < w.kpad; r += 256) {
        float v = r < w.n ? b[r] : 0.f;
        if (!isfinite(v)) bad = 1;
        Bw[r] = v;
        R[r] = v;
        if (w.R16) {
            const uint16_t h = bf16_round(v);
            w.R16[(int64_t)sig * w.kpad + r] = h;
            const double d = (double)bf16_value(h) - (double)v;
            dpart += d * d;
        }
        part += (double)v * (double)v;
    }
    if (bad) atomicOr(&s_bad, 1);
    for (int q = threadIdx.x; q < w.words; q += 256) w.inI[(int64_t)sig * w.words + q] = 0u;
    const double bb = block_sum(part, red);
    const double bd = w.R16 ? block_sum(dpart, red) : 0.0;
    if (threadIdx.x == 0) {
        double lam = a.lambda_dev ? a.lambda_dev[sig] : a.lambda_abs;
        int st = 0;
        if (s_bad || !isfinite(lam) || lam < 0.0) st = BMPL_SIG_NONFINITE;
        w.status[sig] = st;
        w.lam[sig] = a.lam_rel_mode ? 0.0 : lam;
        w.bnorm2[sig] = bb;
        w.iters[sig] = 0;
        w.nI[sig] = 0;
        w.nS[sig] = 0;
        w.nsel[sig] = 0;
        w.glazy[sig] = 0;
        w.jadd[sig] = JADD0;
        w.vmax[sig] = 0.f;
        w.kkt_on[sig] = 0.0;
        w.kkt[sig] = 0.0;
        w.obj[sig] = 0.5 * bb;
        w.obj_prev[sig] = 0.5 * bb;
        w.rr2[sig] = bb;
        w.g0max[sig] = 0.f;
        w.cap[sig] = 0;
        w.blk[sig] = nullptr;
        if (sig == 0) {   // a new solve hands out slot blocks from the start of the arena
            w.arena->top = 0;
            w.arena->starved = 0;
        }
        if (w.rnorm) w.rnorm[sig] = sqrt(bb);
        if (w.dxnorm) w.dxnorm[sig] = sqrt(bd);
    }
    if (w.R8) write_residual_fp8(w, sig, red);
}

// ---------------------------------------------------------------------------
// Stop test and compaction.  For each running signal after a selection pass:
// no violator left -> natural stop; an early-stop rule (Eq. (10), Eq. (13))
// holds -> early stop; no admitted atom -> the active-set cap was hit;
// iteration cap -> stop; otherwise keep it running.
// One workgroup; the running list stays in signal order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void status_compact_kernel(StatusArgs a)
{
    const Workspace& w = a.w;
    const int n_in = a.n_in_dev ? *a.n_in_dev : a.n_in;
    __shared__ int s_scan[1024];
    __shared__ int s_base;
    __shared__ unsigned long long s_res[16];
    __shared__ int s_ng;
    __shared__ unsigned long long s_goff;   // doubles of the grow list's new blocks
    __shared__ int s_maxb;                  // largest support bucket (256 positions each) among kept signals
    if (threadIdx.x == 0) { s_base = 0; s_ng = 0; s_goff = 0; s_maxb = 0; }
    __syncthreads();
    unsigned long long res = 0;   // this thread's share of the slot-block reserve
    int mbk = 0;                  // largest support bucket among this thread's kept signals
    for (int r0 = 0; r0 < n_in; r0 += 1024) {
        const int r = r0 + threadIdx.x;
        int keep = 0, sig = -1;
        if (r < n_in) {
            sig = a.act_in ? a.act_in[r] : r;
            int st = w.status[sig];
            if (a.initial) {
                keep = !(st & BMPL_SIG_NONFINITE);
            } else {
                const double lam = w.lam[sig];
                const int ns = w.nsel[sig];
                const double vm = (double)w.vmax[sig];
                const int it = w.iters[sig];
                if (it == 0) w.g0max[sig] = w.vmax[sig];   // first pass: I is empty, so this is ||A^T b||_inf
                const bool natural = ns == 0 && vm <= lam;
                bool early = false;
                if (!natural) {
                    const double bb = w.bnorm2[sig];
                    if (a.r_inf_rel > 0.0 && vm <= a.r_inf_rel * (double)w.g0max[sig])
                        early = true;                                             // Eq. (10), correlations
                    else if (a.r2_rel > 0.0 && sqrt(w.rr2[sig]) <= a.r2_rel * sqrt(bb))
                        early = true;                                             // Eq. (10), residual norm
                    else if (a.eps_early > 0.0 && it >= 1 &&
                             fabs(w.obj_prev[sig] - w.obj[sig]) <= a.eps_early * a.rho * bb)
                        early = true;                                             // Eq. (13)
                }
                const bool halt = (st & ST_HALT) != 0;   // the solve kernel stopped it (reported inexact)
                st &= ~ST_HALT;
                if (ns == 0 || it >= a.max_outer || early || halt) {
                    double off = vm - lam;
                    off = off > 0.0 ? off : 0.0;
                    double kk = fmax(off, w.kkt_on[sig]);
                    kk = lam > 0.0 ? kk / lam : kk;
                    w.kkt[sig] = kk;
                    if (a.warm_check && ns != 0) st |= BMPL_SIG_FALLBACK;
                    if (halt) {
                        // INEXACT is set already
                    } else if (natural) {
                        if (kk <= a.kkt_tol) st |= BMPL_SIG_CONVERGED;
                    } else if (early) {
                        st |= BMPL_SIG_EARLY;
                    } else if (ns == 0) {
                        if (!(st & BMPL_SIG_INEXACT)) st |= BMPL_SIG_CAP_ACTIVE;
                    } else {
                        st |= BMPL_SIG_CAP_ITERS;
                    }
                    w.status[sig] = st;
                    if (ns != 0) w.nsel[sig] = 0;
                } else {
                    if (a.warm_check) w.status[sig] = st | BMPL_SIG_FALLBACK;
                    keep = 1;
                }
            }
        }
        if (keep) mbk = max(mbk, min(3, w.nS[sig] / 256));
        if (keep && a.grow_list && w.nI[sig] + w.nsel[sig] > w.cap[sig]) {
            // its block grows before the master problem; the new blocks of the whole list are placed here
            // with one fetch-and-add on the arena's offset (below), each at its share of the total
            const int K2 = max(grow_capacity(w.cap[sig], w.nI[sig] + w.nsel[sig], a.slack, a.kcap),
                               min(a.kmin, a.kcap));
            const int e = atomicAdd(&s_ng, 1);
            a.grow_list[e] = sig;
            a.grow_off[e] = atomicAdd(&s_goff, (unsigned long long)block_doubles(K2, w.n));
        }
        if (keep && a.reserve_iters > 0) {
            // the blocks this signal may take while its |I| grows by up to reserve_iters * rho_pass slots
            int Kc = w.cap[sig];
            const int target = min(a.kcap, w.nI[sig] + a.reserve_iters * a.rho_pass);
            while (Kc < target) {
                Kc = grow_capacity(Kc, min(target, Kc + a.rho_pass), a.slack, a.kcap);
                res += (unsigned long long)block_doubles(Kc, w.n);
            }
        }
        // order-preserving compaction: position = kept signals before this one in the round (a ballot
        // within the wave, the counts of the earlier waves from LDS), two barriers per round
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) s_scan[wv] = __popcll(bal);
        __syncthreads();
        int before = s_base, total = 0;
        for (int q = 0; q < 16; ++q) {
            const int c = s_scan[q];
            before += q < wv ? c : 0;
            total += c;
        }
        if (keep) a.act_out[before + __popcll(bal & ((1ull << lane) - 1ull))] = sig;
        __syncthreads();   // every wave has read s_scan and s_base
        if (threadIdx.x == 0) s_base += total;
    }
    if (mbk > 0) atomicMax(&s_maxb, mbk);
    __syncthreads();
    {
        // The running list, largest supports first (buckets of 256 support positions, kept in signal
        // order within a bucket): the master problem's workgroups start with the longest problems and
        // the short ones fill the end of the launch.  Only when some support has 256 positions or more,
        // and for lists of at most 16 entries per thread (longer lists keep their order).
        constexpr int RMAX = 16;
        const int n = s_base;
        const bool reorder = !a.initial && s_maxb > 0 && n <= RMAX * 1024;   // the same in every thread
        int v[RMAX], bk[RMAX];
        if (reorder) {
#pragma unroll
            for (int j = 0; j < RMAX; ++j) {
                const int r = threadIdx.x + 1024 * j;
                v[j] = r < n ? a.act_out[r] : -1;
                bk[j] = v[j] >= 0 ? min(3, w.nS[v[j]] / 256) : -1;
            }
            __syncthreads();                  // every entry is read before any is rewritten
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            int base = 0;
            for (int b = 3; b >= 0; --b) {
#pragma unroll
                for (int j = 0; j < RMAX; ++j) {
                    if (1024 * j >= n) break;  // the same in every thread
                    const bool in = bk[j] == b;
                    const unsigned long long bal = __ballot(in);
                    if (lane == 0) s_scan[wv] = __popcll(bal);
                    __syncthreads();
                    int before = base, total = 0;
                    for (int q = 0; q < 16; ++q) {
                        const int c = s_scan[q];
                        before += q < wv ? c : 0;
                        total += c;
                    }
                    if (in) a.act_out[before + __popcll(bal & ((1ull << lane) - 1ull))] = v[j];
                    __syncthreads();           // every wave has read s_scan
                    base += total;
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        *a.n_out_dev = s_base;
        if (a.n_grow) *a.n_grow = s_ng;
        if (s_ng > 0) w.arena->grow_base = atomicAdd(&w.arena->top, s_goff);
        if (a.clear_cert) *a.clear_cert = 0;   // this pass's certification list is consumed
    }
    if (a.reserve_iters > 0) {
        for (int o = 32; o > 0; o >>= 1) res += __shfl_xor(res, o);
        if ((threadIdx.x & 63) == 0) s_res[threadIdx.x >> 6] = res;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int q = 0; q < 16; ++q) t += s_res[q];
            w.arena->reserve = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Warm start: replace this pass's selection with the proposed atoms.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void warm_select_kernel(WarmArgs a)
{
    __shared__ int s_w[256];
    __shared__ int s_cnt[4];
    const int n_act = *a.n_act_dev;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act[row];
    const Workspace& w = a.w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int cap = a.max_active < w.selcap ? a.max_active : w.selcap;
    cap = cap < 256 ? cap : 256;
    // proposal entry tid: valid atom, first occurrence in the list
    const int j = tid < a.warm_k ? a.warm[(int64_t)sig * a.warm_k + tid] : -1;
    s_w[tid] = j;
    __syncthreads();
    bool keep = j >= 0 && j < w.m;
    for (int t = 0; t < tid && keep; ++t) keep = s_w[t] != j;
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) s_cnt[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w2 = 0; w2 < wave; ++w2) before += s_cnt[w2];
    const int total = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    const int pos = before + __popcll(bal & ((1ull << lane) - 1ull));
    // an empty proposal keeps this pass's own selection
    if (total > 0) {
        if (keep && pos < cap) w.sel[(int64_t)sig * w.selcap + pos] = j;
        if (tid == 0) w.nsel[sig] = total < cap ? total : cap;
    }
}

// ---------------------------------------------------------------------------
// Slot-block growth: a running signal whose active set, with this pass's selection, outgrows its block
// takes a larger one from the arena (grow_capacity) and copies its state over: slots, support order,
// the inverse factor and the Gram matrix of I (restrided).  A request that finds no room is counted in
// the arena's `starved` and leaves the signal as it is (the master-problem kernel then skips it).
// ---------------------------------------------------------------------------
// The stop test lists the signals that need it and places their new blocks with one fetch-and-add
// (one per listed signal on that single address kept the first master problem of 16 384 signals
// waiting half a millisecond); a block that would straddle two chunks is requested again on its own.
// A grid of at most a few hundred workgroups loops over the list.
__global__ __launch_bounds__(256) void grow_kernel(GrowArgs a)
{
    const int n_list = *a.n_list;
    const Workspace& w = a.w;
    const int tid = threadIdx.x;
    __shared__ double* s_blk;
    for (int li = blockIdx.x; li < n_list; li += gridDim.x) {
        const int sig = a.list[li];
        const int nI0 = w.nI[sig], nS = w.nS[sig];
        const int nI = nI0 + w.nsel[sig];
        const int K = w.cap[sig];
        const int K2 = max(grow_capacity(K, nI, a.slack, a.kcap), min(a.kmin, a.kcap));
        if (tid == 0) {
            const unsigned long long sz = (unsigned long long)block_doubles(K2, w.n);
            const Arena& A = *w.arena;
            const unsigned long long off = A.grow_base + a.off[li];
            int c = 0;
            while (c < A.nchunks && off >= A.start[c] + A.size[c]) ++c;
            double* p = nullptr;
            if (c < A.nchunks && off + sz <= A.start[c] + A.size[c]) p = A.base[c] + (off - A.start[c]);
            else p = arena_alloc(w.arena, sz);   // straddles a chunk boundary, or past the last chunk
            if (!p) atomicAdd(&w.arena->starved, 1ull);
            s_blk = p;
        }
        __syncthreads();
        double* nb = s_blk;
        __syncthreads();   // s_blk is rewritten for the next signal
        if (!nb) continue;
        if (K > 0) {
            const SlotBlock o = slot_block(w.blk[sig], K, w.n), d = slot_block(nb, K2, w.n);
            for (int u = tid; u < nI0; u += 256) {
                d.x[u] = o.x[u]; d.c[u] = o.c[u]; d.atom[u] = o.atom[u]; d.theta[u] = o.theta[u];
                d.excl[u] = o.excl[u];
            }
            for (int k = tid; k < nS; k += 256) d.sord[k] = o.sord[k];
            const int tr = (int)tri(nS), tot = nI0 * nI0;
            for (int e0 = tid; e0 < tr; e0 += 8 * 256) {   // eight loads in flight per thread
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = o.Rinv[e0 + q * 256 < tr ? e0 + q * 256 : tr - 1];   // clamped
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (e0 + q * 256 < tr) d.Rinv[e0 + q * 256] = v[q];
            }
            for (int e0 = tid; e0 < tot; e0 += 8 * 256) {   // G restrided from K to K2
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {   // clamped, so all eight loads are issued
                    const int e = e0 + q * 256 < tot ? e0 + q * 256 : tot - 1, u = e / nI0;
                    v[q] = o.G[(int64_t)u * K + (e - u * nI0)];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int e = e0 + q * 256, u = e / nI0;
                    if (e < tot) d.G[(int64_t)u * K2 + (e - u * nI0)] = v[q];
                }
            }
        }
        if (tid == 0) {
            w.blk[sig] = nb;
            w.cap[sig] = K2;
        }
    }
}

// ---------------------------------------------------------------------------
// Master problem on I for every running signal, then its residual and objective.
//
// Working set: the inverse factor Rinv and the per-slot vectors live in LDS
// when they fit (copied in at entry, written back at exit), otherwise they are
// used in place in global memory.  G_II (row-major, stride K) stays global.
// Two kernels share the body: with block appends (for a factor in global memory)
// and without them, whose register footprint is half as large, so twice as many
// workgroups fit on a CU.
// ---------------------------------------------------------------------------
// Residual xi = b - A_S x_S (float64 accumulation, stored float32) and the objective
// lambda ||x||_1 + 1/2 ||xi||^2 of a signal that was just solved (step 7 of Algorithm 1), with the
// norms and reduced-precision copies the next product and its screening band use.  Run by the solve
// workgroup after its write-back: sx / satom hold the support's values and atoms (LDS), xl1 = ||x||_1.
// Four rows per thread, eight atoms' loads in flight, straight from the atom-major dictionary; a
// workgroup that finishes its master problem early computes its residual while others still solve.
__device__ void residual_tail(const Workspace& w, int sig, const float* At, int64_t lda, const float* Bw,
                              const double* sx, const int* satom, int nS, double xl1, double* red)
{
    const int tid = threadIdx.x;
    const float* bw = Bw + (int64_t)sig * w.kpad;
    float* Rres = w.R + (int64_t)sig * w.kpad;
    double rr = 0.0, dr = 0.0;
    // rows 4 q .. 4 q + 3 per step (kpad and lda are multiples of 4)
    const int n4 = w.kpad / 4;
    const int64_t lda4 = lda / 4;
    const float4* At4 = reinterpret_cast<const float4*>(At);
    constexpr int CH = 8;
    for (int q = tid; q < n4; q += NT) {
        const float4 bv = reinterpret_cast<const float4*>(bw)[q];
        double acc[4] = {(double)bv.x, (double)bv.y, (double)bv.z, (double)bv.w};
        int k = 0;
        for (; k + CH <= nS; k += CH) {
            float4 f[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) f[e] = At4[(int64_t)satom[k + e] * lda4 + q];
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const double xv = sx[k + e];
                acc[0] -= (double)f[e].x * xv;
                acc[1] -= (double)f[e].y * xv;
                acc[2] -= (double)f[e].z * xv;
                acc[3] -= (double)f[e].w * xv;
            }
        }
        for (; k < nS; ++k) {
            const float4 f = At4[(int64_t)satom[k] * lda4 + q];
            const double xv = sx[k];
            acc[0] -= (double)f.x * xv;
            acc[1] -= (double)f.y * xv;
            acc[2] -= (double)f.z * xv;
            acc[3] -= (double)f.w * xv;
        }
        float4 out;
        float* o = reinterpret_cast<float*>(&out);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 4 * q + e;
            if (r >= w.n) acc[e] = 0.0;
            o[e] = (float)acc[e];
            if (w.R16) {
                const uint16_t h = bf16_round(o[e]);
                w.R16[(int64_t)sig * w.kpad + r] = h;
                const double d = (double)bf16_value(h) - (double)o[e];
                dr += d * d;
            }
            rr += acc[e] * acc[e];
        }
        reinterpret_cast<float4*>(Rres)[q] = out;
    }
    const double rn = block_sum(rr, red);
    const double rd = w.R16 ? block_sum(dr, red) : 0.0;
    if (tid == 0) {
        w.obj_prev[sig] = w.obj[sig];
        w.obj[sig] = 0.5 * rn + w.lam[sig] * xl1;
        w.rr2[sig] = rn;
        if (w.rnorm) w.rnorm[sig] = sqrt(rn);
        if (w.dxnorm) w.dxnorm[sig] = sqrt(rd);
    }
    if (w.R8) write_residual_fp8(w, sig, red);
}

template <bool BLOCK, bool FOLD>
__device__ __forceinline__ void solve_body(const SolveArgs& a)
{
    extern __shared__ double s_dyn[];
    __shared__ double red[4];
    __shared__ int redi[4];
    __shared__ int s_list[NT];
    __shared__ int s_cnt;

    const int n_act = *a.n_act_dev;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const Workspace& w = a.w;
    const int sig = a.act[row];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nnew = w.nsel[sig];
    if (nnew <= 0) return;
    const int nI0 = w.nI[sig];
    int nS = w.nS[sig];
    const double lam = w.lam[sig];
    int nI = nI0 + nnew;
    if (a.vec_lds && nI > a.kv) {
        // the launch was sized for a smaller |I| (a host-side bound that does not hold): stop the signal
        // at its current iterate, reported inexact, rather than overrun the LDS vectors
        if (tid == 0) w.status[sig] |= BMPL_SIG_INEXACT | ST_HALT;
        return;
    }

    // The signal's slot block (grown by grow_kernel before this launch); a block that could not grow
    // (no arena room) leaves the signal untouched: the host adds room and the next outer iteration
    // selects the same atoms again.
    const int K = w.cap[sig];
    if (nI > K) return;
    double* base = w.blk[sig];
    const SlotBlock hb = slot_block(base, K, w.n);
    const int max_steps = a.max_steps_per_slot * K + 256;
    uint64_t tick = a.phase ? wall_clock64() : 0;

    // global homes of this signal's state
    int* g_atom = hb.atom;
    double* g_x = hb.x;
    double* g_c = hb.c;
    signed char* g_th = hb.theta;
    unsigned char* g_ex = hb.excl;
    int* g_so = hb.sord;
    double* g_R = hb.Rinv;

    Sig s;
    s.K = K;
    // The LDS factor holds up to a.kl support positions; a signal whose support outgrows it moves its
    // factor to the global home and continues there (spill_factor below).
    s.r_lds = a.rinv_lds != 0 && nS <= a.kl;
    s.G = hb.G;
    char* lp = reinterpret_cast<char*>(s_dyn);
    if (a.rinv_lds) {
        s.R = s.r_lds ? reinterpret_cast<double*>(lp) : g_R;
        lp += sizeof(double) * tri(a.kl);
    } else {
        s.R = g_R;
    }
    double *vw, *vz, *vx, *vg;
    double* vzc;   // cached z = Rinv w of the sign-fixed solve, by position (x* is in vx)
    int* vatom;
    const int KV = a.kv;                      // LDS vectors by slot: KV >= |I| during this launch
    const int KP = a.kp;                      // by support position: |S| <= min(|I|, n) <= KP
    if (a.vec_lds) {
        double* d = reinterpret_cast<double*>(lp);
        s.x = d; s.c = d + KV; vg = d + 2 * KV;
        vw = d + 3 * KV; vz = vw + KP; vx = vz + KP; vzc = vx + KP;
        int* ip = reinterpret_cast<int*>(vzc + KP);
        s.so = ip; vatom = ip + KP;
        s.th = reinterpret_cast<signed char*>(vatom + KV);
        s.ex = reinterpret_cast<unsigned char*>(s.th + KV);
    } else {
        double* d = hb.vs;
        s.x = g_x; s.c = g_c; s.th = g_th; s.ex = g_ex; s.so = g_so;
        vw = d; vz = d + K; vx = d + 2 * K; vg = d + 3 * K;
        vatom = reinterpret_cast<int*>(d + 4 * K);
        vzc = d + 5 * K;
    }
    // the gradients' slot list (grad_fold), in the unused end of the global vector scratch
    int* glist = a.vec_lds ? nullptr : reinterpret_cast<int*>(hb.vs + 6 * (int64_t)K);
    // block-append scratch after the vectors (K rows of JB doubles), when the launch provided it
    double* zs = (BLOCK && a.zs_lds) ? reinterpret_cast<double*>(lp + (a.vec_lds ? vec_area_bytes(KV, KP) : 0)) : nullptr;
    // direct Gram staging (no table) after the vectors and the block scratch
    double* snew = a.Q ? nullptr
                       : reinterpret_cast<double*>(lp + (a.vec_lds ? vec_area_bytes(KV, KP) : 0) +
                                                   (a.zs_lds ? block_scratch_bytes(KP) : 0));

    // 1. Load the state, register the new slots.
    if (a.vec_lds) {
        for (int u = tid; u < nI0; u += NT) {
            s.x[u] = g_x[u]; s.c[u] = g_c[u]; s.th[u] = g_th[u]; s.ex[u] = g_ex[u];
        }
        for (int k = tid; k < nS; k += NT) s.so[k] = g_so[k];
    }
    if (s.r_lds) {   // eight loads in flight per thread
        const int64_t T = tri(nS);
        for (int64_t e0 = tid; e0 < T; e0 += 8 * NT) {
            double r[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = g_R[e0 + q * NT < T ? e0 + q * NT : T - 1];   // clamped
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (e0 + q * NT < T) s.R[e0 + q * NT] = r[q];
        }
    }
    for (int u = tid; u < nI0; u += NT) vatom[u] = g_atom[u];
    for (int t = tid; t < nnew; t += NT) {
        const int q = nI0 + t;
        const int atom = w.sel[(int64_t)sig * w.selcap + t];
        g_atom[q] = atom;
        vatom[q] = atom;
        s.x[q] = 0.0;
        s.th[q] = 0;
        s.ex[q] = 0;
        atomicOr(&w.inI[(int64_t)sig * w.words + (atom >> 5)], 1u << (atom & 31));
    }
    __syncthreads();

    // Optional per-phase wall-clock ticks (kernel timing mode): load, Gram, active set,
    // certificate, (appends), write-back; the residual's ticks go to slot 14.
    auto phase_mark = [&](int ph) {
        if (a.phase && tid == 0) {
            const uint64_t now = wall_clock64();
            atomicAdd(reinterpret_cast<unsigned long long*>(a.phase + ph), (unsigned long long)(now - tick));
            tick = now;
        }
    };
    phase_mark(0);
    // time spent in one call of a step of the active-set loop, summed into phase slot `slot`
    auto sub_ticks = [&](int slot, uint64_t t0) {
        if (a.phase && tid == 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(a.phase + slot), (unsigned long long)(wall_clock64() - t0));
    };

    // 2. Gram rows of the new slots and c = A_J^T b, in float64.  With many new slots (a warm start)
    //    the Gram matrix is kept lazily from then on: a new slot's row only against the support
    //    members and itself, and a slot's whole column when it enters S (gather_cols below), which is
    //    every entry the solver reads.  Most proposed slots never enter S.
    const float* bw = a.Bw + (int64_t)sig * w.kpad;
    const bool lazy = a.Q && (w.glazy[sig] != 0 || nnew > LAZY_MIN);
    if (a.Q && lazy) {
        if (tid == 0) w.glazy[sig] = 1;
        const int span = nS + 1;                  // support positions, then the diagonal
        const int tot = nnew * span;
        for (int e0 = tid; e0 < tot; e0 += 4 * NT) {
            double val[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {   // clamped entry index: all four reads issued together
                const int e = e0 + r * NT < tot ? e0 + r * NT : tot - 1;
                const int t = e / span, k = e - t * span;
                const int u = k < nS ? s.so[k] : nI0 + t;
                val[r] = a.Q[(int64_t)vatom[nI0 + t] * a.ldq + vatom[u]];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = e0 + r * NT;
                if (e < tot) {
                    const int t = e / span, k = e - t * span;
                    const int q = nI0 + t;
                    const int u = k < nS ? s.so[k] : q;
                    s.G[(int64_t)q * K + u] = val[r];
                    s.G[(int64_t)u * K + q] = val[r];
                }
            }
        }
    } else if (a.Q) {
        // four table reads per thread in flight before the symmetric stores
        const int tot = nnew * nI;
        for (int e0 = tid; e0 < tot; e0 += 4 * NT) {
            double val[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {   // clamped entry index: all four reads issued together
                const int e = e0 + r * NT < tot ? e0 + r * NT : tot - 1;
                const int t = e / nI, u = e - t * nI;
                val[r] = a.Q[(int64_t)vatom[nI0 + t] * a.ldq + vatom[u]];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = e0 + r * NT;
                if (e < tot) {
                    const int t = e / nI, u = e - t * nI;
                    const int q = nI0 + t;
                    s.G[(int64_t)q * K + u] = val[r];
                    s.G[(int64_t)u * K + q] = val[r];
                }
            }
        }
    }
    if (a.Q) {
        // c_q = a_q^T b: one wave per new atom, float4 loads, all issued before the sums
        for (int t = wave; t < nnew; t += NT / 64) {
            const float4* aj = reinterpret_cast<const float4*>(a.At + (int64_t)vatom[nI0 + t] * a.lda);
            const float4* b4 = reinterpret_cast<const float4*>(bw);
            double acc = 0.0;
            const int n4 = w.kpad / 4;
            for (int k0 = lane; k0 < n4; k0 += 64 * 4) {
                float4 fa[4], fb[4];
                // inside the vectors for the whole wave: no branch, so the eight loads are in flight together
                if (k0 - lane + 64 * 4 <= n4) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        fa[e] = aj[k0 + 64 * e];
                        fb[e] = b4[k0 + 64 * e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = k0 + 64 * e;
                        fa[e] = k < n4 ? aj[k] : make_float4(0.f, 0.f, 0.f, 0.f);
                        fb[e] = k < n4 ? b4[k] : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc += (double)fa[e].x * fb[e].x + (double)fa[e].y * fb[e].y + (double)fa[e].z * fb[e].z +
                           (double)fa[e].w * fb[e].w;
            }
            acc = wave_sum(acc);
            if (lane == 0) s.c[nI0 + t] = acc;
        }
    } else {
        gram_rows_direct(a, s, g_atom, bw, nI0, nnew, nI, snew);
    }
    __syncthreads();

    phase_mark(1);

    // 3. Sign-fixed active-set iterations (twice with subspace exploratory matching: on I u J_omega,
    //    then, after the pruning below, on I_t).
    int steps = 0;
    bool inexact = false;
    bool explored = false;
    bool resolve = false;   // after the pruning: solve on I_t even if no slot outside S violates
    // Violators admitted per step, adapted to the dictionary and carried from one outer iteration to
    // the next: doubled (up to JADD) after a step whose move to the sign-fixed minimiser dropped nothing;
    // on a small support (|S| < 128) halved after one that dropped at least a quarter as many atoms as it
    // admitted (correlated atoms that enter and leave together); otherwise trimmed by an eighth (by one
    // below 8): a large, nearly saturated support sees drops at almost every step, and each admission
    // saved there is a pass over a factor of hundreds of rows.
    int jadd = w.jadd[sig];
    jadd = jadd >= 1 && jadd <= JADD ? jadd : JADD0;
    // the sign-fixed minimiser x* (vx) and z = Rinv w (vzc) are computed in full once, then kept current
    // through appends (xstar_after_append) and drops (rotated z, and x* from the removed row)
    bool xs_ok = false;
    // the last pass of the loop computes the gradient on all of I for the certificate (one call site of
    // the gradient routine: each inlined copy costs the kernel registers)
    bool cert = false;
active_set:
    for (;;) {
        const uint64_t tg = a.phase ? wall_clock64() : 0;
        if (FOLD && glist && nI <= GF_MU * NT && nS <= GF_MS * NT) grad_fold(s, nI, nS, vg, !cert, glist);
        else grad_slots<BLOCK ? 8 : 4>(s, nI, nS, vg, !cert);
        sub_ticks(11, tg);
        if (cert) break;
        const uint64_t tv = a.phase ? wall_clock64() : 0;
        if (wave == 0) {    // violators outside S, in slot order
            int base = 0;
            for (int u0 = 0; u0 < nI && base < NT; u0 += 64) {
                const int u = u0 + lane;
                bool viol = false;
                if (u < nI && s.th[u] == 0 && !s.ex[u])
                    viol = fabs(vg[u]) > lam * (1.0 + 1e-12) && fabs(vg[u]) > 0.0;
                const unsigned long long bal = __ballot(viol);
                const int pre = __popcll(bal & ((1ull << lane) - 1ull));
                if (viol && base + pre < NT) s_list[base + pre] = u;
                base += __popcll(bal);
            }
            if (lane == 0) s_cnt = base < NT ? base : NT;
        }
        __syncthreads();
        int nv = s_cnt;
        if (nv == 0 && !resolve) {
            cert = true;
            continue;
        }
        resolve = false;
        if (nv > jadd) {
            // keep the jadd largest violations (ties to the lower slot), in slot order: adding a few at a
            // time keeps sign changes, and with them drops, rare when many atoms of I violate at once
            int u = -1, rank = 0;
            double gu = 0.0;
            if (tid < nv) {
                u = s_list[tid];
                gu = fabs(vg[u]);
                for (int e = 0; e < nv; ++e) {
                    const int o = s_list[e];
                    const double go = fabs(vg[o]);
                    rank += (go > gu) || (go == gu && o < u);
                }
            }
            __syncthreads();
            const bool keep = tid < nv && rank < jadd;
            // compact the kept slots in slot order (s_list is in slot order)
            const unsigned long long bal = __ballot(keep);
            if (lane == 0) redi[wave] = __popcll(bal);
            __syncthreads();
            int before = 0;
            for (int w2 = 0; w2 < wave; ++w2) before += redi[w2];
            if (keep) s_list[before + __popcll(bal & ((1ull << lane) - 1ull))] = u;
            __syncthreads();
            nv = jadd;
        }
        sub_ticks(12, tv);
        if (lazy && nv > 0) {
            // lazy Gram: the columns of the slots about to enter S, against every slot of I
            const int tot = nv * nI;
            for (int e0 = tid; e0 < tot; e0 += 4 * NT) {
                double val[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {   // clamped entry index: all four reads issued together
                    const int e = e0 + r * NT < tot ? e0 + r * NT : tot - 1;
                    const int t = e / nI, u2 = e - t * nI;
                    val[r] = a.Q[(int64_t)g_atom[s_list[t]] * a.ldq + g_atom[u2]];
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = e0 + r * NT;
                    if (e < tot) {
                        const int t = e / nI, u2 = e - t * nI;
                        const int j = s_list[t];
                        s.G[(int64_t)j * K + u2] = val[r];
                        s.G[(int64_t)u2 * K + j] = val[r];
                    }
                }
            }
            __syncthreads();
        }
        if (s.r_lds && nS + nv > a.kl) {
            // the support outgrows the LDS factor: move it to the global home and continue there
            for (int64_t e = tid; e < tri(nS); e += NT) g_R[e] = s.R[e];
            __syncthreads();
            s.R = g_R;
            s.r_lds = false;
        }
        const int nS_before = nS;
        if (nv == 0) {
            // nothing to append: the pruned problem on I_t is solved from u restricted to it
        } else if (zs) {
            append_list(s, nS, s_list, nv, vg, w.n, zs, a.phase ? a.phase + 6 : nullptr);
        } else {
            for (int e = 0; e < nv; ++e) {
                const int u = s_list[e];
                const signed char th = vg[u] > 0.0 ? 1 : -1;
                if (nS >= w.n) {
                    if (tid == 0) s.ex[u] = 1;
                    __syncthreads();
                    continue;
                }
                chol_append<FOLD>(s, nS, u, th, vw, vz, red, a.phase ? a.phase + 6 : nullptr);
            }
        }
        if (xs_ok && nS > nS_before) {
            const uint64_t tsf = a.phase ? wall_clock64() : 0;
            xstar_after_append(s, nS_before, nS, lam, vw, vzc, vx, red);
            sub_ticks(10, tsf);
        }
        const int added = nS - nS_before;
        // move toward the sign-fixed minimiser, dropping at zero crossings
        int dropped = 0;
        for (;;) {
            if (++steps > max_steps) { inexact = true; break; }
            if (!xs_ok) {
                const uint64_t tsf = a.phase ? wall_clock64() : 0;
                sign_fixed_solve<FOLD>(s, nS, lam, vw, vzc, vx);
                sub_ticks(10, tsf);
                xs_ok = true;
            }
            if (a.phase && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.phase + 8), 1ull);
            const uint64_t tr = a.phase ? wall_clock64() : 0;
            double alpha = 1.0;
            int q = -1;
            for (int k = tid; k < nS; k += NT) {
                const int u = s.so[k];
                const double xo = s.x[u], xn = vx[k], th = (double)s.th[u];
                if (xn * th <= 0.0) {
                    const double ak = (xo == 0.0) ? 0.0 : fmax(xo / (xo - xn), 0.0);
                    if (ak < alpha || (ak == alpha && (q < 0 || k < q))) { alpha = ak; q = k; }
                }
            }
            block_argmin(alpha, q, red, redi);
            for (int k = tid; k < nS; k += NT) {
                const int u = s.so[k];
                const double xo = s.x[u];
                s.x[u] = xo + alpha * (vx[k] - xo);
            }
            __syncthreads();
            sub_ticks(13, tr);
            if (q < 0) break;
            // the atom admitted alone blocks at alpha = 0: a numerically void admission (EX_PASS)
            const bool void_admit = alpha == 0.0 && dropped == 0 && nS == nS_before + 1 && q == nS_before;
            ++dropped;
            // drop position q: downdate the factor (or truncate it and append the later positions again)
            if (a.phase && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.phase + 7), 1ull);
            const int ns_old = nS;
            for (int k = tid; k < ns_old; k += NT) vatom[k] = s.so[k];
            __syncthreads();
            if (tid == 0) {
                const int u = vatom[q];
                s.x[u] = 0.0;
                s.th[u] = 0;
                if (void_admit) s.ex[u] = EX_PASS;
            }
            __syncthreads();
            // downdate the factor in place (vw is free scratch here); support positions past q move down
            const uint64_t td = a.phase ? wall_clock64() : 0;
            // the fold kernel's factors are in global memory; with its vectors there too (large supports)
            // the downdate keeps rows in flight across its barriers
            if (FOLD && ns_old <= 4 * NT && !is_lds(vzc)) chol_drop_global(s, ns_old, q, vw, vzc);
            else chol_drop<BLOCK ? 8 : 4>(s, ns_old, q, vw, vzc);
            // x* on S \ q: with the removed row b (vw) and its z entry zl, x*_new[k] = x*[k'] - b_k zl
            // (k' the position before the shift)
            {
                const double zl = vzc[ns_old - 1];
                for (int k = tid; k < ns_old - 1; k += NT) vz[k] = vx[k < q ? k : k + 1] - vw[k] * zl;
                double* t = vx; vx = vz; vz = t;
            }
            sub_ticks(9, td);
            for (int k = q + 1 + tid; k < ns_old; k += NT) s.so[k - 1] = vatom[k];
            nS = ns_old - 1;
            __syncthreads();
        }
        if (inexact) {
            cert = true;
            continue;
        }
        if (dropped == 0) jadd = jadd < JADD / 2 ? 2 * jadd : JADD;
        else if (nS < 128 && 4 * dropped >= added) jadd = jadd > 1 ? jadd / 2 : 1;
        else jadd = jadd > 8 ? jadd * 7 / 8 : (jadd > 1 ? jadd - 1 : 1);
    }
    if (a.smpl_keep > 0 && !explored && !inexact && nnew > a.smpl_keep && nnew <= NT && a.Q) {
        // Subspace exploratory matching (Algorithm 2): keep the smpl_keep new atoms with the largest |u_j|
        // (ties to the lower atom index); the others leave S (downdates) and I, the kept slots move down
        // to nI0.., and the master problem continues on I_t from u restricted to it.
        explored = true;
        int* s_keep = reinterpret_cast<int*>(vx);     // [nnew] (vx and vg are free once the step ends)
        int* s_newpos = reinterpret_cast<int*>(vg);   // [nnew]
        if (tid < nnew) {
            const int u = nI0 + tid;
            const double xu = fabs(s.x[u]);
            const int au = g_atom[u];
            int rank = 0;
            for (int e = 0; e < nnew; ++e) {
                const double xe = fabs(s.x[nI0 + e]);
                const int ae = g_atom[nI0 + e];
                rank += (xe > xu) || (xe == xu && ae < au);
            }
            s_keep[tid] = rank < a.smpl_keep ? 1 : 0;
        }
        __syncthreads();
        if (tid == 0) {                         // new positions of the kept slots, in slot order
            int pos = nI0;
            for (int e = 0; e < nnew; ++e) s_newpos[e] = s_keep[e] ? pos++ : -1;
        }
        __syncthreads();
        // discarded atoms in S leave it, from the last support position down
        for (int k = nS - 1; k >= 0; --k) {
            const int u = s.so[k];
            if (u < nI0 || s_keep[u - nI0]) continue;
            for (int q = tid; q < nS; q += NT) vatom[q] = s.so[q];   // vatom is scratch after the Gram phase
            __syncthreads();
            chol_drop<BLOCK ? 8 : 4>(s, nS, k, vw, nullptr);
            for (int q = k + 1 + tid; q < nS; q += NT) s.so[q - 1] = vatom[q];
            --nS;
            __syncthreads();
        }
        if (!inexact) {
            // move the kept slots' state down; a slot only moves to a lower position, in increasing
            // order, so every destination has been read already
            for (int e = 0; e < nnew; ++e) {
                const int np = s_newpos[e], u = nI0 + e;
                if (tid == 0) {
                    if (np < 0) {
                        const int atom = g_atom[u];
                        atomicAnd(&w.inI[(int64_t)sig * w.words + (atom >> 5)], ~(1u << (atom & 31)));
                    } else if (np != u) {
                        s.x[np] = s.x[u]; s.c[np] = s.c[u]; s.th[np] = s.th[u]; s.ex[np] = s.ex[u];
                        g_atom[np] = g_atom[u];
                    }
                }
                __syncthreads();
            }
            for (int k = tid; k < nS; k += NT) {
                const int u = s.so[k];
                if (u >= nI0) s.so[k] = s_newpos[u - nI0];
            }
            int kept = 0;
            for (int e = 0; e < nnew; ++e) kept += s_keep[e];
            nI = nI0 + kept;
            __syncthreads();
            // Gram rows of the moved slots again, from the table
            for (int e = tid; e < kept * nI; e += NT) {
                const int t = e / nI, u = e - t * nI;
                const int q = nI0 + t;
                const double val = a.Q[(int64_t)g_atom[q] * a.ldq + g_atom[u]];
                s.G[(int64_t)q * K + u] = val;
                s.G[(int64_t)u * K + q] = val;
            }
            __syncthreads();
            resolve = true;
            xs_ok = false;
            cert = false;
            goto active_set;
        }
    }

    phase_mark(2);

    // 4. Certificate on I (float64), from the gradient on all of I the loop's last pass left in vg.
    double e = 0.0;
    for (int u = tid; u < nI; u += NT) {
        const double gu = vg[u];
        const int th = s.th[u];
        const double d = th != 0 ? fabs(gu - lam * th) : fabs(gu) - lam;
        e = fmax(e, d);
    }
    const double kon = block_max(e, red);
    phase_mark(3);


    // 5. Write the state back (slots left out for this pass only may enter S again).
    if (a.vec_lds) {
        for (int u = tid; u < nI; u += NT) {
            g_x[u] = s.x[u]; g_c[u] = s.c[u]; g_th[u] = s.th[u]; g_ex[u] = s.ex[u] == EX_PASS ? 0 : s.ex[u];
        }
        for (int k = tid; k < nS; k += NT) g_so[k] = s.so[k];
    } else {
        for (int u = tid; u < nI; u += NT)
            if (g_ex[u] == EX_PASS) g_ex[u] = 0;
    }
    if (s.r_lds)
        for (int64_t i = tid; i < tri(nS); i += NT) g_R[i] = s.R[i];
    if (tid == 0) {
        w.nI[sig] = nI;
        w.nS[sig] = nS;
        w.iters[sig] += 1;
        w.kkt_on[sig] = kon > 0.0 ? kon : 0.0;
        w.jadd[sig] = jadd;
        if (inexact) w.status[sig] |= BMPL_SIG_INEXACT;
    }
    phase_mark(5);
    const uint64_t t_res = a.phase ? wall_clock64() : 0;

    // 6. Residual and objective (step 7), from the support's values and atoms gathered into vw / vz
    //    (free after the certificate).
    {
        double* sx = vw;
        int* satom = reinterpret_cast<int*>(vz);
        double l1 = 0.0;
        for (int k = tid; k < nS; k += NT) {
            const int u = s.so[k];
            const double xv = s.x[u];
            sx[k] = xv;
            satom[k] = g_atom[u];
            l1 += fabs(xv);
        }
        const double xl1 = block_sum(l1, red);    // also orders the writes above
        residual_tail(w, sig, a.At, a.lda, a.Bw, sx, satom, nS, xl1, red);
    }
    sub_ticks(14, t_res);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void solve_kernel(SolveArgs a) { solve_body<false, false>(a); }
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void solve_fold_kernel(SolveArgs a) { solve_body<false, true>(a); }
__global__ __launch_bounds__(256) void solve_block_kernel(SolveArgs a) { solve_body<true, false>(a); }

// ---------------------------------------------------------------------------
// Results: support sorted by atom index, float32 values, per-signal scalars.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a)
{
    const int sig = blockIdx.x;
    const Workspace& w = a.w;
    const int nS = (w.status[sig] & BMPL_SIG_NONFINITE) || !w.blk[sig] ? 0 : w.nS[sig];
    const SlotBlock b = slot_block(w.blk[sig], w.cap[sig], w.n);   // only read when nS > 0
    const int* so = b.sord;
    const double* xs = b.x;
    const int* at = b.atom;
    const int64_t K = a.stage_max;
    int cnt = 0;
    if (a.stage && nS <= a.stage_max) {
        // the support's values and atoms (INT_MAX for a zero value) in LDS, then ranks from LDS
        extern __shared__ double s_px[];
        int* s_pa = reinterpret_cast<int*>(s_px + K);
        for (int k = threadIdx.x; k < nS; k += 256) {
            const int u = so[k];
            const double xu = xs[u];
            s_px[k] = xu;
            s_pa[k] = xu != 0.0 ? at[u] : INT_MAX;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nS; k += 256) {
            const int atom = s_pa[k];
            if (atom == INT_MAX) continue;
            int rank = 0;
            for (int k2 = 0; k2 < nS; ++k2) rank += s_pa[k2] < atom;
            if (rank < a.ld_x) {
                a.x_idx[(int64_t)sig * a.ld_x + rank] = atom;
                a.x_val[(int64_t)sig * a.ld_x + rank] = (float)s_px[k];
            }
        }
    } else {
        // rank by atom index among the support positions with a nonzero value
        for (int k = threadIdx.x; k < nS; k += 256) {
            const int u = so[k];
            const double xu = xs[u];
            if (xu == 0.0) continue;
            const int atom = at[u];
            int rank = 0;
            for (int k2 = 0; k2 < nS; ++k2) {
                const int u2 = so[k2];
                if (xs[u2] != 0.0 && at[u2] < atom) ++rank;
            }
            if (rank < a.ld_x) {
                a.x_idx[(int64_t)sig * a.ld_x + rank] = atom;
                a.x_val[(int64_t)sig * a.ld_x + rank] = (float)xu;
            }
        }
    }
    for (int k = threadIdx.x; k < nS; k += 256) cnt += xs[so[k]] != 0.0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    __shared__ int s_c[4];
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = cnt;
    __syncthreads();
    const int tot = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    for (int s = tot + threadIdx.x; s < a.ld_x; s += 256) {   // the rest of the row: -1 / 0
        a.x_idx[(int64_t)sig * a.ld_x + s] = -1;
        a.x_val[(int64_t)sig * a.ld_x + s] = 0.f;
    }
    if (threadIdx.x == 0) {
        a.supp_len[sig] = tot;
        const bool bad = w.status[sig] & BMPL_SIG_NONFINITE;
        if (a.iters) a.iters[sig] = w.iters[sig];
        if (a.kkt) a.kkt[sig] = bad ? NAN : w.kkt[sig];
        if (a.lambda) a.lambda[sig] = w.lam[sig];
        if (a.objective) a.objective[sig] = bad ? NAN : w.obj[sig];
        if (a.status) a.status[sig] = w.status[sig];
    }
}

}  // namespace bmpl
