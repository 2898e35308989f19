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
// Cholesky row append computed with two matrix-vector products, every solve is
// two matrix-vector products, and removing position q truncates the factor to
// q rows and appends the later positions again.
//
// One 256-thread workgroup per signal; signals are independent.
#include <float.h>

#include "../../include/bmpl.h"
#include "bmpl_internal.h"
#include "pursuit.h"

namespace bmpl {
namespace {

constexpr int NT = 256;
constexpr int NB = 16;      // new atoms per Gram pass
constexpr int CH = 128;     // k per Gram staging chunk

__device__ inline double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__device__ inline double block_max(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// (alpha, position) minimum, ties to the smaller position.
__device__ inline void block_argmin(double& a, int& q, double* red, int* redi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        double oa = __shfl_xor(a, o);
        int oq = __shfl_xor(q, o);
        if (oa < a || (oa == a && (unsigned)oq < (unsigned)q)) { a = oa; q = oq; }
    }
    __syncthreads();
    if (lane == 0) { red[wave] = a; redi[wave] = q; }
    __syncthreads();
    a = red[0];
    q = redi[0];
    for (int w = 1; w < 4; ++w)
        if (red[w] < a || (red[w] == a && (unsigned)redi[w] < (unsigned)q)) { a = red[w]; q = redi[w]; }
}

struct SigView {
    int K;
    int* slot_atom;
    double* x;
    double* c;
    signed char* theta;
    unsigned char* excl;
    int* sord;
    double* G;
    double* Rinv;
};

__device__ inline SigView view(const Workspace& w, int sig)
{
    SigView v;
    v.K = w.K;
    const int64_t K = w.K;
    v.slot_atom = w.slot_atom + sig * K;
    v.x = w.x + sig * K;
    v.c = w.c + sig * K;
    v.theta = w.theta + sig * K;
    v.excl = w.excl + sig * K;
    v.sord = w.sord + sig * K;
    v.G = w.G + sig * tri(K);
    v.Rinv = w.Rinv + sig * tri(K);
    return v;
}

// Append slot j with sign th at support position s = *nS.  Returns false (and
// marks j excluded) if its Schur complement pivot vanishes, i.e. a_j is
// numerically in the span of A_S.
__device__ bool chol_append(SigView& v, int& nS, int j, signed char th, double* vw, double* vz,
                            double* red)
{
    const int s = nS;
    const int tid = threadIdx.x;
    for (int k = tid; k < s; k += NT) vw[k] = sym_at(v.G, v.sord[k], j);
    __syncthreads();
    double part = 0.0;
    for (int i = tid; i < s; i += NT) {      // z = Rinv w (row i of the packed factor)
        const double* Ri = v.Rinv + tri(i);
        double acc = 0.0;
        for (int k = 0; k <= i; ++k) acc += Ri[k] * vw[k];
        vz[i] = acc;
        part += acc * acc;
    }
    const double zz = block_sum(part, red);
    const double gjj = v.G[tri(j) + j];
    const double dd = gjj - zz;
    if (!(dd > 1e-11 * gjj)) {
        if (tid == 0) { v.excl[j] = 1; v.theta[j] = 0; v.x[j] = 0.0; }
        __syncthreads();
        return false;
    }
    const double d = sqrt(dd);
    double* Rs = v.Rinv + tri(s);
    for (int k = tid; k < s; k += NT) {      // new row: -(z^T Rinv)_k / d
        const int i0 = k & ~63;
        double acc = 0.0;
        for (int i = i0; i < s; ++i)
            if (i >= k) acc += vz[i] * v.Rinv[tri(i) + k];
        Rs[k] = -acc / d;
    }
    if (tid == 0) {
        Rs[s] = 1.0 / d;
        v.sord[s] = j;
        v.theta[j] = th;
    }
    nS = s + 1;
    __syncthreads();
    return true;
}

// x_S = Rinv^T Rinv (c_S - lambda theta_S) into vx[0..nS).
__device__ void sign_fixed_solve(const SigView& v, int nS, double lam, double* vw, double* vz, double* vx)
{
    const int tid = threadIdx.x;
    for (int k = tid; k < nS; k += NT) {
        const int u = v.sord[k];
        vw[k] = v.c[u] - lam * (double)v.theta[u];
    }
    __syncthreads();
    for (int i = tid; i < nS; i += NT) {
        const double* Ri = v.Rinv + tri(i);
        double acc = 0.0;
        for (int k = 0; k <= i; ++k) acc += Ri[k] * vw[k];
        vz[i] = acc;
    }
    __syncthreads();
    for (int k = tid; k < nS; k += NT) {
        const int i0 = k & ~63;
        double acc = 0.0;
        for (int i = i0; i < nS; ++i)
            if (i >= k) acc += v.Rinv[tri(i) + k] * vz[i];
        vx[k] = acc;
    }
    __syncthreads();
}

// g_u = c_u - sum_{k<nS} G(u, sord[k]) x_{sord[k]} for every slot u < nI (wave per slot).
__device__ void restricted_gradient(const SigView& v, int nI, int nS, double* vg)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int u = wave; u < nI; u += NT / 64) {
        double acc = 0.0;
        for (int k = lane; k < nS; k += 64) {
            const int sv = v.sord[k];
            acc += sym_at(v.G, u, sv) * v.x[sv];
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) vg[u] = v.c[u] - acc;
    }
    __syncthreads();
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
    double part = 0.0;
    int bad = 0;
    for (int r = threadIdx.x; r < w.kpad; r += 256) {
        float v = r < w.n ? b[r] : 0.f;
        if (!isfinite(v)) bad = 1;
        Bw[r] = v;
        R[r] = v;
        part += (double)v * (double)v;
    }
    if (bad) atomicOr(&s_bad, 1);
    for (int q = threadIdx.x; q < w.words; q += 256) w.inI[(int64_t)sig * w.words + q] = 0u;
    const double bb = block_sum(part, red);
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
        w.vmax[sig] = 0.f;
        w.kkt_on[sig] = 0.0;
        w.kkt[sig] = 0.0;
        w.obj[sig] = 0.5 * bb;
    }
}

// ---------------------------------------------------------------------------
// Stop test and compaction.  For each running signal after a selection pass:
// no admitted atom -> stop (natural stop if no violator remains, else the
// active-set cap was hit); iteration cap -> stop; otherwise keep it running.
// One workgroup; the running list stays in signal order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void status_compact_kernel(StatusArgs a)
{
    const Workspace& w = a.w;
    const int n_in = a.n_in_dev ? *a.n_in_dev : a.n_in;
    __shared__ int s_scan[1024];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
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
                if (ns == 0 || w.iters[sig] >= a.max_outer) {
                    double off = vm - lam;
                    off = off > 0.0 ? off : 0.0;
                    double kk = fmax(off, w.kkt_on[sig]);
                    kk = lam > 0.0 ? kk / lam : kk;
                    w.kkt[sig] = kk;
                    if (a.warm_check && ns != 0) st |= BMPL_SIG_FALLBACK;
                    if (ns == 0 && vm <= lam) {
                        if (kk <= a.kkt_tol) st |= BMPL_SIG_CONVERGED;
                    } else if (ns == 0) {
                        st |= BMPL_SIG_CAP_ACTIVE;
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
        s_scan[threadIdx.x] = keep;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {           // inclusive Hillis-Steele scan
            int t = threadIdx.x >= o ? s_scan[threadIdx.x - o] : 0;
            __syncthreads();
            s_scan[threadIdx.x] += t;
            __syncthreads();
        }
        if (keep) a.act_out[s_base + s_scan[threadIdx.x] - 1] = sig;
        __syncthreads();
        if (threadIdx.x == 1023) s_base += s_scan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.n_out_dev = s_base;
}

// ---------------------------------------------------------------------------
// Warm start: replace this pass's selection with the proposed atoms.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void warm_select_kernel(WarmArgs a)
{
    __shared__ int s_sel[256];
    const int n_act = *a.n_act_dev;
    const int row = blockIdx.x;
    if (row >= n_act) return;
    const int sig = a.act[row];
    const Workspace& w = a.w;
    if (threadIdx.x == 0) {
        int cnt = 0;
        int cap = a.max_active < w.selcap ? a.max_active : w.selcap;
        cap = cap < 256 ? cap : 256;
        for (int q = 0; q < a.warm_k && cnt < cap; ++q) {
            const int j = a.warm[(int64_t)sig * a.warm_k + q];
            if (j < 0 || j >= w.m) continue;
            bool dup = false;
            for (int t = 0; t < cnt; ++t) dup |= s_sel[t] == j;
            if (!dup) s_sel[cnt++] = j;
        }
        // an empty proposal keeps this pass's own selection
        if (cnt > 0) {
            for (int t = 0; t < cnt; ++t) w.sel[(int64_t)sig * w.selcap + t] = s_sel[t];
            w.nsel[sig] = cnt;
        }
    }
}

// ---------------------------------------------------------------------------
// Master problem on I for every running signal, then its residual and objective.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void solve_kernel(SolveArgs a)
{
    extern __shared__ double s_dyn[];
    __shared__ double red[4];
    __shared__ int redi[4];
    __shared__ double s_new[CH * NB];
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
    SigView v = view(w, sig);
    const int K = w.K;
    double* vb = a.use_lds ? s_dyn : (w.vscratch + (int64_t)sig * 6 * K);
    double* vw = vb;
    double* vz = vb + K;
    double* vx = vb + 2 * K;
    double* vg = vb + 3 * K;
    int* vatom = reinterpret_cast<int*>(vb + 4 * K);

    const int nI0 = w.nI[sig];
    int nS = w.nS[sig];
    const double lam = w.lam[sig];
    const int nI = nI0 + nnew;

    // 1. New slots.
    for (int t = tid; t < nnew; t += NT) {
        const int q = nI0 + t;
        const int atom = w.sel[(int64_t)sig * w.selcap + t];
        v.slot_atom[q] = atom;
        v.x[q] = 0.0;
        v.theta[q] = 0;
        v.excl[q] = 0;
        atomicOr(&w.inI[(int64_t)sig * w.words + (atom >> 5)], 1u << (atom & 31));
    }
    __syncthreads();

    // 2. Gram rows of the new slots against every slot, and c = a^T b (slot index nI).
    const float* bw = a.Bw + (int64_t)sig * w.kpad;
    for (int g0 = 0; g0 < nnew; g0 += NB) {
        const int nb = nnew - g0 < NB ? nnew - g0 : NB;
        for (int ub = 0; ub <= nI; ub += NT) {
            const int u = ub + tid;
            const bool live = u <= nI;
            const float* col = (u < nI) ? a.At + (int64_t)v.slot_atom[u] * a.lda : bw;
            double acc[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) acc[t] = 0.0;
            for (int kc = 0; kc < w.kpad; kc += CH) {
                __syncthreads();
                for (int e = tid; e < nb * CH; e += NT) {
                    const int t = e / CH, kk = e % CH;
                    const int atom = v.slot_atom[nI0 + g0 + t];
                    s_new[kk * NB + t] = (kc + kk < w.kpad) ? (double)a.At[(int64_t)atom * a.lda + kc + kk] : 0.0;
                }
                __syncthreads();
                if (live) {
                    const int kend = (w.kpad - kc) < CH ? (w.kpad - kc) : CH;
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
                    if (u == nI) v.c[q] = acc[t];
                    else if (u <= q) v.G[tri(q) + u] = acc[t];
                }
            }
        }
    }
    __syncthreads();

    // 3. Sign-fixed active-set iterations.
    int steps = 0;
    bool inexact = false;
    for (;;) {
        restricted_gradient(v, nI, nS, vg);
        // violators outside S in slot order (wave 0 ballot scan)
        if (wave == 0) {
            int base = 0;
            for (int u0 = 0; u0 < nI && base < NT; u0 += 64) {
                const int u = u0 + lane;
                bool viol = false;
                if (u < nI && v.theta[u] == 0 && !v.excl[u])
                    viol = fabs(vg[u]) > lam * (1.0 + 1e-12) && fabs(vg[u]) > 0.0;
                const unsigned long long bal = __ballot(viol);
                const int pre = __popcll(bal & ((1ull << lane) - 1ull));
                if (viol && base + pre < NT) s_list[base + pre] = u;
                base += __popcll(bal);
            }
            if (lane == 0) s_cnt = base < NT ? base : NT;
        }
        __syncthreads();
        const int nv = s_cnt;
        if (nv == 0) break;
        for (int e = 0; e < nv; ++e) {
            const int u = s_list[e];
            const signed char th = vg[u] > 0.0 ? 1 : -1;
            if (nS >= w.n) { if (tid == 0) v.excl[u] = 1; __syncthreads(); continue; }
            chol_append(v, nS, u, th, vw, vz, red);
        }
        // inner loop: move toward the sign-fixed minimiser, dropping at zero crossings
        for (;;) {
            if (++steps > a.max_steps) { inexact = true; break; }
            sign_fixed_solve(v, nS, lam, vw, vz, vx);
            double alpha = 1.0;
            int q = -1;
            for (int k = tid; k < nS; k += NT) {
                const int u = v.sord[k];
                const double xo = v.x[u], xn = vx[k], th = (double)v.theta[u];
                if (xn * th <= 0.0) {
                    const double ak = (xo == 0.0) ? 0.0 : fmax(xo / (xo - xn), 0.0);
                    if (ak < alpha || (ak == alpha && (q < 0 || k < q))) { alpha = ak; q = k; }
                }
            }
            block_argmin(alpha, q, red, redi);
            for (int k = tid; k < nS; k += NT) {
                const int u = v.sord[k];
                const double xo = v.x[u];
                v.x[u] = xo + alpha * (vx[k] - xo);
            }
            __syncthreads();
            if (q < 0) break;
            // drop position q and re-append the later positions in order
            const int ns_old = nS;
            for (int k = tid; k < ns_old; k += NT) vatom[k] = v.sord[k];
            __syncthreads();
            if (tid == 0) {
                const int u = vatom[q];
                v.x[u] = 0.0;
                v.theta[u] = 0;
            }
            __syncthreads();
            nS = q;
            for (int k = q + 1; k < ns_old; ++k) {
                const int u = vatom[k];
                if (!chol_append(v, nS, u, v.theta[u], vw, vz, red)) {
                    if (tid == 0) v.x[u] = 0.0;
                    __syncthreads();
                }
            }
        }
        if (inexact) break;
    }

    // 4. Certificate on I (float64), residual xi = b - A_S x_S, objective.
    restricted_gradient(v, nI, nS, vg);
    double e = 0.0;
    for (int u = tid; u < nI; u += NT) {
        const double gu = vg[u];
        const int th = v.theta[u];
        double d = th != 0 ? fabs(gu - lam * th) : fabs(gu) - lam;
        e = fmax(e, d);
    }
    const double kon = block_max(e, red);
    double l1 = 0.0;
    for (int k = tid; k < nS; k += NT) {
        const int u = v.sord[k];
        vatom[k] = v.slot_atom[u];
        vx[k] = v.x[u];
        l1 += fabs(v.x[u]);
    }
    const double xl1 = block_sum(l1, red);
    double rr = 0.0;
    float* Rres = w.R + (int64_t)sig * w.kpad;
    for (int r = tid; r < w.kpad; r += NT) {
        double acc = (double)bw[r];
        for (int k = 0; k < nS; ++k) acc -= (double)a.At[(int64_t)vatom[k] * a.lda + r] * vx[k];
        if (r >= w.n) acc = 0.0;
        Rres[r] = (float)acc;
        rr += acc * acc;
    }
    const double rn = block_sum(rr, red);
    if (tid == 0) {
        w.nI[sig] = nI;
        w.nS[sig] = nS;
        w.iters[sig] += 1;
        w.kkt_on[sig] = kon > 0.0 ? kon : 0.0;
        w.obj[sig] = 0.5 * rn + lam * xl1;
        if (inexact) w.status[sig] |= BMPL_SIG_INEXACT;
    }
    (void)lane;
}

// ---------------------------------------------------------------------------
// Results: support sorted by atom index, float32 values, per-signal scalars.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a)
{
    const int sig = blockIdx.x;
    const Workspace& w = a.w;
    SigView v = view(w, sig);
    const int nS = (w.status[sig] & BMPL_SIG_NONFINITE) ? 0 : w.nS[sig];
    int cnt = 0;
    // rank by atom index among the support positions with a nonzero value
    for (int k = threadIdx.x; k < nS; k += 256) {
        const int u = v.sord[k];
        const double xu = v.x[u];
        if (xu == 0.0) continue;
        const int atom = v.slot_atom[u];
        int rank = 0;
        for (int k2 = 0; k2 < nS; ++k2) {
            const int u2 = v.sord[k2];
            if (v.x[u2] != 0.0 && v.slot_atom[u2] < atom) ++rank;
        }
        if (rank < a.ld_x) {
            a.x_idx[(int64_t)sig * a.ld_x + rank] = atom;
            a.x_val[(int64_t)sig * a.ld_x + rank] = (float)xu;
        }
    }
    for (int k = threadIdx.x; k < nS; k += 256) cnt += v.x[v.sord[k]] != 0.0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    __shared__ int s_c[4];
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        a.supp_len[sig] = tot;
        const bool bad = w.status[sig] & BMPL_SIG_NONFINITE;
        if (a.iters) a.iters[sig] = w.iters[sig];
        if (a.kkt) a.kkt[sig] = bad ? NAN : w.kkt[sig];
        if (a.lambda) a.lambda[sig] = w.lam[sig];
        if (a.objective) a.objective[sig] = bad ? NAN : w.obj[sig];
        if (a.status) a.status[sig] = w.status[sig];
    }
}

// ---------------------------------------------------------------------------
// Capacity growth: copy the per-signal state from stride K_old to stride K_new.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void restride_kernel(RestrideArgs a)
{
    const int sig = blockIdx.x;
    const int nI = min(a.nI[sig], a.K_old);
    const int nS = min(a.nS[sig], a.K_old);
    const int64_t o1 = (int64_t)sig * a.K_old, n1 = (int64_t)sig * a.K_new;
    for (int u = threadIdx.x; u < nI; u += 256) {
        a.dst.slot_atom[n1 + u] = a.src.slot_atom[o1 + u];
        a.dst.x[n1 + u] = a.src.x[o1 + u];
        a.dst.c[n1 + u] = a.src.c[o1 + u];
        a.dst.theta[n1 + u] = a.src.theta[o1 + u];
        a.dst.excl[n1 + u] = a.src.excl[o1 + u];
    }
    for (int k = threadIdx.x; k < nS; k += 256) a.dst.sord[n1 + k] = a.src.sord[o1 + k];
    const int64_t go = (int64_t)sig * tri(a.K_old), gn = (int64_t)sig * tri(a.K_new);
    for (int64_t e = threadIdx.x; e < tri(nI); e += 256) a.dst.G[gn + e] = a.src.G[go + e];
    for (int64_t e = threadIdx.x; e < tri(nS); e += 256) a.dst.Rinv[gn + e] = a.src.Rinv[go + e];
}

}  // namespace bmpl
