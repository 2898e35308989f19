/*
 * FP64 reference implementation of Matching Pursuit LASSO (MPL) and its batch
 * mode, used only as test infrastructure: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it to check the GPU library.  The product
 * path never links or calls this file.
 *
 * What it computes, per signal b_i (the batch problem, Eq. (3), is separable
 * over the columns of B; read with one half per signal and a per-signal
 * lambda_i, as the LASSO Eq. (2) and the master problem Eq. (7) have it):
 *
 *     x_i* = argmin_x  lambda_i ||x||_1 + 1/2 ||b_i - A x||^2.
 *
 * The steps follow Algorithm 1 (MPL), in the paper's order and notation:
 *   1. x^0 = 0, xi^0 = b, I_0 = {} (initialisation of Algorithm 1);
 *   2. worst-case analysis: g = A^T xi^{t-1} (a full matrix-vector product),
 *      J_t = the rho atoms outside I with the largest |g_j| that violate
 *      |g_j| > lambda (ties go to the lower index), I_t = I_{t-1} u J_t;
 *   3. master problem Eq. (7) on I_t, warm-started at x^{t-1};
 *   4. xi^t = b - A_I x_I;
 *   5. stop when ||A^T xi||_inf <= lambda, the natural stopping condition of
 *      the "Stopping Conditions" subsection (checked here outside I to a
 *      relative 1e-12, since atoms inside I satisfy it through step 3).
 * Without early stopping the result is the LASSO solution (same subsection).
 * With omega > 1, step 2 becomes subspace exploratory matching (Algorithm 2,
 * SMPL): the omega*rho largest violators J_omega enter, the master problem is
 * solved on I u J_omega, the rho atoms of J_omega with the largest |u_j| (ties
 * to the lower index) form J_t and the others leave I; step 3 then solves on
 * I_t warm-started from u restricted to I_t.
 * Early stops (status 64), each off at 0 and checked after the natural stop,
 * in this order:
 *   - Eq. (10): ||A^T xi||_inf <= r_inf or ||xi|| <= r_2, with the two radii
 *     given relative to the signal, r_inf = r_inf_rel ||A^T b||_inf and
 *     r_2 = r2_rel ||b|| (the paper leaves their values open).  Atoms in I
 *     satisfy |a_j^T xi| <= lambda after step 3, so the maximum is taken
 *     outside I: when r_inf < lambda the natural stop comes first anyway.
 *   - Eq. (13): the last outer iteration lowered the objective by at most
 *     eps_early * rho * ||b||^2.  Eq. (11) with tolerance eps is the same
 *     rule with eps_early = eps / 2, since f(x^0) = ||b||^2 / 2.
 * For lambda = 0 and rho = 1 this is OMP (end of the "Stopping Conditions"
 * subsection), and the r_2 rule is OMP's usual residual-norm stop.
 *
 * The paper solves the master problem with proximal gradient (lambda > 0) or
 * conjugate gradient (lambda = 0) to a small tolerance.  This oracle solves it
 * exactly instead: cyclic coordinate descent on the restricted Gram system,
 * then a sign-fixed polish that solves A_S^T A_S x = A_S^T b - lambda s
 * through a Householder QR of A_S, accepted only once the restricted
 * optimality conditions are verified to 1e-10 lambda.  The exact restricted
 * minimiser is the point proximal gradient converges to.
 *
 * Arithmetic: the float32 inputs are promoted exactly to double; everything
 * after that is double.  No blocking or reordering beyond plain loops.
 *
 * Parity is pinned by the CPU test suite against brute-force support
 * enumeration, the LASSO optimality conditions, the dual of Eq. (5), closed
 * forms (orthonormal dictionaries, noiseless sign-consistent recovery), the
 * OMP reduction (lambda = 0, rho = 1) and an independent full-problem
 * coordinate descent.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_CONVERGED   1
#define ST_CAP_ITERS   2
#define ST_CAP_ACTIVE  4
#define ST_NONFINITE   8
#define ST_INEXACT     32   /* restricted solve could not be verified exact */
#define ST_EARLY       64   /* stopped by the objective-decrease rule, Eq. (13) */

#define STOP_REL   1e-12    /* natural stop test outside I, relative to lambda */
#define VERIFY_REL 1e-10    /* restricted optimality accepted to this, relative to lambda */
#define CD_SWEEP_CAP 2000000

typedef struct {
    int n, m;
    const float* A;   /* atom-major: atom j at A + j*lda */
    int64_t lda;
    const float* b;
    double lam;
    int cap;          /* capacity of the active-set arrays */
    int nI;           /* |I| */
    int* I;           /* atom index per slot, insertion order */
    double* x;        /* x_I */
    double* c;        /* c_I = A_I^T b */
    double* G;        /* G_II, cap x cap row-major */
    double* grad;     /* c_I - G_II x_I */
    double* r;        /* residual xi, length n */
    double* g;        /* A^T xi, length m */
    unsigned char* inI;
    double* qr;       /* n x |S| work for the polish */
    double* work;     /* length >= 3n */
    int qr_cap;
} sig_state;

static double dot_f32_f64(const float* a, const double* v, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += (double)a[k] * v[k];
    return s;
}

static double dot_f32_f32(const float* a, const float* b, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += (double)a[k] * (double)b[k];
    return s;
}

static double soft(double z, double lam)
{
    if (z > lam) return z - lam;
    if (z < -lam) return z + lam;
    return 0.0;
}

static int grow(sig_state* st, int need)
{
    if (need <= st->cap) return 0;
    int nc = st->cap ? st->cap : 16;
    while (nc < need) nc *= 2;
    int* I = (int*)realloc(st->I, sizeof(int) * nc);
    if (!I) return -1;
    st->I = I;
    double* x = (double*)realloc(st->x, sizeof(double) * nc);
    if (!x) return -1;
    st->x = x;
    double* c = (double*)realloc(st->c, sizeof(double) * nc);
    if (!c) return -1;
    st->c = c;
    double* gr = (double*)realloc(st->grad, sizeof(double) * nc);
    if (!gr) return -1;
    st->grad = gr;
    double* G = (double*)malloc(sizeof(double) * (size_t)nc * nc);
    if (!G) return -1;
    for (int u = 0; u < st->nI; ++u)
        memcpy(G + (size_t)u * nc, st->G + (size_t)u * st->cap, sizeof(double) * st->nI);
    free(st->G);
    st->G = G;
    st->cap = nc;
    return 0;
}

/* A full matrix-vector product g = A^T xi (the worst-case analysis of Algorithm 1). */
static void full_correlation(sig_state* st)
{
    for (int j = 0; j < st->m; ++j)
        st->g[j] = dot_f32_f64(st->A + (size_t)j * st->lda, st->r, st->n);
}

/* xi = b - A_I x_I (step 7 of Algorithm 1). */
static void residual(sig_state* st)
{
    for (int k = 0; k < st->n; ++k) st->r[k] = (double)st->b[k];
    for (int u = 0; u < st->nI; ++u) {
        double xu = st->x[u];
        if (xu == 0.0) continue;
        const float* a = st->A + (size_t)st->I[u] * st->lda;
        for (int k = 0; k < st->n; ++k) st->r[k] -= (double)a[k] * xu;
    }
}

/* Append atom j to I with x_j = 0: Gram row, c_j and the gradient entry. */
static void append_atom(sig_state* st, int j)
{
    int q = st->nI;
    const float* aj = st->A + (size_t)j * st->lda;
    for (int u = 0; u < q; ++u) {
        double v = dot_f32_f32(aj, st->A + (size_t)st->I[u] * st->lda, st->n);
        st->G[(size_t)q * st->cap + u] = v;
        st->G[(size_t)u * st->cap + q] = v;
    }
    st->G[(size_t)q * st->cap + q] = dot_f32_f32(aj, aj, st->n);
    st->I[q] = j;
    st->x[q] = 0.0;
    st->c[q] = dot_f32_f32(aj, st->b, st->n);
    double gq = st->c[q];
    for (int u = 0; u < q; ++u) gq -= st->G[(size_t)q * st->cap + u] * st->x[u];
    st->grad[q] = gq;
    st->inI[j] = 1;
    st->nI = q + 1;
}

/* Largest violation of the restricted optimality conditions of Eq. (7), using grad = c - G x. */
static double restricted_violation(const sig_state* st)
{
    double v = 0.0;
    for (int u = 0; u < st->nI; ++u) {
        double gu = st->grad[u], e;
        if (st->x[u] > 0.0) e = fabs(gu - st->lam);
        else if (st->x[u] < 0.0) e = fabs(gu + st->lam);
        else e = fabs(gu) - st->lam;
        if (e > v) v = e;
    }
    return v;
}

static void refresh_grad(sig_state* st)
{
    for (int u = 0; u < st->nI; ++u) {
        double s = st->c[u];
        const double* Gu = st->G + (size_t)u * st->cap;
        for (int w = 0; w < st->nI; ++w) s -= Gu[w] * st->x[w];
        st->grad[u] = s;
    }
}

/* One cyclic coordinate-descent sweep over I; returns the number of sign changes. */
static int cd_sweep(sig_state* st)
{
    int changes = 0;
    for (int u = 0; u < st->nI; ++u) {
        const double* Gu = st->G + (size_t)u * st->cap;
        double old = st->x[u];
        double z = st->grad[u] + Gu[u] * old;
        double nw = soft(z, st->lam) / Gu[u];
        if (nw != old) {
            double d = nw - old;
            for (int w = 0; w < st->nI; ++w) st->grad[w] -= st->G[(size_t)w * st->cap + u] * d;
            if ((old > 0) != (nw > 0) || (old < 0) != (nw < 0)) ++changes;
            st->x[u] = nw;
        }
    }
    return changes;
}

/*
 * Sign-fixed polish: with S = supp(x_I) and s = sign(x_S), solve
 * A_S^T A_S x_S = A_S^T b - lambda s via Householder QR of A_S.  Accept it only
 * if sign(x_S) = s and, with xi = b - A_S x_S, |a_j^T xi - lambda s_j| <= tol on
 * S and |a_j^T xi| <= lambda + tol on I \ S.  Returns 1 if accepted (x_I, grad
 * updated), 0 otherwise (state untouched).  For lambda = 0 the set S is all of I.
 */
static int polish(sig_state* st)
{
    const int n = st->n;
    int* S = (int*)malloc(sizeof(int) * (st->nI + 1));
    double* sg = (double*)malloc(sizeof(double) * (st->nI + 1));
    int ns = 0;
    for (int u = 0; u < st->nI; ++u) {
        if (st->lam == 0.0 || st->x[u] != 0.0) {
            S[ns] = u;
            sg[ns] = st->x[u] > 0 ? 1.0 : (st->x[u] < 0 ? -1.0 : 0.0);
            ++ns;
        }
    }
    int ok = 0;
    double* xs = NULL;
    if (ns > n) goto done;
    if (ns > st->qr_cap) {
        free(st->qr);
        st->qr = (double*)malloc(sizeof(double) * (size_t)n * ns);
        st->qr_cap = ns;
    }
    xs = (double*)malloc(sizeof(double) * (ns + 1));
    double* R = st->qr;              /* column-major n x ns; becomes V (below diag) + R */
    double* qtb = st->work;          /* length n */
    double* vv = st->work + n;       /* length n */
    double* diag = st->work + 2 * n; /* length ns <= n */
    for (int s = 0; s < ns; ++s) {
        const float* a = st->A + (size_t)st->I[S[s]] * st->lda;
        for (int k = 0; k < n; ++k) R[(size_t)s * n + k] = (double)a[k];
    }
    for (int k = 0; k < n; ++k) qtb[k] = (double)st->b[k];
    double fro = 0.0;
    for (size_t e = 0; e < (size_t)n * ns; ++e) fro += R[e] * R[e];
    fro = sqrt(fro);
    for (int s = 0; s < ns; ++s) {
        double* col = R + (size_t)s * n;
        double nrm = 0.0;
        for (int k = s; k < n; ++k) nrm += col[k] * col[k];
        nrm = sqrt(nrm);
        if (nrm <= 1e-13 * (fro > 0 ? fro : 1.0)) goto done;   /* rank deficient */
        double alpha = col[s] > 0 ? -nrm : nrm;
        for (int k = s; k < n; ++k) vv[k] = col[k];
        vv[s] -= alpha;
        double vn = 0.0;
        for (int k = s; k < n; ++k) vn += vv[k] * vv[k];
        vn = sqrt(vn);
        for (int k = s; k < n; ++k) vv[k] /= vn;
        for (int t = s; t < ns; ++t) {            /* R[s:, t] -= 2 v (v^T R[s:, t]) */
            double* ct = R + (size_t)t * n;
            double d = 0.0;
            for (int k = s; k < n; ++k) d += vv[k] * ct[k];
            d *= 2.0;
            for (int k = s; k < n; ++k) ct[k] -= d * vv[k];
        }
        double d = 0.0;
        for (int k = s; k < n; ++k) d += vv[k] * qtb[k];
        d *= 2.0;
        for (int k = s; k < n; ++k) qtb[k] -= d * vv[k];
        diag[s] = col[s];
    }
    /* R^T y = s (forward), then R x = Q^T b - lambda y (backward). */
    for (int s = 0; s < ns; ++s) {
        double v = sg[s];
        for (int t = 0; t < s; ++t) v -= R[(size_t)s * n + t] * xs[t];
        xs[s] = v / diag[s];
    }
    for (int s = 0; s < ns; ++s) xs[s] = qtb[s] - st->lam * xs[s];
    for (int s = ns - 1; s >= 0; --s) {
        double v = xs[s];
        for (int t = s + 1; t < ns; ++t) v -= R[(size_t)t * n + s] * xs[t];
        xs[s] = v / diag[s];
    }
    if (st->lam > 0.0) {
        for (int s = 0; s < ns; ++s)
            if (!(xs[s] * sg[s] > 0.0)) goto done;
    }
    {
        /* verify on the true residual */
        double* r = st->work;   /* reuse: qtb no longer needed */
        double bn = 0.0;
        for (int k = 0; k < n; ++k) { r[k] = (double)st->b[k]; bn += r[k] * r[k]; }
        for (int s = 0; s < ns; ++s) {
            const float* a = st->A + (size_t)st->I[S[s]] * st->lda;
            for (int k = 0; k < n; ++k) r[k] -= (double)a[k] * xs[s];
        }
        double tol = st->lam > 0.0 ? VERIFY_REL * st->lam : 1e-11 * sqrt(bn);
        unsigned char* inS = (unsigned char*)calloc(st->nI, 1);
        for (int s = 0; s < ns; ++s) inS[S[s]] = 1;
        int good = 1;
        for (int s = 0, u = 0; u < st->nI; ++u) {
            double gj = dot_f32_f64(st->A + (size_t)st->I[u] * st->lda, r, n);
            if (inS[u]) {
                if (fabs(gj - st->lam * sg[s]) > tol) good = 0;
                ++s;
            } else if (fabs(gj) > st->lam + tol) {
                good = 0;
            }
        }
        free(inS);
        if (!good) goto done;
    }
    for (int u = 0; u < st->nI; ++u) st->x[u] = 0.0;
    for (int s = 0; s < ns; ++s) st->x[S[s]] = xs[s];
    refresh_grad(st);
    ok = 1;
done:
    free(xs);
    free(S);
    free(sg);
    return ok;
}

/* Master problem Eq. (7) on I, warm-started at the current x_I (step 4 of Algorithm 1). */
static int master_solve(sig_state* st)
{
    refresh_grad(st);
    long sweeps = 0;
    int stable = 0;
    for (;;) {
        int ch = cd_sweep(st);
        ++sweeps;
        stable = ch == 0 ? stable + 1 : 0;
        double viol = restricted_violation(st);
        int try_now = viol <= VERIFY_REL * (st->lam > 0 ? st->lam : 1.0)
                      || (stable >= 3 && (sweeps % 8) == 0);
        if (try_now && polish(st)) return 0;
        if (sweeps >= CD_SWEEP_CAP) return ST_INEXACT;
    }
}

typedef struct {
    double* obj;     /* objective after each outer iteration, [0] = initial */
    int* added;      /* atoms added, in order */
    double* gsel;    /* g_j of each added atom at selection time */
    int* nadd;       /* atoms added per iteration */
    int cap_iters;
} trace_t;

static void free_state(sig_state* st)
{
    free(st->I); free(st->x); free(st->c); free(st->G); free(st->grad);
    free(st->r); free(st->g); free(st->inI); free(st->qr); free(st->work);
}

static double objective(const sig_state* st)
{
    double rr = 0.0, l1 = 0.0;
    for (int k = 0; k < st->n; ++k) rr += st->r[k] * st->r[k];
    for (int u = 0; u < st->nI; ++u) l1 += fabs(st->x[u]);
    return 0.5 * rr + st->lam * l1;
}

/* Solve one signal; results go to the output slots of signal `col`. */
/* Subspace exploratory matching (Algorithm 2): of the atoms J_omega appended since slot `first`
 * (after the master problem on I u J_omega was solved), keep the `keep` with the largest |u_j|, ties to
 * the lower atom index, in their selection order; the others leave I.  The kept atoms are appended
 * again (fresh Gram rows and c) with their u values, the old slots keep theirs. */
static void smpl_prune(sig_state* st, int first, int keep)
{
    int nj = st->nI - first;
    if (nj <= keep) return;
    int* atoms = (int*)malloc(sizeof(int) * nj);
    double* u = (double*)malloc(sizeof(double) * nj);
    unsigned char* kept = (unsigned char*)calloc(nj, 1);
    for (int q = 0; q < nj; ++q) { atoms[q] = st->I[first + q]; u[q] = st->x[first + q]; }
    for (int r = 0; r < keep; ++r) {          /* r-th largest |u|, ties to the lower atom index */
        int best = -1;
        for (int q = 0; q < nj; ++q) {
            if (kept[q]) continue;
            if (best < 0 || fabs(u[q]) > fabs(u[best]) || (fabs(u[q]) == fabs(u[best]) && atoms[q] < atoms[best]))
                best = q;
        }
        kept[best] = 1;
    }
    for (int q = 0; q < nj; ++q) st->inI[atoms[q]] = 0;
    st->nI = first;
    for (int q = 0; q < nj; ++q) {
        if (!kept[q]) continue;
        append_atom(st, atoms[q]);
        st->x[st->nI - 1] = u[q];
    }
    free(atoms); free(u); free(kept);
}

static void solve_one(const float* A, int64_t lda, int n, int m, const float* b, double lam,
                      int rho, int omega, double eps_early, double r_inf_rel, double r2_rel,
                      int max_outer, int max_active, double* xdense, int* iters, double* kkt, double* obj, double* margin,
                      double* gap, int* status, int* supp_len, trace_t* tr)
{
    sig_state st;
    memset(&st, 0, sizeof st);
    st.n = n; st.m = m; st.A = A; st.lda = lda; st.b = b; st.lam = lam;
    st.r = (double*)malloc(sizeof(double) * n);
    st.g = (double*)malloc(sizeof(double) * m);
    st.inI = (unsigned char*)calloc(m, 1);
    st.work = (double*)malloc(sizeof(double) * 3 * (size_t)n + 8);
    for (int j = 0; j < m; ++j) xdense[j] = 0.0;
    int stat = 0, t = 0;
    int finite = isfinite(lam) && lam >= 0.0;
    for (int k = 0; k < n; ++k) if (!isfinite(b[k])) finite = 0;
    if (!finite) {
        *iters = 0; *kkt = NAN; *obj = NAN; *margin = NAN; *gap = NAN;
        *status = ST_NONFINITE; *supp_len = 0;
        free_state(&st);
        return;
    }
    residual(&st);
    if (tr) tr->obj[0] = objective(&st);
    double bb = 0.0;
    for (int k = 0; k < n; ++k) bb += (double)b[k] * (double)b[k];
    double f_prev = objective(&st), f_cur = f_prev;
    double r_inf = 0.0;                       /* r_inf_rel ||A^T b||_inf, set at t = 0 */
    const double r_2 = r2_rel * sqrt(bb);
    for (;;) {
        full_correlation(&st);
        double vmax = 0.0;
        for (int j = 0; j < m; ++j)
            if (!st.inI[j] && fabs(st.g[j]) > vmax) vmax = fabs(st.g[j]);
        if (t == 0) r_inf = r_inf_rel * vmax;
        if (vmax <= lam * (1.0 + STOP_REL)) { stat |= ST_CONVERGED; break; }
        /* early stop, Eq. (10): small correlations or a small residual (off unless the radii are > 0) */
        if (r_inf_rel > 0.0 && vmax <= r_inf) { stat |= ST_EARLY; break; }
        if (r2_rel > 0.0) {
            double rr = 0.0;
            for (int k = 0; k < n; ++k) rr += st.r[k] * st.r[k];
            if (sqrt(rr) <= r_2) { stat |= ST_EARLY; break; }
        }
        /* early stop, Eq. (13): the last outer iteration lowered the objective by at most
         * eps * rho * ||b||^2 (off unless eps_early > 0) */
        if (eps_early > 0.0 && t >= 1 && fabs(f_prev - f_cur) <= eps_early * rho * bb) { stat |= ST_EARLY; break; }
        if (t >= max_outer) { stat |= ST_CAP_ITERS; break; }
        if (st.nI >= max_active) { stat |= ST_CAP_ACTIVE; break; }
        int want = rho;
        if (st.nI + want > max_active) want = max_active - st.nI;
        const int explore = omega > 1 ? omega * want : want;   /* SMPL: omega rho candidates (Algorithm 2) */
        if (grow(&st, st.nI + explore) != 0) { stat |= ST_INEXACT; break; }
        const int first = st.nI;
        /* J_t (or J_omega): the largest |g_j| outside I that exceed lambda, ties to the lower index. */
        int nsel = 0;
        for (int q = 0; q < explore; ++q) {
            int best = -1;
            double bv = lam;
            for (int j = 0; j < m; ++j) {
                if (st.inI[j]) continue;
                double v = fabs(st.g[j]);
                if (v > bv) { bv = v; best = j; }
            }
            if (best < 0) break;
            append_atom(&st, best);
            ++nsel;
        }
        if (omega > 1 && nsel > want) {
            /* exploratory master problem on I u J_omega, then keep the `want` atoms with the largest |u| */
            stat |= master_solve(&st);
            smpl_prune(&st, first, want);
            nsel = st.nI - first;
        }
        if (tr) {
            for (int q = 0; q < nsel; ++q) {
                tr->added[t * rho + q] = st.I[first + q];
                tr->gsel[t * rho + q] = st.g[st.I[first + q]];
            }
            tr->nadd[t] = nsel;
        }
        stat |= master_solve(&st);
        residual(&st);
        ++t;
        f_prev = f_cur;
        f_cur = objective(&st);
        if (tr) tr->obj[t] = f_cur;
    }
    /* Outputs: x, the certificate kappa, the objective, the margin and the duality gap of Eq. (5). */
    double F = objective(&st);
    double kap = 0.0, mu = INFINITY, ginf = 0.0;
    int ns = 0;
    for (int u = 0; u < st.nI; ++u) xdense[st.I[u]] = st.x[u];
    for (int j = 0; j < m; ++j) {
        double gj = st.g[j], xj = xdense[j];
        if (fabs(gj) > ginf) ginf = fabs(gj);
        double e;
        if (xj != 0.0) {
            ++ns;
            e = fabs(gj - (xj > 0 ? lam : -lam));
            if (fabs(xj) < mu) mu = fabs(xj);
        } else {
            e = fabs(gj) - lam;
            if (e < 0) e = 0;
            if (lam - fabs(gj) < mu) mu = lam - fabs(gj);
        }
        if (e > kap) kap = e;
    }
    double scale = ginf > lam ? lam / ginf : 1.0;   /* alpha = xi * min(1, lambda/||A^T xi||_inf) */
    double aa = 0.0, ab = 0.0;
    for (int k = 0; k < n; ++k) {
        double a = st.r[k] * scale;
        aa += a * a;
        ab += a * (double)b[k];
    }
    *iters = t;
    *kkt = lam > 0 ? kap / lam : kap;
    *obj = F;
    *margin = mu;
    *gap = F - (-0.5 * aa + ab);
    *status = stat;
    *supp_len = ns;
    free_state(&st);
}

int mpl_oracle_abi_version(void) { return 4; }

/*
 * Batch solve: p independent signals (Eq. (3)), one per OpenMP thread.
 * At: atom j at At + j*lda (float32, lda >= n).  Bt: signal i at Bt + i*ldb.
 * lam[i]: lambda_i (>= 0).  X: dense m x p output, signal i at X + i*ldx.
 * Per-signal outputs are arrays of length p.  Returns 0, or -1 on bad arguments.
 */
int mpl_oracle_solve(const float* At, int64_t lda, int n, int m, const float* Bt, int64_t ldb,
                     int p, const double* lam, int rho, int omega, double eps_early, double r_inf_rel,
                     double r2_rel, int max_outer, int max_active,
                     int nthreads,
                     double* X, int64_t ldx, int* iters, double* kkt, double* obj, double* margin,
                     double* gap, int* status, int* supp_len)
{
    if (!At || !Bt || !lam || !X || n <= 0 || m <= 0 || p < 0 || lda < n || ldb < n || ldx < m
        || rho <= 0 || omega < 1 || max_outer < 0 || max_active <= 0
        || !(eps_early >= 0.0) || !(r_inf_rel >= 0.0) || !(r2_rel >= 0.0))
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int i = 0; i < p; ++i)
        solve_one(At, lda, n, m, Bt + (size_t)i * ldb, lam[i], rho, omega, eps_early, r_inf_rel, r2_rel,
                  max_outer, max_active,
                  X + (size_t)i * ldx, iters + i, kkt + i, obj + i, margin + i, gap + i,
                  status + i, supp_len + i, NULL);
    return 0;
}

/* Number of threads the OpenMP runtime will use for mpl_oracle_solve with nthreads <= 0. */
int mpl_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * One signal with a per-iteration trace: obj[0..T] (obj[0] = 1/2||b||^2),
 * added[t*rho + q] / gsel[t*rho + q] for q < nadd[t], t < T.  Arrays must hold
 * max_outer + 1 (obj), max_outer * rho (added, gsel) and max_outer (nadd).
 */
int mpl_oracle_trace(const float* At, int64_t lda, int n, int m, const float* b, double lam,
                     int rho, int omega, double eps_early, double r_inf_rel, double r2_rel,
                     int max_outer, int max_active, double* x, int* iters,
                     double* kkt,
                     double* objv, double* margin, double* gap, int* status, int* supp_len,
                     double* obj_trace, int* added, double* gsel, int* nadd)
{
    if (!At || !b || !x || n <= 0 || m <= 0 || lda < n || rho <= 0 || omega < 1 || max_outer < 0 || max_active <= 0
        || !(eps_early >= 0.0) || !(r_inf_rel >= 0.0) || !(r2_rel >= 0.0))
        return -1;
    trace_t tr = { obj_trace, added, gsel, nadd, max_outer };
    solve_one(At, lda, n, m, b, lam, rho, omega, eps_early, r_inf_rel, r2_rel, max_outer, max_active, x, iters, kkt,
              objv, margin, gap,
              status, supp_len, &tr);
    return 0;
}
