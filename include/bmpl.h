/*
 * bmpl.h - C ABI of the batch-mode Matching Pursuit LASSO library for
 * AMD MI355X (gfx950).
 *
 * Problem (the batch sparse-recovery problem, Eq. (3), read with one half per
 * signal and a per-signal lambda_i, which makes it separable over signals and
 * equal to p copies of the LASSO, Eq. (2)):
 *
 *     for every column b_i of B:   min_x  lambda_i ||x||_1 + 1/2 ||b_i - A x||^2
 *
 * solved by Matching Pursuit LASSO (Algorithm 1) run on all p signals at once:
 * each outer iteration computes the correlations G = A^T (B - A X) of every
 * still-running signal as one matrix product (the full matrix-vector products
 * of the "Implementation Concerns" subsection, batched), adds to each signal's
 * active set I the rho atoms outside I with the largest |g_j| > lambda_i
 * (the worst-case analysis), solves the master problem Eq. (7) restricted to I
 * exactly, and stops a signal once ||A^T xi||_inf <= lambda_i, the natural
 * stopping condition of the "Stopping Conditions" subsection.  Without early
 * stopping the result is the LASSO solution.
 *
 * Conventions shared by every entry point
 *  - All pointers named *_dev are device pointers (hipMalloc'd memory or
 *    PyTorch CUDA tensors) on the device that is current when the context is
 *    created.  Host pointers are named without the suffix.
 *  - A is column-major n x m: element (r, j) is A_dev[r + j*lda], lda >= n, so
 *    atom a_j is contiguous (the atom-by-atom storage of "Implementation
 *    Concerns").  B is column-major n x p with leading dimension ldb >= n.
 *  - Calls that take a `hip_stream` enqueue their work on that stream
 *    (NULL = the null stream) and may return before it finishes; outputs are
 *    valid once the stream is synchronised.  bmpl_solve reads back how many
 *    signals are still running (a stream synchronisation) once per outer
 *    iteration, or once per captured segment of four iterations with
 *    BMPL_FLAG_GRAPH; with BMPL_FLAG_GRAPH and an iteration cap
 *    (bmpl_options.max_outer) of at most 64 it captures the whole solve as one
 *    graph, sizes every signal's slot memory for that cap up front, and does
 *    not synchronise at all (when that memory fits; see BMPL_FLAG_GRAPH).
 *  - Every call returns a bmpl_status; on failure bmpl_last_error(ctx) describes
 *    it.  A context is not re-entrant: one call in flight per context.
 */
#ifndef BMPL_H
#define BMPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmpl_ctx bmpl_ctx;

typedef enum {
    BMPL_OK = 0,
    BMPL_E_INVALID = -1,      /* bad shape, pointer or option */
    BMPL_E_NOMEM = -2,        /* device allocation failed */
    BMPL_E_HIP = -3,          /* a HIP runtime call failed */
    BMPL_E_UNSUPPORTED = -4   /* valid request this build does not implement */
} bmpl_status;

typedef enum {
    BMPL_LAMBDA_ABS = 0,          /* lambda_i = value, or lambda_dev[i] when given to bmpl_solve */
    BMPL_LAMBDA_REL_MAX_ATB = 1   /* lambda_i = value * ||A^T b_i||_inf (Section IV-A's rule) */
} bmpl_lambda_mode;

typedef enum {
    BMPL_PREC_FP32 = 0,   /* correlation product in float32 (MFMA, float32 accumulation) */
    BMPL_PREC_BF16 = 1,   /* bfloat16 screening product, float32 re-score before admission */
    BMPL_PREC_FP8 = 2     /* e4m3 ranking product (power-of-two scales per atom and per signal) after
                             the first pass: its highest-ranked atoms are re-scored in float32 and the
                             exact violators among them admitted; a signal with none is decided by the
                             certified bfloat16 pass, which also runs the first pass (lambda rule) */
} bmpl_precision;

/* Per-signal status bits (bmpl_result.sig_status). */
#define BMPL_SIG_CONVERGED   1   /* natural stop reached: kkt <= kkt_tol */
#define BMPL_SIG_CAP_ITERS   2   /* max_outer outer iterations done, not converged */
#define BMPL_SIG_CAP_ACTIVE  4   /* |I| reached max_active, not converged */
#define BMPL_SIG_NONFINITE   8   /* b_i or lambda_i not finite: x_i = 0 */
#define BMPL_SIG_FALLBACK   16   /* a warm-start proposal failed the certificate */
#define BMPL_SIG_INEXACT    32   /* a restricted solve hit its step cap */
#define BMPL_SIG_EARLY      64   /* stopped early by Eq. (10) or Eq. (13) (bmpl_options.eps_early,
                                    r_inf_rel, r2_rel); kkt reports how far from the natural stop */

/* bmpl_options.flags bits. */
#define BMPL_FLAG_TIMING 1          /* time every kernel launch with HIP events (see bmpl_get_timing) */
#define BMPL_FLAG_NO_GRAM_TABLE 2   /* do not precompute Q = A^T A; Gram rows by direct dot products */
#define BMPL_FLAG_GRAPH 4           /* run the outer iterations as captured HIP graphs of 4 iterations each
                                       (2 once fewer than 64 signals run), one launch and one read-back per
                                       segment (ignored with TIMING).  With max_outer in 1..64 the whole
                                       solve is one graph of max_outer iterations (passes after the last
                                       signal's stop run as empty launches) with no read-back: each
                                       signal's slot memory is then sized for |I| up to the cap
                                       (p (K^2 + K(K+1)/2 + ...) float64, K = the cap's bound on |I|),
                                       which must fit in the memory the context already holds for it plus
                                       half of the free device memory, else the segments are used */
#define BMPL_FLAG_Q_ROUTE 32        /* Section III's batch correlation, Eq. (12): after the first pass,
                                       g = beta - Q_{:,S} x_S with beta = A^T b (float64, computed once
                                       per solve) and the float64 Gram table, instead of the MFMA product
                                       A^T xi; needs the Gram table and the float32 screen */
#define BMPL_FLAG_PHASES 16         /* with TIMING: also count the master-problem kernel's phases, factor
                                       appends, drops and solves (device atomics and clock reads inside the
                                       kernel, which slow it; the per-kernel times of TIMING alone do not) */
#define BMPL_FLAG_BLOCK_APPEND 8    /* grow the master problem's inverse Cholesky factor in blocks of up
                                       to 8 atoms when it lives in global memory, instead of one atom at
                                       a time (same factor in exact arithmetic).  Off by default: on the
                                       4096-signal ragged batch (1024 x 32768, supports up to ~980)
                                       single appends take 14.4 s against 17.0 s */

/* Tile shapes of the correlation kernel (bmpl_autotune, bmpl_set_tuning), signals x atoms (waves of
 * 64 lanes, each computing the sub-tile in parentheses): 0 128x128 (64x64), 1 256x256 (64x64, 16 waves),
 * 2 256x128 (64x64), 3 64x128 (32x64), 4 32x64 (32x32), 5 64x64 (32x32), 6 256x256 (128x128, 4 waves),
 * 7 256x256 (128x64, 8 waves); bfloat16 screening only (the dictionary's fragments read from global
 * memory in the matrix instruction's order, the residual tile through LDS): 8 256x256 (128x64, 8 waves),
 * 9 128x256 (64x64, 8 waves), 10 256x128 (128x64, 4 waves); both operand tiles copied from global
 * memory straight into LDS (no staging registers): 11 256x256 (128x64, 8 waves), 12 256x256 (64x64, 16
 * waves), 13 128x128 (64x64, 4 waves), 14 256x256 (128x128, 4 waves).  A shape a precision lacks is
 * rejected by bmpl_set_tuning and not timed by bmpl_autotune. */
#define BMPL_CORR_SHAPES 15

/* bmpl_create precomputes the float64 Gram table Q = A^T A (8 m^2 bytes, the
 * precomputed Q of Section III, Eq. (12)) when it is at most this large. */
#define BMPL_GRAM_TABLE_MAX_BYTES (16.0 * 1024.0 * 1024.0 * 1024.0)

typedef struct {
    int32_t rho;            /* atoms added per outer iteration (Algorithm 1, step 3); default 10 */
    int32_t max_outer;      /* outer-iteration cap; <= 0 selects ceil(m / rho) */
    int32_t max_active;     /* cap on |I|; <= 0 selects min(m, 2n) */
    double kkt_tol;         /* certificate tolerance relative to lambda_i; default 1e-4 */
    bmpl_precision screen;  /* precision of the correlation product; default FP32 */
    int32_t flags;          /* BMPL_FLAG_* bits; default 0 */
    int32_t omega;          /* subspace exploratory matching (Algorithm 2, SMPL) when > 1: omega * rho
                               candidates enter, the master problem is solved on I u J_omega, the rho
                               with the largest |u_j| stay (ties to the lower index) and the master
                               problem is solved again on I_t; needs the Gram table and
                               omega * rho <= 64; default 1 (MPL) */
    /* Early stops of the "Stopping Conditions" subsection and of the experimental settings, each off at
     * 0 (the default) and tested, per signal, after the natural stop at the start of an outer iteration,
     * in this order (status BMPL_SIG_EARLY, the current x is returned):
     *   Eq. (10): max_{j not in I} |a_j^T xi| <= r_inf_rel * ||A^T b_i||_inf (atoms in I meet
     *             |a_j^T xi| <= lambda_i, so this is ||A^T xi||_inf <= r_inf once r_inf >= lambda_i), or
     *             ||xi|| <= r2_rel * ||b_i||; ||A^T b_i||_inf comes from the first correlation pass;
     *   Eq. (13): the last outer iteration lowered the objective by at most eps_early * rho * ||b_i||^2
     *             (rho = the rho above).  Eq. (11) with tolerance eps is eps_early = eps / 2, since
     *             f(x^0) = ||b_i||^2 / 2.
     * With lambda = 0 and rho = 1 the solve is OMP and r2_rel its residual-norm stop. */
    double eps_early;
    double r_inf_rel;
    double r2_rel;
} bmpl_options;

/*
 * Caller-owned device result buffers, filled by bmpl_solve.  For signal i:
 * x_idx[i*ld_x + s], x_val[i*ld_x + s] for s < supp_len[i] hold the nonzero
 * coefficients sorted by atom index, and -1 / 0 for supp_len[i] <= s < ld_x (every entry is
 * written, so the caller need not clear the buffers); ld_x >= min(max_active, n).
 * kkt[i] = max( max_{j not in S}(|a_j^T xi| - lambda)_+ , max_{j in S}|a_j^T xi - lambda sign x_j| ) / lambda,
 * computed in float64 on I; outside I from the correlation product with its rounding bounded: atoms
 * whose reduced-precision or float32 |g~_j| lies within the product's error bound of lambda are re-scored
 * exactly (float32 data, float64 sums) before the natural stop is accepted, so a signal is never reported
 * CONVERGED while an atom outside I has an exact |a_j^T xi| > lambda.
 * objective[i] = lambda ||x||_1 + 1/2 ||b - A x||^2 in float64.
 * lambda[i] = the lambda_i actually used.  iters[i] = outer iterations that added atoms.
 * Any pointer except x_idx/x_val/supp_len may be NULL to skip that output.
 */
typedef struct {
    float* x_val_dev;
    int32_t* x_idx_dev;
    int32_t* supp_len_dev;
    int32_t* iters_dev;
    double* kkt_dev;
    double* lambda_dev;
    double* objective_dev;
    int32_t* sig_status_dev;
    int32_t ld_x;
} bmpl_result;

/* Fill `o` with the defaults listed in bmpl_options.  Returns BMPL_E_INVALID for NULL. */
bmpl_status bmpl_options_default(bmpl_options* o);

/*
 * Create a context for dictionary A (n x m, see conventions) and the lambda rule.
 * The library copies A into its own device memory (float32, rows padded to a
 * multiple of 32 with zeros), so the caller may free A_dev after the call, and
 * unless BMPL_FLAG_NO_GRAM_TABLE is set (or the table would exceed
 * BMPL_GRAM_TABLE_MAX_BYTES) computes the float64 Gram table Q = A^T A, from
 * which the master problem gathers the Gram rows of atoms entering an active set.
 * `o` may be NULL for the defaults.  Work is enqueued on `hip_stream` and the
 * stream is synchronised before returning.  Errors: BMPL_E_INVALID for n <= 0,
 * m <= 0, lda < n, NULL pointers, lambda < 0 or a non-finite lambda, rho <= 0;
 * BMPL_E_NOMEM / BMPL_E_HIP on runtime failures.  *out is NULL on failure.
 */
bmpl_status bmpl_create(const float* A_dev, int64_t lda, int32_t n, int32_t m,
                        bmpl_lambda_mode mode, double lambda, const bmpl_options* o,
                        void* hip_stream, bmpl_ctx** out);

/*
 * Solve the p signals in B (n x p, leading dimension ldb) with the context's
 * dictionary, lambda rule and options (Algorithm 1 batched over signals, see
 * the top of this file).  lambda_dev (p float64 values) overrides the context's
 * lambda with per-signal absolute values when non-NULL.  warm_idx_dev (p x
 * warm_k atom indices, -1 = unused entry) seeds each active set: the master
 * problem is solved on the proposal first and the pursuit continues from there,
 * so the result is the same LASSO solution; NULL / warm_k = 0 for none.
 * Workspace grows on demand and is kept in the context.  Per-signal outcomes
 * never fail the call; they are reported in sig_status.  Errors:
 * BMPL_E_INVALID (bad pointers, ldb < n, p < 0, ld_x too small),
 * BMPL_E_NOMEM, BMPL_E_HIP.
 */
bmpl_status bmpl_solve(bmpl_ctx* c, const float* B_dev, int64_t ldb, int32_t p,
                       const double* lambda_dev, const int32_t* warm_idx_dev, int32_t warm_k,
                       const bmpl_result* out, void* hip_stream);

/* Release the context and all its device memory.  NULL is accepted. */
bmpl_status bmpl_destroy(bmpl_ctx* c);

/* Message describing the last failure of a call made on this thread (kept per thread, so it also
 * covers a bmpl_create that returned no context; c may be NULL); valid until the next call. */
const char* bmpl_last_error(const bmpl_ctx* c);

/*
 * Diagnostic entry points (one step of the pursuit each, used by the kernel
 * parity tests and the benchmark's per-kernel timing).
 */

/*
 * The batched correlation step: G[i*ldg + j] = a_j^T r_i for j < m, i < p,
 * where r_i = R_dev + i*ldr (n float32 values, ldr >= n), in the context's
 * screening precision with float32 accumulation (FP8 contexts: e4m3 operands
 * with power-of-two scales per atom and per residual, the ranking product).  This is the full
 * matrix-vector product g = A^T xi of Algorithm 1, step 3, for p residuals at
 * once.  ldg >= m.  Errors: BMPL_E_INVALID.
 */
bmpl_status bmpl_correlate(bmpl_ctx* c, const float* R_dev, int64_t ldr, int32_t p,
                           float* G_dev, int64_t ldg, void* hip_stream);

/*
 * bmpl_correlate for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, layouts and result (the same kernels,
 * so bit-identical to bmpl_correlate), but it allocates nothing and never synchronises: the residuals
 * are staged in a library-owned device array of BMPL_NOALLOC_SCRATCH_BYTES per GPU (held until the
 * process ends), and every launch is asynchronous on hip_stream (kernels only: no memset or memcpy
 * nodes).  The staging needs (p + 1) * kpad * 4 bytes, kpad = n rounded up to 64 (128 with e4m3
 * ranking), plus (p + 1) * kpad * 2 with bfloat16 screening or (p + 1) * (kpad + 4) with e4m3 ranking,
 * each part rounded up to 256 bytes; a larger p returns BMPL_E_INVALID.  Every call on one GPU shares
 * that GPU's array (it keeps the last call's contents; nothing needs clearing): calls that overlap in
 * time on one GPU (different streams, threads or contexts) race and must be ordered by the caller.
 */
#define BMPL_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
bmpl_status bmpl_correlate_noalloc(bmpl_ctx* c, const float* R_dev, int64_t ldr, int32_t p, float* G_dev,
                                   int64_t ldg, void* hip_stream);

/*
 * The worst-case analysis of Algorithm 1, step 3, on given correlations:
 * for each row i of G (p rows, leading dimension ldg >= m) pick up to k atoms j
 * with |G[i,j]| > lambda_dev[i] and mask bit j of excl_dev clear, largest
 * |G[i,j]| first, ties to the lower index.  excl_dev holds p bitmaps of
 * ceil(m/32) uint32 words (bit j of word j/32), or NULL for none.  Writes
 * sel_dev[i*k + q] (atom, -1 past the end) and nsel_dev[i]; also
 * vmax_dev[i] = max over unmasked j of |G[i,j]| (0 if none).  1 <= k <= 64.
 */
bmpl_status bmpl_select(bmpl_ctx* c, const float* G_dev, int64_t ldg, int32_t p,
                        const double* lambda_dev, const uint32_t* excl_dev, int32_t k,
                        int32_t* sel_dev, int32_t* nsel_dev, float* vmax_dev, void* hip_stream);

/*
 * Sparse-representation classification, the face-recognition use of the solver
 * (Section V follows the class-residual rule of sparse-representation-based
 * classification): for signal i (B column-major, ldb >= n) with the code of
 * `sol` (x_idx / x_val / supp_len / ld_x as filled by bmpl_solve), every class c
 * with an atom in the support is scored by ||b_i - A delta_c(x_i)||_2, where
 * delta_c keeps the coefficients of the atoms j with class_of_atom_dev[j] == c
 * (device int32 array of m class indices >= 0).  labels_dev[i] receives the
 * class with the smallest residual (ties to the lower class index; -1 for an
 * empty support) and resid_dev[i] (optional, float64) that residual.  Float64
 * sums from the float32 data; asynchronous on hip_stream.
 * Errors: BMPL_E_INVALID.
 */
bmpl_status bmpl_classify(bmpl_ctx* c, const float* B_dev, int64_t ldb, int32_t p, const bmpl_result* sol,
                          const int32_t* class_of_atom_dev, int32_t* labels_dev, double* resid_dev,
                          void* hip_stream);

/*
 * Autotuner of the correlation product: times every tile shape of the MFMA
 * kernel that runs the outer iterations (float32, bfloat16 or e4m3 by the
 * context's screening precision) on this context's dictionary for three
 * running-signal counts (min(p, 4096), min(p, 128), min(p, 32), representing the
 * buckets >= 512, 64..511 and < 64 running signals) and keeps the fastest shape
 * per bucket in the context; later solves use it.  shapes (3 ints) receives the
 * chosen shape per bucket and ms (3 x BMPL_CORR_SHAPES doubles, bucket-major) the
 * average milliseconds per
 * launch of every shape (-1 where not timed or not launchable); both may be
 * NULL.  Synchronises `hip_stream`.  Errors: BMPL_E_INVALID (NULL context,
 * p < 1), BMPL_E_NOMEM, BMPL_E_HIP.
 */
bmpl_status bmpl_autotune(bmpl_ctx* c, int32_t p, int32_t* shapes, double* ms, void* hip_stream);

/*
 * Set the correlation tile shape per bucket by hand (3 ints in [0, BMPL_CORR_SHAPES), the
 * same meaning as bmpl_autotune's `shapes`), e.g. from a cached tuning.
 * Errors: BMPL_E_INVALID for NULL or an out-of-range shape.
 */
bmpl_status bmpl_set_tuning(bmpl_ctx* c, const int32_t* shapes);

/*
 * Read-only access to the context's float64 Gram table Q = A^T A (the
 * precomputed Q of Section III, Eq. (12)): *Q_dev receives the device pointer
 * (owned by the context, valid until bmpl_destroy; NULL when no table was
 * built) and *ldq its leading dimension (m, or 0).  Q[i*ldq + j] = a_i^T a_j,
 * accumulated in float64 from the float32 atoms.  Errors: BMPL_E_INVALID for NULL.
 */
bmpl_status bmpl_gram_table(const bmpl_ctx* c, const double** Q_dev, int64_t* ldq);

/*
 * Kernel timing accumulated over the solves run since the last reset, recorded
 * with HIP events on the solve's stream when the context was created with
 * BMPL_FLAG_TIMING (all zero otherwise).  corr_flops counts the algorithmic
 * 2 * m * n * p_running flops of every correlation launch (no padding);
 * corr_bytes the algorithmic bytes e * (m * n + n * p_running) + 4 * m * p_running
 * (dictionary and residuals read once in the product's precision, e = 4, 2 or 1 bytes, correlations
 * written once in float32); corr_roof_ms the sum over those launches of their roofline time on MI355X,
 * max(flops / matrix peak of the precision (157.3 / 2500 / 5000 TFLOP/s), bytes / 8 TB/s), so
 * corr_roof_ms / corr_ms is the achieved fraction of the roofline, HBM-bound launches (few running
 * signals) included.  Times are
 * milliseconds.  With timing on, bmpl_solve synchronises its stream before
 * returning.
 */
typedef struct {
    double corr_ms; int64_t corr_launches; double corr_flops; double corr_bytes;
    double select_ms; int64_t select_launches;
    double solve_ms; int64_t solve_launches;
    double residual_ms;     /* 0: the residual xi = b - A_S x_S and objective are the last step of the
                               master-problem kernel and count in solve_ms */
    double other_ms;        /* set-up, compaction, packing */
    double wall_ms;         /* first to last event of each solve, summed */
    int64_t solves;
    int64_t outer_iters;
    /* master-problem kernel, summed over its workgroups (wall-clock counter, microseconds; these and
     * the three counts below need BMPL_FLAG_PHASES):
     * [0] state load, [1] Gram rows, [2] active-set iterations (with the gradient on all of I that
     * the certificate uses), [3] certificate on I,
     * [4] of which inside factor appends, [5] state write-back */
    double solve_phase_us[6];
    int64_t factor_appends;     /* Cholesky row appends (including re-appends after drops) */
    int64_t factor_drops;       /* support positions removed at a zero crossing */
    int64_t sign_fixed_solves;  /* sign-fixed minimiser evaluations */
    double corr_roof_ms;        /* roofline time of the correlation launches (see above) */
    double solve_step_us[6];    /* with BMPL_FLAG_PHASES: time inside the active-set iterations spent in
                                   [0] factor downdates (drops), [1] sign-fixed minimiser evaluations,
                                   [2] gradients outside S (and on all of I for the certificate),
                                   [3] the violator list and its ranking,
                                   [4] the ratio test and step toward the minimiser; [5] the residual
                                   and objective after the write-back; summed over workgroups
                                   (microseconds) */
} bmpl_timing;

/* Copy the accumulated timing into *t.  Errors: BMPL_E_INVALID for NULL. */
bmpl_status bmpl_get_timing(const bmpl_ctx* c, bmpl_timing* t);

/* Zero the accumulated timing.  Errors: BMPL_E_INVALID for NULL. */
bmpl_status bmpl_reset_timing(bmpl_ctx* c);

/* ------------------------------------------------------------------------
 * Learned support proposal.
 *
 * Not part of the paper.  Algorithm 1 keeps the previous iterate as the warm
 * start of every master problem (step 5), and its natural stopping condition
 * (Eq. (9)) certifies the final answer whatever the starting active set was;
 * this network only proposes that starting set (bmpl_solve's warm_idx_dev).
 * A wrong proposal costs iterations, never correctness: atoms proposed in
 * error end with a zero coefficient, atoms it misses are added by the
 * ordinary worst-case analysis, and the signal's status carries
 * BMPL_SIG_FALLBACK when the first check after the proposal found violators.
 *
 * Model, for a signal b (column of B):
 *   z  = (A P)^T b scaled to unit root-mean-square (P: a fixed m x d_in
 *        matrix supplied by the caller, e.g. i.i.d. N(0, 1/d_in); the LASSO
 *        support under the relative lambda rule does not depend on the scale
 *        of b, so neither does the proposal)
 *   h1 = gelu(W1 z + b1), h2 = gelu(W2 h1 + b2), s = W3 h2 + b3   (s: m scores)
 *   gelu(u) = u * Phi(u), Phi the standard normal CDF (exact erf form).
 * Training loss: binary cross-entropy with logits and positive-class weight
 * w, summed over the m atoms and averaged over the batch:
 *   l(s, y) = w y log(1 + e^-s) + (1 - y) log(1 + e^s),
 * targets y_j = 1 for the atoms of a given support (e.g. the supports a
 * bmpl_solve returned).  Optimiser: Adam with bias correction.
 * Arithmetic: bfloat16 weights and activations in the matrix products
 * (MFMA, float32 accumulation); float32 master weights, pre-activations,
 * scores, gradients and Adam moments.
 *
 * Flat parameter vector (float32, row-major blocks in this order):
 *   W1 [d_hidden][d_in], b1 [d_hidden], W2 [d_hidden][d_hidden], b2 [d_hidden],
 *   W3 [m][d_hidden], b3 [m];  length bmpl_mlp_param_count(d_in, d_hidden, m).
 * ---------------------------------------------------------------------- */
typedef struct bmpl_mlp bmpl_mlp;

typedef struct {
    double lr;      /* step size */
    double beta1;   /* first-moment decay (0.9 is usual) */
    double beta2;   /* second-moment decay (0.999) */
    double eps;     /* denominator guard (1e-8) */
} bmpl_adam;

/* Number of floats in the flat parameter vector. */
int64_t bmpl_mlp_param_count(int32_t d_in, int32_t d_hidden, int32_t m);

/*
 * Create a proposal network for the dictionary A (column-major n x m,
 * leading dimension lda >= n, the layout of bmpl_create) and the projection
 * P_dev (row-major m x d_in float32: P[j*d_in + c]).  Computes (A P)^T once
 * (float32 accumulation, stored as bfloat16); A and P may be freed after the
 * call returns.  Parameters start at zero: set them with bmpl_mlp_set_params.
 * max_batch bounds the rows of one bmpl_mlp_loss_grad call and the chunk of
 * signals that bmpl_mlp_forward / bmpl_mlp_propose process at once (they
 * accept any p).  Requires d_in and d_hidden to be positive multiples of 64,
 * m <= 38912 (one row of scores fits the selection kernel's LDS), n, m,
 * max_batch >= 1.  Errors: BMPL_E_INVALID, BMPL_E_NOMEM, BMPL_E_HIP.
 */
bmpl_status bmpl_mlp_create(const float* A_dev, int64_t lda, int32_t n, int32_t m, const float* P_dev,
                            int32_t d_in, int32_t d_hidden, int32_t max_batch, void* hip_stream,
                            bmpl_mlp** out);

/* Release everything the network owns.  NULL is accepted. */
bmpl_status bmpl_mlp_destroy(bmpl_mlp* net);

/*
 * Copy a flat parameter vector (device, float32) into the network's float32
 * master weights, refresh their bfloat16 copies and reset the Adam moments
 * and step count.  bmpl_mlp_get_params copies the master weights out.
 */
bmpl_status bmpl_mlp_set_params(bmpl_mlp* net, const float* params_dev, void* hip_stream);
bmpl_status bmpl_mlp_get_params(const bmpl_mlp* net, float* params_dev, void* hip_stream);

/*
 * The unit-RMS embeddings z of p signals (B column-major n x p, ldb >= n),
 * rounded to bfloat16 as the network consumes them and returned widened to
 * float32: Z_dev[i*ldz + c], ldz >= d_in.
 */
bmpl_status bmpl_mlp_embed(bmpl_mlp* net, const float* B_dev, int64_t ldb, int32_t p, float* Z_dev,
                           int64_t ldz, void* hip_stream);

/* Scores s of p signals: S_dev[i*lds + j], j < m, lds >= m (float32). */
bmpl_status bmpl_mlp_forward(bmpl_mlp* net, const float* B_dev, int64_t ldb, int32_t p, float* S_dev,
                             int64_t lds, void* hip_stream);

/*
 * Loss and gradient on one batch of p <= max_batch signals with target
 * supports supp_dev[i*ld_supp + t], t < supp_len_dev[i] (atom indices;
 * entries outside [0, m) are ignored, so bmpl_solve's x_idx / supp_len can
 * be passed as they are).  *loss_dev (device double) receives the mean loss;
 * grad_dev (device float32, bmpl_mlp_param_count floats, flat layout)
 * receives the gradient, or NULL to keep it inside the network for
 * bmpl_mlp_adam_step.  pos_weight > 0.
 */
bmpl_status bmpl_mlp_loss_grad(bmpl_mlp* net, const float* B_dev, int64_t ldb, int32_t p,
                               const int32_t* supp_dev, int32_t ld_supp, const int32_t* supp_len_dev,
                               double pos_weight, float* grad_dev, double* loss_dev, void* hip_stream);

/*
 * One Adam step on the master weights with the gradient grad_dev (flat
 * layout), or with the gradient of the last bmpl_mlp_loss_grad when NULL;
 * refreshes the bfloat16 copies.  The step count t starts at 1 after
 * bmpl_mlp_set_params.
 */
bmpl_status bmpl_mlp_adam_step(bmpl_mlp* net, const float* grad_dev, const bmpl_adam* hp, void* hip_stream);

/*
 * Proposal: for each of p signals the k (1..256) atoms with the largest
 * scores, ties to the lower index, listed in ascending atom order:
 * idx_dev[i*ld_idx + q], q < k (ld_idx >= k).  This is the warm_idx_dev /
 * warm_k input of bmpl_solve.
 */
bmpl_status bmpl_mlp_propose(bmpl_mlp* net, const float* B_dev, int64_t ldb, int32_t p, int32_t k,
                             int32_t* idx_dev, int32_t ld_idx, void* hip_stream);

/*
 * The selection step of bmpl_mlp_propose on its own, for any score matrix:
 * per row of S_dev[r*lds + j], j < L, the k (1..256) largest entries' column
 * indices in ascending order, ties to the lower index, NaN ranked lowest,
 * -1 padding when L < k.  L <= 38912.
 */
bmpl_status bmpl_topk(const float* S_dev, int64_t lds, int32_t rows, int32_t L, int32_t k, int32_t* idx_dev,
                      int32_t ld_idx, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BMPL_H */
