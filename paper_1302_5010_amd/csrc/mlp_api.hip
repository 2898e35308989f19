// Host side of the learned support proposal (bmpl_mlp_* in include/bmpl.h):
// buffers, the forward pass, the backward pass by the chain rule and the
// Adam step, each a short sequence of the kernels in mlp.hip on the caller's
// stream.
//
// Layouts (row = signal): signals as bfloat16 rows [rows][npad]; embeddings,
// activations and pre-activations [rows][d] / [rows][h]; scores [rows][mpad].
// Transposes for the backward products: a product that contracts over the
// batch (weight gradients) takes [features][capP] copies of both factors, and
// dH = dU W takes W^T.  npad, mpad, capP: n, m, max_batch rounded up to 64,
// with zeros in the padding so that it adds nothing to any contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/bmpl.h"
#include "host_util.h"
#include "mlp.h"

using namespace bmpl;

struct bmpl_mlp {
    int device = 0;
    int n = 0, npad = 0, m = 0, mpad = 0, d = 0, h = 0, cap = 0, capP = 0;
    int64_t count = 0;
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;   // offsets in the flat vector

    float* master = nullptr;     // [count] float32 parameters
    float* m1 = nullptr;         // [count] Adam first moment
    float* m2 = nullptr;         // [count] Adam second moment
    float* grad = nullptr;       // [count] gradient of the last loss_grad (internal target)
    uint16_t* w16 = nullptr;     // [count] bfloat16 copy of the parameters
    uint16_t* w2t = nullptr;     // [h][h]    W2^T
    uint16_t* w3t = nullptr;     // [h][mpad] W3^T
    bool wt_stale = true;        // the transposes lag the parameters
    int64_t t = 0;               // Adam steps taken since set_params
    uint16_t* apt = nullptr;     // [d][npad] (A P)^T

    // forward buffers, cap rows
    uint16_t* b16 = nullptr;     // [cap][npad]
    float* z = nullptr;          // [cap][d]
    uint16_t* x0 = nullptr;      // [cap][d]
    uint16_t* h1 = nullptr;      // [cap][h]
    uint16_t* h2 = nullptr;      // [cap][h]
    float* logits = nullptr;     // [cap][mpad]
    // training buffers, allocated on the first loss_grad
    float* u1 = nullptr;         // [cap][h] pre-activations
    float* u2 = nullptr;
    uint16_t* ds16 = nullptr;    // [cap][mpad] dl/ds, bfloat16
    float* du2 = nullptr;        // [cap][h] dl/du2 and its bfloat16 copy
    uint16_t* du2_16 = nullptr;
    float* du1 = nullptr;        // [cap][h] dl/du1
    uint16_t* du1_16 = nullptr;
    uint16_t* tx0 = nullptr;     // [d][capP]
    uint16_t* th1 = nullptr;     // [h][capP]
    uint16_t* th2 = nullptr;     // [h][capP]
    uint16_t* tdu = nullptr;     // [h][capP]
    uint16_t* tds = nullptr;     // [m][capP]
    float* rowloss = nullptr;    // [cap]
};

namespace {

void free_all(bmpl_mlp* q)
{
    dfree(q->master); dfree(q->m1); dfree(q->m2); dfree(q->grad); dfree(q->w16); dfree(q->w2t); dfree(q->w3t);
    dfree(q->apt); dfree(q->b16); dfree(q->z); dfree(q->x0); dfree(q->h1); dfree(q->h2); dfree(q->logits);
    dfree(q->u1); dfree(q->u2); dfree(q->ds16); dfree(q->du2); dfree(q->du2_16); dfree(q->du1); dfree(q->du1_16);
    dfree(q->tx0); dfree(q->th1); dfree(q->th2); dfree(q->tdu); dfree(q->tds); dfree(q->rowloss);
}

bmpl_status ensure_train_buffers(bmpl_mlp* q)
{
    if (q->u1) return BMPL_OK;
    const size_t cap = q->cap, h = q->h;
    HIPC(dalloc(&q->u1, cap * h));
    HIPC(dalloc(&q->u2, cap * h));
    HIPC(dalloc(&q->ds16, cap * q->mpad));
    HIPC(dalloc(&q->du2, cap * h));
    HIPC(dalloc(&q->du2_16, cap * h));
    HIPC(dalloc(&q->du1, cap * h));
    HIPC(dalloc(&q->du1_16, cap * h));
    HIPC(dalloc(&q->tx0, (size_t)q->d * q->capP));
    HIPC(dalloc(&q->th1, h * q->capP));
    HIPC(dalloc(&q->th2, h * q->capP));
    HIPC(dalloc(&q->tdu, h * q->capP));
    HIPC(dalloc(&q->tds, (size_t)q->m * q->capP));
    HIPC(dalloc(&q->rowloss, cap));
    return BMPL_OK;
}

// Embedding of `rows` signals into x0 (and widened into Zout when given).
bmpl_status embed_rows(bmpl_mlp* q, const float* B, int64_t ldb, int rows, float* Zout, int64_t ldz, hipStream_t s)
{
    HIPC(mlp_signals_bf16(B, ldb, q->n, rows, q->b16, q->npad, s));
    HIPC(mlp_gemm_store(q->b16, q->npad, rows, q->apt, q->npad, q->d, q->npad, q->z, q->d, nullptr, s));
    HIPC(mlp_embed_norm(q->z, q->d, rows, q->x0, Zout, ldz, s));
    return BMPL_OK;
}

// The three layers from x0; scores into S [rows][lds]; pre-activations kept when `keep`.
bmpl_status layers(bmpl_mlp* q, int rows, bool keep, float* S, int64_t lds, hipStream_t s)
{
    const int d = q->d, h = q->h;
    HIPC(mlp_gemm_bias_gelu(q->x0, d, rows, q->w16 + q->oW1, d, h, d, q->master + q->ob1, keep ? q->u1 : nullptr, h,
                            q->h1, h, s));
    HIPC(mlp_gemm_bias_gelu(q->h1, h, rows, q->w16 + q->oW2, h, h, h, q->master + q->ob2, keep ? q->u2 : nullptr, h,
                            q->h2, h, s));
    HIPC(mlp_gemm_store(q->h2, h, rows, q->w16 + q->oW3, h, q->m, h, S, lds, q->master + q->ob3, s));
    return BMPL_OK;
}

bmpl_status refresh_transposes(bmpl_mlp* q, hipStream_t s)
{
    if (!q->wt_stale) return BMPL_OK;
    HIPC(mlp_transpose(q->w16 + q->oW2, q->h, q->h, q->h, q->w2t, q->h, s));
    HIPC(mlp_transpose(q->w16 + q->oW3, q->h, q->m, q->h, q->w3t, q->mpad, s));
    q->wt_stale = false;
    return BMPL_OK;
}

bmpl_status check_signals(const bmpl_mlp* q, const float* B, int64_t ldb, int p, const char* who)
{
    if (!q) return fail(BMPL_E_INVALID, "%s: NULL network", who);
    if (p < 0 || ldb < q->n) return fail(BMPL_E_INVALID, "%s: bad p=%d or ldb=%lld", who, p, (long long)ldb);
    if (p > 0 && !B) return fail(BMPL_E_INVALID, "%s: NULL B", who);
    return BMPL_OK;
}

}  // namespace

extern "C" {

int64_t bmpl_mlp_param_count(int32_t d_in, int32_t d_hidden, int32_t m)
{
    if (d_in < 1 || d_hidden < 1 || m < 1) return 0;
    const int64_t d = d_in, h = d_hidden, mm = m;
    return h * d + h + h * h + h + mm * h + mm;
}

bmpl_status bmpl_mlp_create(const float* A_dev, int64_t lda, int32_t n, int32_t m, const float* P_dev,
                            int32_t d_in, int32_t d_hidden, int32_t max_batch, void* hip_stream, bmpl_mlp** out)
{
    if (!out) return fail(BMPL_E_INVALID, "bmpl_mlp_create: NULL out");
    *out = nullptr;
    if (!A_dev || !P_dev) return fail(BMPL_E_INVALID, "bmpl_mlp_create: NULL A or P");
    if (n < 1 || m < 1 || lda < n || max_batch < 1)
        return fail(BMPL_E_INVALID, "bmpl_mlp_create: bad n=%d m=%d lda=%lld max_batch=%d", n, m, (long long)lda,
                    max_batch);
    if (d_in < 64 || d_in % 64 || d_hidden < 64 || d_hidden % 64)
        return fail(BMPL_E_INVALID, "bmpl_mlp_create: d_in=%d and d_hidden=%d must be positive multiples of 64", d_in,
                    d_hidden);
    if ((size_t)m * 4 > TOPK_MAX_LDS)
        return fail(BMPL_E_INVALID, "bmpl_mlp_create: m=%d exceeds the selection kernel's limit of %zu atoms", m,
                    TOPK_MAX_LDS / 4);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    bmpl_mlp* q = new bmpl_mlp;
    auto bail = [&](bmpl_status st) { free_all(q); delete q; return st; };
    if (hipGetDevice(&q->device) != hipSuccess) return bail(fail(BMPL_E_HIP, "bmpl_mlp_create: hipGetDevice failed"));
    q->n = n; q->npad = round_up(n, 64); q->m = m; q->mpad = round_up(m, 64);
    q->d = d_in; q->h = d_hidden; q->cap = max_batch; q->capP = round_up(max_batch, 64);
    q->count = bmpl_mlp_param_count(d_in, d_hidden, m);
    const int64_t d = d_in, h = d_hidden;
    q->oW1 = 0; q->ob1 = h * d; q->oW2 = q->ob1 + h; q->ob2 = q->oW2 + h * h; q->oW3 = q->ob2 + h; q->ob3 = q->oW3 + m * h;
    bmpl_status st = [&]() -> bmpl_status {
        HIPC(dalloc(&q->master, q->count));
        HIPC(dalloc(&q->m1, q->count));
        HIPC(dalloc(&q->m2, q->count));
        HIPC(dalloc(&q->grad, q->count));
        HIPC(dalloc(&q->w16, q->count));
        HIPC(dalloc(&q->w2t, (size_t)h * h));
        HIPC(dalloc(&q->w3t, (size_t)h * q->mpad));
        HIPC(dalloc(&q->apt, (size_t)d * q->npad));
        const size_t cap = max_batch;
        HIPC(dalloc(&q->b16, cap * q->npad));
        HIPC(dalloc(&q->z, cap * d));
        HIPC(dalloc(&q->x0, cap * d));
        HIPC(dalloc(&q->h1, cap * h));
        HIPC(dalloc(&q->h2, cap * h));
        HIPC(dalloc(&q->logits, cap * q->mpad));
        HIPC(hipMemsetAsync(q->master, 0, q->count * sizeof(float), s));
        HIPC(hipMemsetAsync(q->m1, 0, q->count * sizeof(float), s));
        HIPC(hipMemsetAsync(q->m2, 0, q->count * sizeof(float), s));
        HIPC(hipMemsetAsync(q->w16, 0, q->count * sizeof(uint16_t), s));
        HIPC(mlp_project(A_dev, lda, n, m, P_dev, d_in, q->apt, q->npad, s));
        HIPC(hipStreamSynchronize(s));
        return BMPL_OK;
    }();
    if (st != BMPL_OK) return bail(st);
    *out = q;
    return BMPL_OK;
}

bmpl_status bmpl_mlp_destroy(bmpl_mlp* net)
{
    if (!net) return BMPL_OK;
    (void)hipDeviceSynchronize();
    free_all(net);
    delete net;
    return BMPL_OK;
}

bmpl_status bmpl_mlp_set_params(bmpl_mlp* q, const float* params_dev, void* hip_stream)
{
    if (!q || !params_dev) return fail(BMPL_E_INVALID, "bmpl_mlp_set_params: NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    HIPC(hipMemcpyAsync(q->master, params_dev, q->count * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPC(hipMemsetAsync(q->m1, 0, q->count * sizeof(float), s));
    HIPC(hipMemsetAsync(q->m2, 0, q->count * sizeof(float), s));
    HIPC(mlp_params_bf16(q->master, q->w16, q->count, s));
    q->t = 0;
    q->wt_stale = true;
    return BMPL_OK;
}

bmpl_status bmpl_mlp_get_params(const bmpl_mlp* q, float* params_dev, void* hip_stream)
{
    if (!q || !params_dev) return fail(BMPL_E_INVALID, "bmpl_mlp_get_params: NULL argument");
    HIPC(hipMemcpyAsync(params_dev, q->master, q->count * sizeof(float), hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(hip_stream)));
    return BMPL_OK;
}

bmpl_status bmpl_mlp_embed(bmpl_mlp* q, const float* B_dev, int64_t ldb, int32_t p, float* Z_dev, int64_t ldz,
                           void* hip_stream)
{
    bmpl_status st = check_signals(q, B_dev, ldb, p, "bmpl_mlp_embed");
    if (st != BMPL_OK) return st;
    if (p > 0 && (!Z_dev || ldz < q->d)) return fail(BMPL_E_INVALID, "bmpl_mlp_embed: need Z with ldz >= %d", q->d);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    for (int r0 = 0; r0 < p; r0 += q->cap) {
        const int rows = std::min(q->cap, p - r0);
        st = embed_rows(q, B_dev + (int64_t)r0 * ldb, ldb, rows, Z_dev + (int64_t)r0 * ldz, ldz, s);
        if (st != BMPL_OK) return st;
    }
    return BMPL_OK;
}

bmpl_status bmpl_mlp_forward(bmpl_mlp* q, const float* B_dev, int64_t ldb, int32_t p, float* S_dev, int64_t lds,
                             void* hip_stream)
{
    bmpl_status st = check_signals(q, B_dev, ldb, p, "bmpl_mlp_forward");
    if (st != BMPL_OK) return st;
    if (p > 0 && (!S_dev || lds < q->m)) return fail(BMPL_E_INVALID, "bmpl_mlp_forward: need S with lds >= %d", q->m);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    for (int r0 = 0; r0 < p; r0 += q->cap) {
        const int rows = std::min(q->cap, p - r0);
        st = embed_rows(q, B_dev + (int64_t)r0 * ldb, ldb, rows, nullptr, 0, s);
        if (st == BMPL_OK) st = layers(q, rows, false, S_dev + (int64_t)r0 * lds, lds, s);
        if (st != BMPL_OK) return st;
    }
    return BMPL_OK;
}

bmpl_status bmpl_mlp_loss_grad(bmpl_mlp* q, const float* B_dev, int64_t ldb, int32_t p, const int32_t* supp_dev,
                               int32_t ld_supp, const int32_t* supp_len_dev, double pos_weight, float* grad_dev,
                               double* loss_dev, void* hip_stream)
{
    bmpl_status st = check_signals(q, B_dev, ldb, p, "bmpl_mlp_loss_grad");
    if (st != BMPL_OK) return st;
    if (p < 1 || p > q->cap) return fail(BMPL_E_INVALID, "bmpl_mlp_loss_grad: p=%d outside [1, max_batch=%d]", p, q->cap);
    if (!supp_len_dev || !supp_dev || ld_supp < 0 || !loss_dev)
        return fail(BMPL_E_INVALID, "bmpl_mlp_loss_grad: need supports, their lengths and a loss pointer");
    if (!(pos_weight > 0.0)) return fail(BMPL_E_INVALID, "bmpl_mlp_loss_grad: pos_weight must be > 0");
    st = ensure_train_buffers(q);
    if (st != BMPL_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int d = q->d, h = q->h, m = q->m, mpad = q->mpad, capP = q->capP;
    const int kB = round_up(p, 64);     // batch contraction length (zero-padded columns)
    float* g = grad_dev ? grad_dev : q->grad;

    st = refresh_transposes(q, s);
    if (st != BMPL_OK) return st;
    // forward, keeping pre-activations; scores in q->logits
    st = embed_rows(q, B_dev, ldb, p, nullptr, 0, s);
    if (st == BMPL_OK) st = layers(q, p, true, q->logits, mpad, s);
    if (st != BMPL_OK) return st;
    // output layer: dS (in place of the scores, float32) and its bfloat16 copy
    HIPC(mlp_bce_grad(q->logits, mpad, q->ds16, mpad, m, mpad, p, supp_dev, ld_supp, supp_len_dev, (float)pos_weight,
                      q->rowloss, loss_dev, s));
    HIPC(mlp_colsum(q->logits, mpad, p, m, g + q->ob3, s));                          // db3
    HIPC(mlp_transpose(q->ds16, mpad, p, m, q->tds, capP, s));
    HIPC(mlp_transpose(q->h2, h, p, h, q->th2, capP, s));
    HIPC(mlp_gemm_store(q->tds, capP, m, q->th2, capP, h, kB, g + q->oW3, h, nullptr, s));   // dW3 = dS^T H2
    // second layer: dU2 = (dS W3) * gelu'(U2)
    HIPC(mlp_gemm_gelu_back(q->ds16, mpad, p, q->w3t, mpad, h, mpad, q->u2, h, q->du2, h, q->du2_16, h, s));
    HIPC(mlp_colsum(q->du2, h, p, h, g + q->ob2, s));                                // db2
    HIPC(mlp_transpose(q->du2_16, h, p, h, q->tdu, capP, s));
    HIPC(mlp_transpose(q->h1, h, p, h, q->th1, capP, s));
    HIPC(mlp_gemm_store(q->tdu, capP, h, q->th1, capP, h, kB, g + q->oW2, h, nullptr, s));   // dW2 = dU2^T H1
    // first layer: dU1 = (dU2 W2) * gelu'(U1)
    HIPC(mlp_gemm_gelu_back(q->du2_16, h, p, q->w2t, h, h, h, q->u1, h, q->du1, h, q->du1_16, h, s));
    HIPC(mlp_colsum(q->du1, h, p, h, g + q->ob1, s));                                // db1
    HIPC(mlp_transpose(q->du1_16, h, p, h, q->tdu, capP, s));
    HIPC(mlp_transpose(q->x0, d, p, d, q->tx0, capP, s));
    HIPC(mlp_gemm_store(q->tdu, capP, h, q->tx0, capP, d, kB, g + q->oW1, d, nullptr, s));   // dW1 = dU1^T Z
    return BMPL_OK;
}

bmpl_status bmpl_mlp_adam_step(bmpl_mlp* q, const float* grad_dev, const bmpl_adam* hp, void* hip_stream)
{
    if (!q || !hp) return fail(BMPL_E_INVALID, "bmpl_mlp_adam_step: NULL argument");
    if (!(hp->lr > 0.0) || !(hp->beta1 >= 0.0 && hp->beta1 < 1.0) || !(hp->beta2 >= 0.0 && hp->beta2 < 1.0) ||
        !(hp->eps > 0.0))
        return fail(BMPL_E_INVALID, "bmpl_mlp_adam_step: need lr > 0, beta1, beta2 in [0, 1), eps > 0");
    q->t += 1;
    const double bc1 = 1.0 - std::pow(hp->beta1, (double)q->t);
    const double bc2 = 1.0 - std::pow(hp->beta2, (double)q->t);
    HIPC(mlp_adam(q->master, q->m1, q->m2, grad_dev ? grad_dev : q->grad, q->w16, q->count, (float)hp->lr,
                  (float)hp->beta1, (float)hp->beta2, (float)hp->eps, (float)bc1, (float)bc2,
                  reinterpret_cast<hipStream_t>(hip_stream)));
    q->wt_stale = true;
    return BMPL_OK;
}

bmpl_status bmpl_mlp_propose(bmpl_mlp* q, const float* B_dev, int64_t ldb, int32_t p, int32_t k, int32_t* idx_dev,
                             int32_t ld_idx, void* hip_stream)
{
    bmpl_status st = check_signals(q, B_dev, ldb, p, "bmpl_mlp_propose");
    if (st != BMPL_OK) return st;
    if (k < 1 || k > 256 || ld_idx < k || (p > 0 && !idx_dev))
        return fail(BMPL_E_INVALID, "bmpl_mlp_propose: need 1 <= k=%d <= 256, ld_idx >= k and an output", k);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    for (int r0 = 0; r0 < p; r0 += q->cap) {
        const int rows = std::min(q->cap, p - r0);
        st = embed_rows(q, B_dev + (int64_t)r0 * ldb, ldb, rows, nullptr, 0, s);
        if (st == BMPL_OK) st = layers(q, rows, false, q->logits, q->mpad, s);
        if (st != BMPL_OK) return st;
        HIPC(mlp_topk(q->logits, q->mpad, rows, q->m, k, idx_dev + (int64_t)r0 * ld_idx, ld_idx, s));
    }
    return BMPL_OK;
}

bmpl_status bmpl_topk(const float* S_dev, int64_t lds, int32_t rows, int32_t L, int32_t k, int32_t* idx_dev,
                      int32_t ld_idx, void* hip_stream)
{
    if (rows < 0 || L < 1 || lds < L || k < 1 || k > 256 || ld_idx < k)
        return fail(BMPL_E_INVALID, "bmpl_topk: bad rows=%d L=%d lds=%lld k=%d ld_idx=%d", rows, L, (long long)lds, k,
                    ld_idx);
    if ((size_t)L * 4 > TOPK_MAX_LDS) return fail(BMPL_E_INVALID, "bmpl_topk: L=%d above %zu", L, TOPK_MAX_LDS / 4);
    if (rows > 0 && (!S_dev || !idx_dev)) return fail(BMPL_E_INVALID, "bmpl_topk: NULL pointer");
    HIPC(mlp_topk(S_dev, lds, rows, L, k, idx_dev, ld_idx, reinterpret_cast<hipStream_t>(hip_stream)));
    return BMPL_OK;
}

}  // extern "C"
