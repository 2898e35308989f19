// Host side of the C ABI (include/bmpl.h): context, workspace management and
// the outer loop of the batched pursuit (Algorithm 1 run over all signals).
//
// Per outer iteration, on the caller's stream:
//   corr_gemm   G = A^T Xi for the running signals (worst-case analysis, step 3)
//   select      J_t per signal: top-rho violators of |g_j| <= lambda outside I
//   status      stop test (natural stop, Eq. (9); caps) and compaction of the running list
//   solve       master problem Eq. (7) on I_t = I_{t-1} u J_t, residual xi^t (steps 4-8)
// The running count is read back once per iteration to size the next grids.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bmpl.h"
#include "bmpl_internal.h"
#include "classify.h"
#include "host_util.h"
#include "pursuit.h"
#include "qroute.h"

using namespace bmpl;

namespace {

constexpr int WARM_KL = 64;        // LDS factor capacity of the master solve right after a warm start
constexpr int RESCORE_LDS_SMALL = 512;   // candidates per signal in the first re-score pass's LDS
constexpr int CANDCAP_DEF = 4096;  // screening candidates per signal
constexpr int CAND8 = 64;          // e4m3-ranked candidates re-scored per signal (at most; 2 rho are used)

// Device scratch of bmpl_correlate_noalloc (staged residuals and their reduced-precision copies).  Each
// device holds its own copy; host code uses the per-device address from hipGetSymbolAddress, never the
// array's name.
static __device__ __align__(256) unsigned char scratch[BMPL_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {};   // per device, looked up once

// The current device's address of `scratch` (looked up on first use per device; the device is current).
bmpl_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= 64) return fail(BMPL_E_UNSUPPORTED, "device %d out of the supported range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BMPL_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return BMPL_OK;
}

// Rows 0..p-1 of dst = the residuals r_i = R + i ldr (n values, zeros up to kpad); row p all zero.
__global__ __launch_bounds__(256) void stage_rows_kernel(const float* __restrict__ R, int64_t ldr, int n, int p,
                                                         float* __restrict__ dst, int kpad)
{
    const int i = blockIdx.x;
    float* d = dst + (int64_t)i * kpad;
    for (int r = threadIdx.x; r < kpad; r += 256) d[r] = (i < p && r < n) ? R[(int64_t)i * ldr + r] : 0.0f;
}

}  // namespace

struct bmpl_ctx {
    int device = 0;
    int n = 0, m = 0, kpad = 0;
    float* At = nullptr;          // [m][kpad] float32 dictionary, atom-major
    double* Q = nullptr;          // [m][m] float64 Gram table A^T A, or null
    uint16_t* A16 = nullptr;      // [m + 1][kpad] bfloat16 dictionary (screening), row m zero
    uint16_t* A16p = nullptr;     // the same in the matrix instruction's fragment order (packed_bf16_elems)
    uint8_t* A8 = nullptr;        // [m + 1][kpad] e4m3 dictionary (FP8 ranking), row m zero
    float* ascale8 = nullptr;     // [m + 1] power-of-two scale per e4m3 atom
    int* cand8 = nullptr;         // [p_cap][CAND8] e4m3-ranked candidates
    int* ncand8 = nullptr;        // [p_cap]
    float* vmax8 = nullptr;       // [p_cap] scratch of the ranking pass
    double* zeros = nullptr;      // [p_cap] zero thresholds for the ranking pass
    int* cert = nullptr;          // [p_cap] left for the certified pass
    int* cert32 = nullptr;        // [p_cap] float32 product: rows whose stop needs the exact re-score
    int* n_cert32 = nullptr;      // their count
    int* grow_list = nullptr;     // [p_cap] signals whose slot block grows before the next master problem
    int* n_grow = nullptr;        // their count
    unsigned long long* grow_off = nullptr;   // [p_cap] their new blocks' offsets from arena->grow_base
    int* cert_act = nullptr;      // [p_cap] compacted list of those signals
    int* n_cert_dev = nullptr;    // its length
    double band_x = 0.0, band_dx = 0.0;   // bfloat16 band: eps_i = band_x ||xi_i|| + band_dx ||bf16(xi_i) - xi_i||
    double band32 = 0.0;          // float32 product: |g~_j - g_j| <= band32 ||xi_i|| (2 n 2^-24 max_j ||a_j||)
    int* spill = nullptr;         // [p_cap] re-score rows left to the second pass (row + 1, 0 = none)
    int* spill_act = nullptr;     // [p_cap] their signals
    int* n_spill_dev = nullptr;   // their count
    int* cand = nullptr;          // [p_cap][CANDCAP] screening candidates
    int* ncand = nullptr;         // [p_cap]
    uint16_t* diag16 = nullptr;   // bfloat16 staging of bmpl_correlate
    size_t lds_dyn_max = 0;       // dynamic LDS a solve workgroup may use (bytes)
    bool block_append = false;    // inverse-factor appends in blocks (BMPL_FLAG_BLOCK_APPEND sets it)
    bool qroute = false;          // correlation as beta - Q_{:,S} x_S after the first pass (BMPL_FLAG_Q_ROUTE)
    double* beta = nullptr;       // [p_cap][ldg] beta = A^T b in float64 (Q-route)
    bmpl_lambda_mode mode = BMPL_LAMBDA_ABS;
    double lambda = 0.0;
    bmpl_options opt{};

    // per-signal workspace
    Workspace w{};
    int p_cap = 0;
    int selcap = 0;
    // arena of the per-signal slot blocks (device state, its chunks, and pinned host views)
    Arena* arena_dev = nullptr;
    Arena* h_arena = nullptr;     // pinned: the chunk list as the host last wrote it
    Arena* h_arena_rd = nullptr;  // pinned: top / starved / reserve read back with the running count
    unsigned long long arena_total = 0;   // doubles over all chunks
    float* Bw = nullptr;          // [p_cap][kpad]
    float* Gc = nullptr;          // [p_cap][ldg] correlations
    int64_t ldg = 0;
    int* act[2] = {nullptr, nullptr};
    int* n_act_dev = nullptr;     // [2] running counts (inside the arena header)
    int* h_count = nullptr;       // pinned host int

    // correlation tile shape per running-signal bucket (>= 512, 64..511, < 64), set by bmpl_autotune
    int corr_shape[3] = {0, 3, 4};
    int corr_variant(int n_act) const { return corr_shape[n_act >= 512 ? 0 : (n_act >= 64 ? 1 : 2)]; }

    // diagnostic correlate staging
    float* diagR = nullptr;
    int diag_cap = 0;
    unsigned char* scratch = nullptr;   // this device's address of the no-allocation scratch

    // kernel timing (BMPL_FLAG_TIMING)
    bmpl_timing timing{};
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Span { size_t a, b; int kind; double flops, bytes, roof_ms; };
    std::vector<Span> spans;
    uint64_t* phase_dev = nullptr;     // [15] solve-kernel phase ticks and counters
    int wall_khz = 0;

    // graph capture of iteration segments (BMPL_FLAG_GRAPH)
    hipStream_t cap_stream = nullptr;
    long ws_gen = 0;                   // bumped whenever workspace buffers move
    // A segment's kernels bake in the bounds on |I| of each of its iterations, which follow from the
    // bound at the segment's start (i0) and its end (kl, clamped to max_active): both are in the key.
    struct GraphKey {
        int p, cur, i0, kl, shapes[3];
        long gen;
        int variant;  // bit 0: the large tile also covers the middle count bucket; bit 1: a 2-iteration segment;
                      // bit 2: the whole solve (i0 = -1 - warm_k, kl = max_outer)
        bool operator==(const GraphKey& o) const
        {
            return p == o.p && cur == o.cur && i0 == o.i0 && kl == o.kl && gen == o.gen &&
                   shapes[0] == o.shapes[0] && shapes[1] == o.shapes[1] && shapes[2] == o.shapes[2] &&
                   variant == o.variant;
        }
    };
    struct GraphEntry { GraphKey key; hipGraph_t g; hipGraphExec_t ge; };
    std::vector<GraphEntry> graphs;
};

namespace {

enum { K_CORR = 0, K_SELECT = 1, K_SOLVE = 2, K_OTHER = 3 };

bool timing_on(const bmpl_ctx* c) { return (c->opt.flags & BMPL_FLAG_TIMING) != 0; }

// Record an event on `s` (timing mode only); returns its pool index.
size_t mark(bmpl_ctx* c, hipStream_t s)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
        c->ev_pool.push_back(e);
    }
    size_t i = c->ev_used++;
    if (hipEventRecord(c->ev_pool[i], s) != hipSuccess) return (size_t)-1;
    return i;
}

void span(bmpl_ctx* c, size_t a, size_t b, int kind, double flops = 0.0, double bytes = 0.0, double roof_ms = 0.0)
{
    if (a != (size_t)-1 && b != (size_t)-1) c->spans.push_back({a, b, kind, flops, bytes, roof_ms});
}

// Fold the recorded spans of one solve into the totals (the stream must be idle).
void fold_timing(bmpl_ctx* c, size_t first, size_t last)
{
    for (const auto& sp : c->spans) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pool[sp.a], c->ev_pool[sp.b]) != hipSuccess) continue;
        switch (sp.kind) {
        case K_CORR:
            c->timing.corr_ms += ms; c->timing.corr_launches++;
            c->timing.corr_flops += sp.flops; c->timing.corr_bytes += sp.bytes;
            c->timing.corr_roof_ms += sp.roof_ms;
            break;
        case K_SELECT: c->timing.select_ms += ms; c->timing.select_launches++; break;
        case K_SOLVE: c->timing.solve_ms += ms; c->timing.solve_launches++; break;
        default: c->timing.other_ms += ms; break;
        }
    }
    float wall = 0.f;
    if (first != (size_t)-1 && last != (size_t)-1 &&
        hipEventElapsedTime(&wall, c->ev_pool[first], c->ev_pool[last]) == hipSuccess)
        c->timing.wall_ms += wall;
    c->timing.solves++;
    c->spans.clear();
    c->ev_used = 0;
}

}  // namespace

namespace {

void free_signals(bmpl_ctx* c)
{
    Workspace& w = c->w;
    dfree(w.R); dfree(w.bnorm2); dfree(w.lam); dfree(w.status); dfree(w.iters); dfree(w.nI);
    dfree(w.nS); dfree(w.nsel); dfree(w.sel); dfree(w.vmax); dfree(w.kkt_on); dfree(w.obj);
    dfree(w.kkt); dfree(w.inI); dfree(w.glazy); dfree(w.jadd); dfree(w.obj_prev); dfree(w.rr2); dfree(w.g0max);
    dfree(w.cap); dfree(w.blk);
    dfree(c->Bw); dfree(c->Gc); dfree(c->act[0]); dfree(c->act[1]);
    dfree(w.R16); dfree(w.rnorm); dfree(w.dxnorm); dfree(c->cand); dfree(c->ncand);
    dfree(w.R8); dfree(w.rscale8); dfree(c->cand8); dfree(c->ncand8); dfree(c->vmax8); dfree(c->zeros);
    dfree(c->cert); dfree(c->cert_act); dfree(c->n_cert_dev);
    dfree(c->spill); dfree(c->spill_act); dfree(c->n_spill_dev);
    dfree(c->cert32); dfree(c->n_cert32); dfree(c->grow_list); dfree(c->n_grow); dfree(c->grow_off);
    dfree(c->beta);
    c->p_cap = 0;
}

// Add a chunk of at least `min_doubles` (preferably `want_doubles`) to the slot-block arena; the
// device sees the new chunk list from the next kernel on `s` on.
bmpl_status arena_add(bmpl_ctx* c, unsigned long long min_doubles, unsigned long long want_doubles, hipStream_t s)
{
    Arena& H = *c->h_arena;
    if (H.nchunks >= ARENA_CHUNKS)
        return fail(BMPL_E_NOMEM, "slot-block arena: all %d chunks in use", ARENA_CHUNKS);
    double* p = nullptr;
    unsigned long long sz = std::max(want_doubles, min_doubles);
    hipError_t e = dalloc(&p, (size_t)sz);
    if (e != hipSuccess && sz > min_doubles) {
        (void)hipGetLastError();
        sz = min_doubles;
        e = dalloc(&p, (size_t)sz);
    }
    if (e != hipSuccess)
        return fail(BMPL_E_NOMEM, "slot-block arena: allocating %.3g GB failed: %s", 8.0 * sz / 1e9,
                    hipGetErrorString(e));
    const int k = H.nchunks;
    H.base[k] = p;
    H.start[k] = k ? H.start[k - 1] + H.size[k - 1] : 0;
    H.size[k] = sz;
    H.nchunks = k + 1;
    c->arena_total += sz;
    // the chunk list only (top, starved and reserve stay as the device has them)
    const size_t off = offsetof(Arena, nchunks);
    HIPC(hipMemcpyAsync(reinterpret_cast<char*>(c->arena_dev) + off, reinterpret_cast<char*>(c->h_arena) + off,
                        sizeof(Arena) - off, hipMemcpyHostToDevice, s));
    return BMPL_OK;
}

// Make sure `need` doubles of slot blocks (with a margin for chunk tails) can be handed out after the
// first `used` doubles of this solve.  `used` may lie past the chunks' end: the stop test places the
// grow list's blocks before the host adds room, and a block placed past the end lies in the next chunk
// once it is added (grow_kernel finds it there), so the offset is never moved back.
bmpl_status arena_ensure(bmpl_ctx* c, unsigned long long used, unsigned long long need, hipStream_t s)
{
    const unsigned long long want = need + need / 8 + (1ull << 20);
    if (c->arena_total >= used + want) return BMPL_OK;
    const unsigned long long missing = used + want - c->arena_total;
    return arena_add(c, missing, std::max(missing, c->arena_total / 4), s);
}

// Doubles of slot blocks one signal may take while |I| grows from nI (capacity K) by `iters` passes of
// up to `rho_pass` atoms (the first of them adding `first` atoms): the growth steps of the solve kernel.
unsigned long long block_reserve(int K, int nI, int first, int iters, int rho_pass, int slack, int kcap, int n)
{
    unsigned long long r = 0;
    int need = std::min(kcap, nI + first);
    for (int t = 0; t < iters; ++t) {
        while (K < need) {
            K = grow_capacity(K, std::min(need, K + std::max(1, rho_pass)), slack, kcap);
            r += (unsigned long long)block_doubles(K, n);
        }
        need = std::min(kcap, need + rho_pass);
    }
    return r;
}

// Size the per-signal workspace for p signals and selection capacity selcap.
bmpl_status ensure_workspace(bmpl_ctx* c, int p, int selcap)
{
    if (p <= c->p_cap && selcap <= c->selcap) return BMPL_OK;
    free_signals(c);
    Workspace& w = c->w;
    const size_t P = p;
    HIPC(dalloc(&w.R, (P + 1) * c->kpad));
    HIPC(hipMemset(w.R + P * c->kpad, 0, c->kpad * sizeof(float)));   // the correlation's zero row
    HIPC(dalloc(&w.bnorm2, P));
    HIPC(dalloc(&w.lam, P));
    HIPC(dalloc(&w.status, P));
    HIPC(dalloc(&w.iters, P));
    HIPC(dalloc(&w.nI, P));
    HIPC(dalloc(&w.nS, P));
    HIPC(dalloc(&w.nsel, P));
    HIPC(dalloc(&w.sel, P * selcap));
    HIPC(dalloc(&w.vmax, P));
    HIPC(dalloc(&w.kkt_on, P));
    HIPC(dalloc(&w.obj, P));
    HIPC(dalloc(&w.obj_prev, P));
    HIPC(dalloc(&w.rr2, P));
    HIPC(dalloc(&w.g0max, P));
    HIPC(dalloc(&w.kkt, P));
    HIPC(dalloc(&w.inI, P * w.words));
    HIPC(dalloc(&w.glazy, P));
    HIPC(dalloc(&w.jadd, P));
    HIPC(dalloc(&w.cap, P));
    HIPC(dalloc(&w.blk, P));
    w.arena = c->arena_dev;
    HIPC(dalloc(&c->Bw, P * c->kpad));
    HIPC(dalloc(&c->Gc, P * (size_t)c->ldg));
    HIPC(dalloc(&c->act[0], P));
    HIPC(dalloc(&c->act[1], P));
    HIPC(dalloc(&c->cert32, P));
    HIPC(dalloc(&c->n_cert32, 1));
    HIPC(dalloc(&c->grow_list, P));
    HIPC(dalloc(&c->grow_off, P));
    HIPC(dalloc(&c->n_grow, 1));
    HIPC(hipMemset(c->n_grow, 0, sizeof(int)));
    HIPC(hipMemset(c->n_cert32, 0, sizeof(int)));
    if (c->opt.screen != BMPL_PREC_FP32) {
        HIPC(dalloc(&w.R16, (P + 1) * c->kpad));
        HIPC(hipMemset(w.R16 + P * c->kpad, 0, c->kpad * sizeof(uint16_t)));
        HIPC(dalloc(&w.rnorm, P));
        HIPC(dalloc(&w.dxnorm, P));
        HIPC(dalloc(&c->cand, P * CANDCAP_DEF));
        HIPC(dalloc(&c->ncand, P));
        HIPC(dalloc(&c->spill, P));
        HIPC(dalloc(&c->spill_act, P));
        HIPC(dalloc(&c->n_spill_dev, 1));
    }
    if (c->qroute) HIPC(dalloc(&c->beta, P * (size_t)c->ldg));
    if (c->opt.screen == BMPL_PREC_FP8) {
        HIPC(dalloc(&w.R8, (P + 1) * c->kpad));
        HIPC(hipMemset(w.R8 + P * c->kpad, 0, c->kpad));
        HIPC(dalloc(&w.rscale8, P + 1));
        const float one = 1.0f;
        HIPC(hipMemcpy(w.rscale8 + P, &one, sizeof(float), hipMemcpyHostToDevice));
        HIPC(dalloc(&c->cand8, P * CAND8));
        HIPC(dalloc(&c->ncand8, P));
        HIPC(dalloc(&c->vmax8, P));
        HIPC(dalloc(&c->zeros, P));
        HIPC(hipMemset(c->zeros, 0, P * sizeof(double)));
        HIPC(dalloc(&c->cert, P));
        HIPC(dalloc(&c->cert_act, P));
        HIPC(dalloc(&c->n_cert_dev, 1));
    }
    c->p_cap = p;
    c->selcap = selcap;
    w.selcap = selcap;
    c->ws_gen++;
    return BMPL_OK;
}

constexpr int GRAPH_DEPTH = 4;   // outer iterations per captured segment (even: act buffers return)
constexpr size_t VEC_LDS_QUARTER = 38 * 1024;   // a quarter of a CU's 160 KB of LDS, less static LDS
constexpr int FULL_DEPTH_MAX = 64;   // the most iterations captured as one graph for a whole solve

void drop_graphs(bmpl_ctx* c)
{
    for (auto& e : c->graphs) {
        (void)hipGraphExecDestroy(e.ge);
        (void)hipGraphDestroy(e.g);
    }
    c->graphs.clear();
}

// The instantiated graph of one segment for this configuration, captured on first use by
// `enqueue(stream)` on the context's capture stream.
template <class F>
bmpl_status segment_graph(bmpl_ctx* c, int p, int cur, int i0, int kl, int variant, hipGraphExec_t* out,
                          F&& enqueue)
{
    bmpl_ctx::GraphKey key{p, cur, i0, kl, {c->corr_shape[0], c->corr_shape[1], c->corr_shape[2]}, c->ws_gen,
                           variant};
    for (auto& e : c->graphs)
        if (e.key == key) {
            *out = e.ge;
            return BMPL_OK;
        }
    if (c->graphs.size() >= 16) drop_graphs(c);
    if (!c->cap_stream) HIPC(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPC(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    bmpl_status st = enqueue(c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != BMPL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(BMPL_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(BMPL_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    c->graphs.push_back({key, g, ge});
    *out = ge;
    return BMPL_OK;
}

int default_max_active(const bmpl_ctx* c)
{
    return std::min(c->m, 2 * c->n);
}

}  // namespace

extern "C" {

bmpl_status bmpl_options_default(bmpl_options* o)
{
    if (!o) return fail(BMPL_E_INVALID, "bmpl_options_default: NULL options");
    o->rho = 10;
    o->max_outer = 0;
    o->max_active = 0;
    o->kkt_tol = 1e-4;
    o->screen = BMPL_PREC_FP32;
    o->flags = 0;
    o->omega = 1;
    o->eps_early = 0.0;
    o->r_inf_rel = 0.0;
    o->r2_rel = 0.0;
    return BMPL_OK;
}

const char* bmpl_last_error(const bmpl_ctx* c)
{
    (void)c;   // the message is per thread: it also describes failures that left no context (bmpl_create)
    return g_err.c_str();
}

bmpl_status bmpl_create(const float* A_dev, int64_t lda, int32_t n, int32_t m, bmpl_lambda_mode mode,
                        double lambda, const bmpl_options* o, void* hip_stream, bmpl_ctx** out)
{
    if (!out) return fail(BMPL_E_INVALID, "bmpl_create: NULL out");
    *out = nullptr;
    if (!A_dev) return fail(BMPL_E_INVALID, "bmpl_create: NULL A");
    if (n <= 0 || m <= 0 || lda < n)
        return fail(BMPL_E_INVALID, "bmpl_create: bad shape n=%d m=%d lda=%lld", n, m, (long long)lda);
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(BMPL_E_INVALID, "bmpl_create: lambda must be finite and >= 0");
    if (mode != BMPL_LAMBDA_ABS && mode != BMPL_LAMBDA_REL_MAX_ATB)
        return fail(BMPL_E_INVALID, "bmpl_create: unknown lambda mode %d", (int)mode);
    bmpl_options opt;
    bmpl_options_default(&opt);
    if (o) opt = *o;
    if (opt.rho <= 0 || opt.rho > 64) return fail(BMPL_E_INVALID, "bmpl_create: rho must be in [1, 64]");
    if (opt.omega < 1 || opt.omega * opt.rho > 64)
        return fail(BMPL_E_INVALID, "bmpl_create: omega must be >= 1 with omega * rho <= 64");
    if (!(opt.kkt_tol >= 0.0)) return fail(BMPL_E_INVALID, "bmpl_create: kkt_tol must be >= 0");
    if (!(opt.eps_early >= 0.0) || !(opt.r_inf_rel >= 0.0) || !(opt.r2_rel >= 0.0) || !std::isfinite(opt.eps_early)
        || !std::isfinite(opt.r_inf_rel) || !std::isfinite(opt.r2_rel))
        return fail(BMPL_E_INVALID, "bmpl_create: eps_early, r_inf_rel and r2_rel must be finite and >= 0");
    if (opt.screen != BMPL_PREC_FP32 && opt.screen != BMPL_PREC_BF16 && opt.screen != BMPL_PREC_FP8)
        return fail(BMPL_E_UNSUPPORTED, "bmpl_create: screening precision %d not available", (int)opt.screen);
    if (opt.max_active > m) opt.max_active = m;

    bmpl_ctx* c = new bmpl_ctx();
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { delete c; return fail(BMPL_E_HIP, "hipGetDevice: %s", hipGetErrorString(e)); }
    c->n = n;
    c->m = m;
    c->kpad = round_up(n, opt.screen == BMPL_PREC_FP8 ? 128 : 64);   // whole k stages of every product
    c->mode = mode;
    c->lambda = lambda;
    c->opt = opt;
    c->ldg = round_up(m, 64);
    c->w.n = n;
    c->w.kpad = c->kpad;
    c->w.m = m;
    c->w.words = (m + 31) / 32;
    e = dalloc(&c->At, (size_t)(m + 1) * c->kpad);   // row m stays zero
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->h_count), sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->h_arena), sizeof(Arena), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->h_arena_rd), sizeof(Arena), hipHostMallocDefault);
    if (e == hipSuccess) e = dalloc(reinterpret_cast<char**>(&c->arena_dev), sizeof(Arena));
    if (e == hipSuccess) {   // the no-allocation entry point's scratch: its address on this device
        void* sp = nullptr;
        if (scratch_address(c->device, &sp) != BMPL_OK) {
            const std::string msg = g_err;
            bmpl_destroy(c);
            return fail(BMPL_E_HIP, "bmpl_create: %s", msg.c_str());
        }
        c->scratch = static_cast<unsigned char*>(sp);
    }
    if (e == hipSuccess)   // the running counts live in the arena header: one read-back holds both
        c->n_act_dev = reinterpret_cast<int*>(reinterpret_cast<char*>(c->arena_dev) + offsetof(Arena, n_act));
    if (e == hipSuccess) {
        std::memset(c->h_arena, 0, sizeof(Arena));
        std::memset(c->h_arena_rd, 0, sizeof(Arena));
        e = hipMemcpyAsync(c->arena_dev, c->h_arena, sizeof(Arena), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemsetAsync(c->At, 0, (size_t)(m + 1) * c->kpad * sizeof(float), s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(c->At, c->kpad * sizeof(float), A_dev, lda * sizeof(float), n * sizeof(float), m,
                             hipMemcpyDeviceToDevice, s);
    // float32 product band: the deterministic bound 2 n 2^-24 ||a_j|| ||xi|| of an n-term float32 dot
    // product (products and sums rounded), with the largest atom norm and a 1 % margin
    if (e == hipSuccess) {
        float* norms = nullptr;
        e = dalloc(&norms, (size_t)3 * m);
        if (e == hipSuccess) e = launch_atom_norms(c->At, c->kpad, c->kpad, norms, m, s);
        std::vector<float> hn((size_t)m);
        if (e == hipSuccess) e = hipMemcpyAsync(hn.data(), norms, sizeof(float) * m, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (norms) (void)hipFree(norms);
        double amax = 0.0;
        for (int j = 0; j < m; ++j) amax = std::max(amax, (double)hn[j]);
        c->band32 = 2.0 * n * std::ldexp(1.0, -24) * amax * 1.01;
    }
    // bfloat16 copy of the dictionary and the factors of the screening band.
    if (e == hipSuccess && opt.screen != BMPL_PREC_FP32) {
        float* norms = nullptr;
        e = dalloc(&c->A16, (size_t)(m + 1) * c->kpad);
        if (e == hipSuccess) e = hipMemsetAsync(c->A16, 0, (size_t)(m + 1) * c->kpad * sizeof(uint16_t), s);
        if (e == hipSuccess) e = launch_to_bf16(c->At, c->kpad, c->A16, c->kpad, m, c->kpad, s);
        if (e == hipSuccess) e = dalloc(&c->A16p, packed_bf16_elems(m, c->kpad));
        if (e == hipSuccess) e = launch_pack_bf16(c->A16, c->kpad, m, c->kpad, c->A16p, s);
        if (e == hipSuccess) e = dalloc(&norms, (size_t)3 * m);
        if (e == hipSuccess) e = launch_atom_norms(c->At, c->kpad, c->kpad, norms, m, s);
        std::vector<float> hn((size_t)3 * m);
        if (e == hipSuccess) e = hipMemcpyAsync(hn.data(), norms, sizeof(float) * 3 * m, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (norms) (void)hipFree(norms);
        if (e == hipSuccess) {
            // |g~ - g| <= ||a^||  ||dx|| + ||da|| ||x|| + n 2^-24 ||a^|| (||x|| + ||dx||) with a^ = bf16(a),
            // da = a^ - a, dx = bf16(x) - x; maxima over the atoms, 1 % margin for the rounding of the norms
            double ahat = 0.0, da = 0.0;
            for (int j = 0; j < m; ++j) {
                ahat = std::max(ahat, (double)hn[(size_t)m + j]);
                da = std::max(da, (double)hn[(size_t)2 * m + j]);
            }
            const double acc = n * std::ldexp(1.0, -24);
            c->band_x = (da + acc * ahat) * 1.01;
            c->band_dx = ahat * (1.0 + acc) * 1.01;
        }
    }
    // e4m3 copy with per-atom power-of-two scales for the FP8 ranking product (row m zero, scale 1)
    if (e == hipSuccess && opt.screen == BMPL_PREC_FP8) {
        e = dalloc(&c->A8, (size_t)(m + 1) * c->kpad);
        if (e == hipSuccess) e = hipMemsetAsync(c->A8, 0, (size_t)(m + 1) * c->kpad, s);
        if (e == hipSuccess) e = dalloc(&c->ascale8, (size_t)m + 1);
        if (e == hipSuccess) e = launch_atoms_fp8(c->At, c->kpad, c->kpad, c->A8, c->ascale8, m, s);
        const float one = 1.0f;
        if (e == hipSuccess) e = hipMemcpyAsync(c->ascale8 + m, &one, sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    c->block_append = (opt.flags & BMPL_FLAG_BLOCK_APPEND) != 0;
    c->qroute = (opt.flags & BMPL_FLAG_Q_ROUTE) != 0;
    // Gram table Q = A^T A (float64) unless disabled or larger than the table budget.
    const double q_bytes = 8.0 * (double)m * (double)m;
    if (e == hipSuccess && !(opt.flags & BMPL_FLAG_NO_GRAM_TABLE) && q_bytes <= BMPL_GRAM_TABLE_MAX_BYTES) {
        e = dalloc(&c->Q, (size_t)m * (size_t)m);
        if (e == hipSuccess) e = launch_gram_table(c->At, c->kpad, m, c->kpad, c->Q, m, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && opt.omega > 1 && !c->Q) {
        bmpl_destroy(c);
        return fail(BMPL_E_UNSUPPORTED, "bmpl_create: subspace exploratory matching (omega > 1) needs the Gram "
                                        "table");
    }
    if (e == hipSuccess && c->qroute && (!c->Q || opt.screen != BMPL_PREC_FP32)) {
        bmpl_destroy(c);
        return fail(BMPL_E_UNSUPPORTED, "bmpl_create: the Q-route needs the Gram table (at most %.0f bytes, not "
                                        "disabled) and the float32 screen", (double)BMPL_GRAM_TABLE_MAX_BYTES);
    }
    if (e == hipSuccess) {
        int per_block = 0, optin = 0;
        hipFuncAttributes fa{};
        (void)hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
        if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, c->device) != hipSuccess)
            optin = 0;
        // the solve kernels get the largest dynamic LDS the device allows; the budget is the smallest
        size_t dyn = SIZE_MAX;
        for (const void* fn : {reinterpret_cast<const void*>(solve_kernel), reinterpret_cast<const void*>(solve_fold_kernel),
                               reinterpret_cast<const void*>(solve_block_kernel)}) {
            e = hipFuncGetAttributes(&fa, fn);
            if (e != hipSuccess) break;
            size_t total = (size_t)per_block;
            if (optin > per_block &&
                hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    optin - (int)fa.sharedSizeBytes) == hipSuccess)
                total = (size_t)optin;
            (void)hipGetLastError();
            dyn = std::min(dyn, total > fa.sharedSizeBytes + 256 ? total - fa.sharedSizeBytes - 256 : (size_t)0);
        }
        if (e == hipSuccess) c->lds_dyn_max = dyn;
    }
    if (e != hipSuccess) {
        bmpl_status st = fail(e == hipErrorOutOfMemory ? BMPL_E_NOMEM : BMPL_E_HIP, "bmpl_create: %s",
                              hipGetErrorString(e));
        bmpl_destroy(c);
        return st;
    }
    *out = c;
    return BMPL_OK;
}

bmpl_status bmpl_destroy(bmpl_ctx* c)
{
    if (!c) return BMPL_OK;
    free_signals(c);
    dfree(c->At);
    dfree(c->Q);
    dfree(c->A16);
    dfree(c->A16p);
    dfree(c->A8);
    dfree(c->ascale8);
    dfree(c->diag16);
    dfree(c->diagR);
    dfree(c->phase_dev);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->h_count) (void)hipHostFree(c->h_count);
    if (c->h_arena) {
        for (int k = 0; k < c->h_arena->nchunks; ++k) (void)hipFree(c->h_arena->base[k]);
        (void)hipHostFree(c->h_arena);
    }
    if (c->h_arena_rd) (void)hipHostFree(c->h_arena_rd);
    if (c->arena_dev) (void)hipFree(c->arena_dev);
    delete c;
    return BMPL_OK;
}

bmpl_status bmpl_correlate(bmpl_ctx* c, const float* R_dev, int64_t ldr, int32_t p, float* G_dev, int64_t ldg,
                           void* hip_stream)
{
    if (!c || !R_dev || !G_dev) return fail(BMPL_E_INVALID, "bmpl_correlate: NULL argument");
    if (p < 0 || ldr < c->n || ldg < c->m) return fail(BMPL_E_INVALID, "bmpl_correlate: bad shape");
    if (p == 0) return BMPL_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (p > c->diag_cap) {
        dfree(c->diagR);
        HIPC(dalloc(&c->diagR, (size_t)(p + 1) * c->kpad));
        c->diag_cap = p;
    }
    HIPC(hipMemsetAsync(c->diagR, 0, (size_t)(p + 1) * c->kpad * sizeof(float), s));
    HIPC(hipMemcpy2DAsync(c->diagR, c->kpad * sizeof(float), R_dev, ldr * sizeof(float), c->n * sizeof(float), p,
                          hipMemcpyDeviceToDevice, s));
    if (c->A8) {
        uint8_t* d8 = nullptr;
        float* sc8 = nullptr;
        hipError_t e = dalloc(&d8, (size_t)(p + 1) * c->kpad);
        if (e == hipSuccess) e = dalloc(&sc8, (size_t)p + 1);
        if (e == hipSuccess) e = launch_atoms_fp8(c->diagR, c->kpad, c->kpad, d8, sc8, p + 1, s);
        if (e == hipSuccess)
            e = launch_corr_gemm_fp8(c->corr_variant(p), c->A8, c->kpad, c->m, c->kpad, d8, c->kpad, nullptr,
                                     nullptr, p, G_dev, ldg, p, 0, 1 << 30, c->ascale8, sc8, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(d8);
        dfree(sc8);
        HIPC(e);
        return BMPL_OK;
    }
    if (c->A16) {
        dfree(c->diag16);
        HIPC(dalloc(&c->diag16, (size_t)(p + 1) * c->kpad));
        HIPC(launch_to_bf16(c->diagR, c->kpad, c->diag16, c->kpad, p + 1, c->kpad, s));
        HIPC(launch_corr_gemm_bf16(c->corr_variant(p), c->A16, c->A16p, c->kpad, c->m, c->kpad, c->diag16, c->kpad, nullptr,
                                   nullptr, p, G_dev, ldg, p, 0, 1 << 30, s));
        HIPC(hipStreamSynchronize(s));
        return BMPL_OK;
    }
    HIPC(launch_corr_gemm_f32(c->corr_variant(p), c->At, c->kpad, c->m, c->kpad, c->diagR, c->kpad, nullptr, nullptr, p, G_dev, ldg, p, 0, 1 << 30, s));
    return BMPL_OK;
}

bmpl_status bmpl_correlate_noalloc(bmpl_ctx* c, const float* R_dev, int64_t ldr, int32_t p, float* G_dev,
                                   int64_t ldg, void* hip_stream)
{
    if (!c || !R_dev || !G_dev) return fail(BMPL_E_INVALID, "bmpl_correlate_noalloc: NULL argument");
    if (p < 0 || ldr < c->n || ldg < c->m) return fail(BMPL_E_INVALID, "bmpl_correlate_noalloc: bad shape");
    if (p == 0) return BMPL_OK;
    // scratch layout: float32 rows [p + 1][kpad] | bfloat16 rows [p + 1][kpad] (bfloat16 screening) |
    // e4m3 rows [p + 1][kpad] and their scales [p + 1] (e4m3 ranking), each part 256-byte aligned
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t rows = (size_t)p + 1, kp = (size_t)c->kpad;
    const size_t o16 = al(rows * kp * sizeof(float));
    const size_t o8 = o16 + (c->A16 && !c->A8 ? al(rows * kp * sizeof(uint16_t)) : 0);
    const size_t os = o8 + (c->A8 ? al(rows * kp) : 0);
    const size_t need = os + (c->A8 ? al(rows * sizeof(float)) : 0);
    if (need > (size_t)BMPL_NOALLOC_SCRATCH_BYTES)
        return fail(BMPL_E_INVALID, "bmpl_correlate_noalloc: %d residuals of %d values need %zu bytes of scratch, "
                                    "more than BMPL_NOALLOC_SCRATCH_BYTES (%zu)", p, c->n, need,
                    (size_t)BMPL_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    float* stage = reinterpret_cast<float*>(c->scratch);
    hipLaunchKernelGGL(stage_rows_kernel, dim3(p + 1), dim3(256), 0, s, R_dev, ldr, c->n, p, stage, c->kpad);
    HIPC(hipGetLastError());
    if (c->A8) {
        uint8_t* r8 = c->scratch + o8;
        float* sc8 = reinterpret_cast<float*>(c->scratch + os);
        HIPC(launch_atoms_fp8(stage, c->kpad, c->kpad, r8, sc8, p + 1, s));
        HIPC(launch_corr_gemm_fp8(c->corr_variant(p), c->A8, c->kpad, c->m, c->kpad, r8, c->kpad, nullptr, nullptr, p,
                                  G_dev, ldg, p, 0, 1 << 30, c->ascale8, sc8, s));
        return BMPL_OK;
    }
    if (c->A16) {
        uint16_t* r16 = reinterpret_cast<uint16_t*>(c->scratch + o16);
        HIPC(launch_to_bf16(stage, c->kpad, r16, c->kpad, p + 1, c->kpad, s));
        HIPC(launch_corr_gemm_bf16(c->corr_variant(p), c->A16, c->A16p, c->kpad, c->m, c->kpad, r16, c->kpad, nullptr, nullptr,
                                   p, G_dev, ldg, p, 0, 1 << 30, s));
        return BMPL_OK;
    }
    HIPC(launch_corr_gemm_f32(c->corr_variant(p), c->At, c->kpad, c->m, c->kpad, stage, c->kpad, nullptr, nullptr, p,
                              G_dev, ldg, p, 0, 1 << 30, s));
    return BMPL_OK;
}

bmpl_status bmpl_select(bmpl_ctx* c, const float* G_dev, int64_t ldg, int32_t p, const double* lambda_dev,
                        const uint32_t* excl_dev, int32_t k, int32_t* sel_dev, int32_t* nsel_dev, float* vmax_dev,
                        void* hip_stream)
{
    if (!c || !G_dev || !lambda_dev || !sel_dev || !nsel_dev || !vmax_dev)
        return fail(BMPL_E_INVALID, "bmpl_select: NULL argument");
    if (p < 0 || ldg < c->m || k < 1 || k > 64) return fail(BMPL_E_INVALID, "bmpl_select: bad shape or k");
    if (p == 0) return BMPL_OK;
    SelectArgs a{};
    a.G = G_dev; a.ldg = ldg; a.m = c->m;
    a.act = nullptr; a.n_act_dev = nullptr; a.p_grid = p;
    a.lam = const_cast<double*>(lambda_dev); a.lam_rel = 0.0;
    a.excl = excl_dev; a.words = (c->m + 31) / 32;
    a.k = k; a.sel = sel_dev; a.selcap = k; a.nsel = nsel_dev; a.vmax = vmax_dev;
    a.nI = nullptr; a.max_active = 0;
    HIPC(launch_select(a, reinterpret_cast<hipStream_t>(hip_stream)));
    return BMPL_OK;
}

bmpl_status bmpl_solve(bmpl_ctx* c, const float* B_dev, int64_t ldb, int32_t p, const double* lambda_dev,
                       const int32_t* warm_idx_dev, int32_t warm_k, const bmpl_result* out, void* hip_stream)
{
    if (!c || !out) return fail(BMPL_E_INVALID, "bmpl_solve: NULL context or result");
    if (p < 0 || ldb < c->n) return fail(BMPL_E_INVALID, "bmpl_solve: bad p=%d or ldb=%lld", p, (long long)ldb);
    if (p == 0) return BMPL_OK;
    if (!B_dev) return fail(BMPL_E_INVALID, "bmpl_solve: NULL B");
    if (!out->x_val_dev || !out->x_idx_dev || !out->supp_len_dev)
        return fail(BMPL_E_INVALID, "bmpl_solve: x_val, x_idx and supp_len are required");
    const int max_active = c->opt.max_active > 0 ? c->opt.max_active : default_max_active(c);
    const int need_ld = std::min(max_active, c->n);
    if (out->ld_x < need_ld)
        return fail(BMPL_E_INVALID, "bmpl_solve: ld_x=%d < min(max_active, n)=%d", out->ld_x, need_ld);
    if (warm_k < 0 || warm_k > 256 || (warm_k > 0 && !warm_idx_dev))
        return fail(BMPL_E_INVALID, "bmpl_solve: warm_k must be in [0, 256] with a proposal array");
    const bool warm = warm_idx_dev && warm_k > 0;
    const int max_outer = c->opt.max_outer > 0 ? c->opt.max_outer : (c->m + c->opt.rho - 1) / c->opt.rho;
    // atoms selected per pass: rho, or omega rho candidates of which rho stay (subspace exploratory matching)
    const int rho = c->opt.rho * c->opt.omega;
    const int smpl_keep = c->opt.omega > 1 ? c->opt.rho : 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    // graph capture of whole segments; kernel timing needs per-launch events, so it uses the host loop
    const bool graph = (c->opt.flags & BMPL_FLAG_GRAPH) != 0 && !timing_on(c);

    const int first_add = warm ? std::max(warm_k, rho) : rho;
    const int slack = 2 * rho;   // slot-block growth: room for two more passes past the need
    bmpl_status st = ensure_workspace(c, std::max(p, c->p_cap), std::max(rho, warm ? warm_k : 0));
    if (st != BMPL_OK) return st;
    // Full depth: with an iteration cap of at most FULL_DEPTH_MAX, graph mode captures every pass of
    // the solve as one graph and gives each signal, at its first master problem, a slot block for the
    // largest |I| the cap allows (first_add + (max_outer - 1) rho), so nothing waits for the host: the
    // solve is enqueued and bmpl_solve returns without synchronising.  Used when those blocks take at
    // most the arena already held plus half of the free device memory; otherwise the segments below.
    int kfull = 0;
    if (graph && c->opt.max_outer > 0 && c->opt.max_outer <= FULL_DEPTH_MAX) {
        const int bound = std::min(max_active, first_add + (max_outer - 1) * rho);
        const int k = grow_capacity(0, bound, slack, max_active);
        const unsigned long long need = (unsigned long long)p * block_doubles(k, c->n);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        if (8.0 * (double)need <= 8.0 * (double)c->arena_total + 0.5 * (double)free_b) kfull = k;
    }
    const bool full = kfull > 0;
    // Slot blocks for every signal up to the first host read-back: the first master problem (a
    // proposal's atoms or rho) and, in graph mode, the iterations of the first segment; in full depth,
    // the whole solve.
    const int iters0 = (graph && !warm) ? 1 + GRAPH_DEPTH : 1;
    st = arena_ensure(c, 0, (unsigned long long)p *
                               (full ? (unsigned long long)block_doubles(kfull, c->n)
                                     : block_reserve(0, 0, first_add, iters0, rho, slack, max_active, c->n)), s);
    if (st != BMPL_OK) return st;
    Workspace& w = c->w;
    w.p = p;

    const bool rel = c->mode == BMPL_LAMBDA_REL_MAX_ATB && !lambda_dev;
    const bool tm = timing_on(c);
    c->spans.clear();
    c->ev_used = 0;
    const bool phases = tm && (c->opt.flags & BMPL_FLAG_PHASES);
    if (phases && !c->phase_dev) {
        HIPC(dalloc(&c->phase_dev, PHASE_SLOTS));
        HIPC(hipMemsetAsync(c->phase_dev, 0, PHASE_SLOTS * sizeof(uint64_t), s));
        HIPC(hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, c->device));
    }
    const size_t ev_first = tm ? mark(c, s) : (size_t)-1;
    PrepArgs pa{w, B_dev, ldb, c->Bw, lambda_dev, c->lambda, rel ? 1 : 0};
    hipLaunchKernelGGL(prep_kernel, dim3(p), dim3(256), 0, s, pa);
    HIPC(hipGetLastError());
    if (c->qroute) HIPC(launch_atb_f64(c->At, c->kpad, c->m, c->Bw, c->kpad, p, c->n, c->beta, c->ldg, s));

    StatusArgs sa{};
    sa.w = w; sa.act_in = nullptr; sa.n_in_dev = nullptr; sa.n_in = p;
    sa.act_out = c->act[0]; sa.n_out_dev = c->n_act_dev; sa.initial = 1;
    sa.max_outer = max_outer; sa.kkt_tol = c->opt.kkt_tol; sa.warm_check = 0;
    sa.eps_early = c->opt.eps_early; sa.r_inf_rel = c->opt.r_inf_rel; sa.r2_rel = c->opt.r2_rel;
    sa.rho = c->opt.rho;
    // slot-block reserve for the iterations up to the next read-back (a graph segment at most)
    sa.reserve_iters = full ? 0 : (graph ? GRAPH_DEPTH : 1); sa.rho_pass = rho; sa.slack = slack;
    sa.kcap = max_active;
    sa.clear_cert = c->n_cert32;
    sa.grow_list = c->grow_list; sa.n_grow = c->n_grow; sa.grow_off = c->grow_off; sa.kmin = kfull;
    hipLaunchKernelGGL(status_compact_kernel, dim3(1), dim3(1024), 0, s, sa);
    HIPC(hipGetLastError());
    // In graph mode the host does not wait for the running count until the first captured segment has
    // been launched: every kernel reads the count on the device, p bounds it, and the GPU runs set-up,
    // the first pass and the first segment back to back.
    int n_act = p;
    if (!graph) {
        HIPC(hipMemcpyAsync(c->h_count, c->n_act_dev, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        n_act = *c->h_count;
    }
    if (tm) span(c, ev_first, mark(c, s), K_OTHER);

    bool merge_mid = false;   // graph segments: see the gated product below
    // One pass of the worst-case analysis on the running list act[cur] (n_grid bounds its
    // size): correlation, selection, stop test and compaction into act[nxt].  With `gated`
    // every correlation tile shape is enqueued and each runs only for its own bucket of the
    // device-side count (graph capture); otherwise the shape of n_grid's bucket is used and,
    // in timing mode, every kernel is bracketed by events.
    auto enqueue_select_pass = [&](hipStream_t q, int cur, int n_grid, bool first, bool warm_check,
                                   bool gated) -> bmpl_status {
        const int nxt = 1 - cur;
        const bool ev = tm && !gated;
        // e4m3 ranking for every pass after the first; the first (the lambda rule) is certified in bfloat16
        const bool fp8 = c->A8 && !first;
        size_t e0 = ev ? mark(c, q) : 0;
        // One correlation product over a running list (prec 0 float32, 1 bfloat16, 2 e4m3).  Gated:
        // every tile shape is enqueued and runs only for its own bucket of the device-side count.
        auto product = [&](int prec, const int* lst, const int* cnt, bool gate) -> hipError_t {
            auto gemm = [&](int shape, int grid, int lo, int hi) -> hipError_t {
                if (prec == 2)
                    return launch_corr_gemm_fp8(shape, c->A8, c->kpad, c->m, c->kpad, w.R8, c->kpad, lst, cnt, grid,
                                                c->Gc, c->ldg, c->p_cap, lo, hi, c->ascale8, w.rscale8, q);
                if (prec == 1)
                    return launch_corr_gemm_bf16(shape, c->A16, c->A16p, c->kpad, c->m, c->kpad, w.R16, c->kpad, lst, cnt,
                                                 grid, c->Gc, c->ldg, c->p_cap, lo, hi, q);
                return launch_corr_gemm_f32(shape, c->At, c->kpad, c->m, c->kpad, w.R, c->kpad, lst, cnt, grid,
                                            c->Gc, c->ldg, c->p_cap, lo, hi, q);
            };
            if (gate) {
                // count buckets of the three tile shapes; in a segment that starts with 512 or more running
                // signals the large tile also takes the middle bucket (one launch less per iteration: the
                // count rarely falls that far within four iterations)
                const int lo[3] = {merge_mid ? 64 : 512, 64, 1}, hi[3] = {1 << 30, 512, 64};
                for (int b = 0; b < 3; ++b) {
                    if (b == 1 && merge_mid) continue;
                    const int grid = std::min(n_grid, hi[b] - 1);
                    if (grid < lo[b]) continue;
                    const hipError_t e = gemm(c->corr_shape[b], grid, lo[b], hi[b]);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }
            return gemm(c->corr_variant(n_grid), n_grid, 0, 1 << 30);
        };
        const bool qr = c->qroute && !first;
        if (qr) {
            QCorrArgs qa{w, c->Q, c->m, c->beta, c->ldg, c->act[cur], c->n_act_dev + cur, n_grid, c->Gc, c->ldg};
            HIPC(launch_q_corr(qa, q));
        } else {
            HIPC(product(fp8 ? 2 : (c->A16 ? 1 : 0), c->act[cur], c->n_act_dev + cur, gated));
        }
        if (ev) {
            const double mm = c->m, nn = c->n, pp = n_grid;
            const size_t e1 = mark(c, q);
            // algorithmic work of this launch: operands read once in their precision, correlations written
            // once in float32; its roofline time on MI355X (matrix peak of the precision, 8 TB/s HBM)
            const double eb = fp8 ? 1.0 : (c->A16 ? 2.0 : 4.0);
            const double peak = fp8 ? 5.0e15 : (c->A16 ? 2.5e15 : 157.3e12);
            const double fl = 2.0 * mm * nn * pp, by = eb * (mm * nn + nn * pp) + 4.0 * mm * pp;
            const double roof = std::max(fl / peak, by / 8.0e12) * 1e3;
            // the Q-route's work depends on the supports: its time is kept, its flops are not counted
            span(c, e0, e1, K_CORR, qr ? 0.0 : fl, qr ? 0.0 : by, qr ? 0.0 : roof);
            e0 = e1;
        }
        // certified bfloat16 screening of a list: band test, candidates, exact re-score and selection
        auto screen_pass = [&](const int* lst, const int* cnt) -> hipError_t {
            ScreenArgs sc{};
            sc.G = c->Gc; sc.ldg = c->ldg; sc.m = c->m;
            sc.act = lst; sc.n_act_dev = cnt; sc.p_grid = n_grid;
            sc.lam = w.lam; sc.lam_rel = (rel && first) ? c->lambda : 0.0;
            sc.rnorm = w.rnorm; sc.dxnorm = w.dxnorm; sc.band_x = c->band_x; sc.band_dx = c->band_dx;
            sc.excl = w.inI; sc.words = w.words;
            sc.k = rho; sc.nI = w.nI; sc.max_active = max_active;
            sc.cand = c->cand; sc.candcap = CANDCAP_DEF; sc.ncand = c->ncand;
            sc.clear_count = c->n_spill_dev;
            hipError_t e = launch_screen(sc, q);
            if (e != hipSuccess) return e;
            RescoreArgs rs{};
            rs.At = c->At; rs.lda = c->kpad; rs.kpad = c->kpad;
            rs.R = w.R; rs.ldr = c->kpad;
            rs.G = c->Gc; rs.ldg = c->ldg; rs.rnorm = w.rnorm; rs.dxnorm = w.dxnorm;
            rs.band_x = c->band_x; rs.band_dx = c->band_dx;
            rs.act = lst; rs.n_act_dev = cnt; rs.p_grid = n_grid;
            rs.cand = c->cand; rs.candcap = CANDCAP_DEF;
            rs.ncand = c->ncand;
            rs.lam = w.lam; rs.lam_rel = sc.lam_rel;
            rs.k = rho; rs.nI = w.nI; rs.max_active = max_active;
            rs.sel = w.sel; rs.selcap = w.selcap; rs.nsel = w.nsel; rs.vmax = w.vmax; rs.status = w.status;
            // first pass: up to RESCORE_LDS_SMALL candidate values (12 bytes each) in LDS, so many
            // workgroups fit a CU; the few signals with more go to a second pass over their list with
            // candidate values and the staged residual within 60 KB of LDS
            rs.candcap_lds = RESCORE_LDS_SMALL;
            rs.spill_row = c->spill; rs.row_of = nullptr;
            rs.spill_act = c->spill_act; rs.n_spill = c->n_spill_dev;   // appended in any order
            e = launch_rescore(rs, q);
            if (e != hipSuccess) return e;
            RescoreArgs r2 = rs;
            r2.candcap_lds = std::max(64, std::min(CANDCAP_DEF, (61440 - 4 * c->kpad) / 12 / 4 * 4));
            r2.act = c->spill_act; r2.n_act_dev = c->n_spill_dev;
            r2.spill_row = nullptr; r2.row_of = c->spill;
            return launch_rescore(r2, q);
        };
        SelectArgs a{};
        a.G = c->Gc; a.ldg = c->ldg; a.m = c->m;
        a.act = c->act[cur]; a.n_act_dev = c->n_act_dev + cur; a.p_grid = n_grid;
        a.lam = w.lam; a.lam_rel = (rel && first) ? c->lambda : 0.0;
        a.excl = w.inI; a.words = w.words;
        a.k = rho; a.sel = w.sel; a.selcap = w.selcap; a.nsel = w.nsel; a.vmax = w.vmax;
        a.nI = w.nI; a.max_active = max_active;
        if (fp8) {
            // ranking: the 2 rho largest |g~| outside I (zero threshold) ...
            SelectArgs r8 = a;
            r8.lam = c->zeros; r8.lam_rel = 0.0;
            r8.k = std::min(CAND8, 2 * rho); r8.sel = c->cand8; r8.selcap = CAND8; r8.nsel = c->ncand8;
            r8.vmax = c->vmax8;
            r8.clear_count = c->n_cert_dev;
            HIPC(launch_select(r8, q));
            // ... re-scored exactly; the exact violators among them are admitted
            Rank8Args rk{};
            rk.At = c->At; rk.lda = c->kpad; rk.kpad = c->kpad; rk.R = w.R; rk.ldr = c->kpad;
            rk.act = c->act[cur]; rk.n_act_dev = c->n_act_dev + cur; rk.p_grid = n_grid;
            rk.cand = c->cand8; rk.candcap = CAND8; rk.ncand = c->ncand8;
            rk.lam = w.lam; rk.k = rho; rk.nI = w.nI; rk.max_active = max_active;
            rk.sel = w.sel; rk.selcap = w.selcap; rk.nsel = w.nsel; rk.vmax = w.vmax; rk.cert = c->cert;
            // signals with no exact violator among their candidates go to cert_act (any order): the
            // certified bfloat16 pass decides them
            rk.cert_act = c->cert_act; rk.n_cert = c->n_cert_dev;
            HIPC(launch_rank8(rk, q));
            HIPC(product(1, c->cert_act, c->n_cert_dev, true));
            HIPC(screen_pass(c->cert_act, c->n_cert_dev));
        } else if (c->A16) {
            HIPC(screen_pass(c->act[cur], c->n_act_dev + cur));
        } else {
            a.rr2 = w.rr2; a.band = c->band32; a.cert_list = c->cert32; a.n_cert = c->n_cert32;
            HIPC(launch_select(a, q));
            // the natural stop certified against the float32 product's rounding (exact re-score of the
            // atoms within the band of lambda when nothing was admitted)
            CertifyArgs cf{};
            cf.G = c->Gc; cf.ldg = c->ldg; cf.m = c->m;
            cf.act = c->act[cur]; cf.n_act_dev = c->n_act_dev + cur; cf.p_grid = n_grid;
            cf.lam = w.lam; cf.rr2 = w.rr2; cf.band = c->band32;
            cf.excl = w.inI; cf.words = w.words;
            cf.At = c->At; cf.lda = c->kpad; cf.n = c->n;
            cf.R = w.R; cf.ldr = c->kpad;
            cf.k = rho; cf.nI = w.nI; cf.max_active = max_active;
            cf.sel = w.sel; cf.selcap = w.selcap; cf.nsel = w.nsel; cf.vmax = w.vmax;
            cf.cert_list = c->cert32; cf.n_cert = c->n_cert32;
            HIPC(launch_certify(cf, q));
        }
        if (ev) {
            const size_t e1 = mark(c, q);
            span(c, e0, e1, K_SELECT);
            e0 = e1;
        }
        if (first && warm) {
            WarmArgs wa{w, c->act[cur], c->n_act_dev + cur, warm_idx_dev, warm_k, max_active};
            hipLaunchKernelGGL(warm_select_kernel, dim3(n_grid), dim3(256), 0, q, wa);
            HIPC(hipGetLastError());
        }
        StatusArgs sb = sa;
        sb.w = w;
        sb.initial = 0;
        sb.act_in = c->act[cur]; sb.n_in_dev = c->n_act_dev + cur; sb.n_in = n_grid;
        sb.act_out = c->act[nxt]; sb.n_out_dev = c->n_act_dev + nxt;
        sb.warm_check = warm_check ? 1 : 0;
        hipLaunchKernelGGL(status_compact_kernel, dim3(1), dim3(1024), 0, q, sb);
        HIPC(hipGetLastError());
        if (ev) span(c, e0, mark(c, q), K_OTHER);
        return BMPL_OK;
    };

    // Master problem and residual for the running list act[idx] (steps 4-8 of Algorithm 1),
    // with the factor held in LDS for capacity kl when it fits.  A signal whose support outgrows kl
    // moves its factor to global memory inside the kernel and continues there (slower), so kl is
    // |I|'s bound for ordinary passes, where most of I is in S, and smaller after a warm start.
    // `explore`: the pass before selected omega rho candidates (not a warm-start proposal)
    // `ibound`: |I| after this pass's selection is at most this (the LDS vectors are sized by it)
    auto enqueue_master = [&](hipStream_t q, int idx, int n_grid, int kl, int ibound, bool gated,
                              bool explore) -> bmpl_status {
        const bool ev = tm && !gated;
        size_t e0 = ev ? mark(c, q) : 0;
        SolveArgs so{};
        so.w = w; so.At = c->At; so.lda = c->kpad; so.Bw = c->Bw;
        so.Q = c->Q; so.ldq = c->m;
        so.max_steps_per_slot = 16;
        so.smpl_keep = explore ? smpl_keep : 0;
        so.phase = phases ? c->phase_dev : nullptr;
        // the exploratory pass of SMPL briefly holds omega rho new slots: the full capacity then
        so.kv = std::min(max_active, std::max(1, ibound));
        const int kp = std::max(std::min(so.kv, c->n), so.smpl_keep > 0 ? rho : 1);   // |S| <= n
        so.kp = kp;
        const size_t vec_bytes = vec_area_bytes(so.kv, kp);
        const size_t stage = c->Q ? 0 : GRAM_STAGE_BYTES;   // direct Gram staging, only without the table
        so.kl = std::min(kl, so.kv);
        const size_t rinv_bytes = 8 * (size_t)tri(so.kl);
        // With the factor in LDS the vectors go there too.  With a factor in global memory, vectors of
        // more than a quarter of the CU's LDS would cap the workgroups per CU below the four the kernel's
        // registers allow, and the latency-bound solve gains more from the extra workgroups than it
        // loses to vectors in global memory (4096-signal ragged batch: 13.2 -> 12.4 s).
        const bool rinv_fits = vec_bytes + rinv_bytes + stage <= c->lds_dyn_max;
        so.vec_lds = vec_bytes + stage <= (rinv_fits ? c->lds_dyn_max : std::min(c->lds_dyn_max, VEC_LDS_QUARTER)) ? 1 : 0;
        so.rinv_lds = (so.vec_lds && rinv_fits) ? 1 : 0;
        size_t lds = (so.rinv_lds ? rinv_bytes : 0) + (so.vec_lds ? vec_bytes : 0) + stage;
        // block appends pay off when the factor streams from global memory; with an LDS-resident
        // factor single appends are cheaper and keep the workgroup's LDS (and occupancy) smaller
        so.zs_lds = (c->block_append && !so.rinv_lds && lds + block_scratch_bytes(kp) <= c->lds_dyn_max) ? 1 : 0;
        if (so.zs_lds) lds += block_scratch_bytes(kp);
        so.act = c->act[idx]; so.n_act_dev = c->n_act_dev + idx;
        GrowArgs ga{w, c->grow_list, c->n_grow, c->grow_off, slack, max_active, kfull};
        hipLaunchKernelGGL(grow_kernel, dim3(std::min(n_grid, 512)), dim3(256), 0, q, ga);
        HIPC(hipGetLastError());
        // factors that start in global memory take the kernel whose appends and solves read them in
        // one pass (its larger register footprint stays out of the LDS-factor kernel)
        if (so.zs_lds)
            hipLaunchKernelGGL(solve_block_kernel, dim3(n_grid), dim3(256), lds, q, so);
        else if (!so.rinv_lds)
            hipLaunchKernelGGL(solve_fold_kernel, dim3(n_grid), dim3(256), lds, q, so);
        else
            hipLaunchKernelGGL(solve_kernel, dim3(n_grid), dim3(256), lds, q, so);
        HIPC(hipGetLastError());
        if (ev) span(c, e0, mark(c, q), K_SOLVE);   // the residual is the solve kernel's last step
        return BMPL_OK;
    };
    // The running count and the arena's state (blocks handed out, failed requests, the reserve the
    // running signals may need before the next read-back), then arena space for that reserve.
    auto read_count = [&](int idx) -> bmpl_status {
        HIPC(hipMemcpyAsync(c->h_arena_rd, c->arena_dev, offsetof(Arena, nchunks), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        n_act = c->h_arena_rd->n_act[idx];
        const Arena& R = *c->h_arena_rd;
        if (R.starved) HIPC(hipMemsetAsync(&c->arena_dev->starved, 0, sizeof(unsigned long long), s));
        if (n_act == 0) return BMPL_OK;
        // the offset stays where it is, also past the chunks' end (blocks placed there by the stop test
        // become valid in the chunk added next)
        return arena_ensure(c, R.top, R.reserve, s);
    };

    // Iteration 0: lambda rule and the first selection (or the warm-start proposal).
    int cur = 0;
    if (n_act > 0) {
        c->timing.outer_iters += tm ? 1 : 0;
        st = enqueue_select_pass(s, 0, n_act, true, false, false);
        if (st != BMPL_OK) return st;
        cur = 1;
        if (!graph || (warm && !full)) {
            st = read_count(cur);
            if (st != BMPL_OK) return st;
        }
    }
    if (full && n_act > 0) {
        // every pass of the solve in one graph: max_outer master problems and selection passes (the stop
        // test stops each signal by then); passes after the last signal's stop are empty launches
        merge_mid = false;
        hipGraphExec_t ge = nullptr;
        st = segment_graph(c, p, cur, -1 - (warm ? warm_k : 0), max_outer, 4, &ge, [&](hipStream_t q) -> bmpl_status {
            int cc = cur, im = 0;
            for (int d = 0; d < max_outer; ++d) {
                const bool wd = warm && d == 0;   // the master problem on a warm start's proposal
                im = std::min(max_active, im + (wd ? first_add : rho));
                bmpl_status r = enqueue_master(q, cc, p, wd ? std::min(im, WARM_KL) : im, im, true, !wd);
                if (r != BMPL_OK) return r;
                r = enqueue_select_pass(q, cc, p, false, wd, true);
                if (r != BMPL_OK) return r;
                cc = 1 - cc;
            }
            return BMPL_OK;
        });
        if (st != BMPL_OK) return st;
        HIPC(hipGraphLaunch(ge, s));
        n_act = 0;
    }
    // Then per iteration: master problem on I_t, next selection pass.
    int imax = 0;
    bool after_warm = warm;
    while (n_act > 0) {
        if (graph && !after_warm) {
            // GRAPH_DEPTH iterations as one captured graph launch (two once fewer than 64 signals run: the
            // last few usually stop within two).  The kernels read the running count on the device, so
            // iterations past the last signal's stop are empty launches.
            const int depth = n_act < 64 ? 2 : GRAPH_DEPTH;
            const int need = std::min(max_active, imax + depth * rho);
            hipGraphExec_t ge = nullptr;
            merge_mid = n_act >= 512;
            st = segment_graph(c, p, cur, imax, need, (merge_mid ? 1 : 0) | (depth == 2 ? 2 : 0), &ge,
                               [&](hipStream_t q) -> bmpl_status {
                int cc = cur;
                for (int d = 0; d < depth; ++d) {
                    // factor capacity for this iteration's |I| (a smaller LDS footprint fits more signals per CU)
                    const int ib = std::min(need, imax + (d + 1) * rho);
                    bmpl_status r = enqueue_master(q, cc, p, ib, ib, true, true);
                    if (r != BMPL_OK) return r;
                    r = enqueue_select_pass(q, cc, p, false, false, true);
                    if (r != BMPL_OK) return r;
                    cc = 1 - cc;
                }
                return BMPL_OK;
            });
            if (st != BMPL_OK) return st;
            HIPC(hipGraphLaunch(ge, s));
            imax = need;
            st = read_count(cur);    // the depth is even: the running list is back in act[cur]
            if (st != BMPL_OK) return st;
            continue;
        }
        const int add = after_warm ? std::max(warm_k, rho) : rho;
        imax = std::min(max_active, imax + add);
        c->timing.outer_iters += tm ? 1 : 0;
        // a warm start's proposal is mostly zeros: an LDS factor for WARM_KL support positions
        st = enqueue_master(s, cur, n_act, after_warm ? std::min(imax, WARM_KL) : imax, imax, false, !after_warm);
        if (st != BMPL_OK) return st;
        st = enqueue_select_pass(s, cur, n_act, false, after_warm, false);
        if (st != BMPL_OK) return st;
        after_warm = false;
        cur = 1 - cur;
        st = read_count(cur);
        if (st != BMPL_OK) return st;
    }
    const size_t e_pack = tm ? mark(c, s) : 0;
    const int stage_max = std::min(max_active, c->n);   // |S| <= min(|I|, n)
    const size_t pack_lds = (size_t)stage_max * 12;
    PackArgs pk{w, out->x_val_dev, out->x_idx_dev, out->supp_len_dev, out->iters_dev, out->kkt_dev,
                out->lambda_dev, out->objective_dev, out->sig_status_dev, out->ld_x, pack_lds <= 48 * 1024 ? 1 : 0,
                stage_max};
    hipLaunchKernelGGL(pack_kernel, dim3(p), dim3(256), pk.stage ? pack_lds : 0, s, pk);
    HIPC(hipGetLastError());
    if (tm) {
        const size_t e_last = mark(c, s);
        span(c, e_pack, e_last, K_OTHER);
        HIPC(hipStreamSynchronize(s));
        fold_timing(c, ev_first, e_last);
    }
    return BMPL_OK;
}

bmpl_status bmpl_classify(bmpl_ctx* c, const float* B_dev, int64_t ldb, int32_t p, const bmpl_result* sol,
                          const int32_t* class_of_atom_dev, int32_t* labels_dev, double* resid_dev, void* hip_stream)
{
    if (!c || !sol) return fail(BMPL_E_INVALID, "bmpl_classify: NULL context or solution");
    if (p < 0 || ldb < c->n) return fail(BMPL_E_INVALID, "bmpl_classify: bad p=%d or ldb=%lld", p, (long long)ldb);
    if (p == 0) return BMPL_OK;
    if (!B_dev || !class_of_atom_dev || !labels_dev || !sol->x_idx_dev || !sol->x_val_dev || !sol->supp_len_dev ||
        sol->ld_x < 1)
        return fail(BMPL_E_INVALID, "bmpl_classify: signals, classes, labels and the solution's x_idx, x_val, "
                                    "supp_len (ld_x >= 1) are required");
    ClassifyArgs a{};
    a.At = c->At; a.lda = c->kpad; a.n = c->n; a.m = c->m;
    a.B = B_dev; a.ldb = ldb; a.p = p;
    a.x_idx = sol->x_idx_dev; a.x_val = sol->x_val_dev; a.supp_len = sol->supp_len_dev; a.ld_x = sol->ld_x;
    a.class_of_atom = class_of_atom_dev; a.labels = labels_dev; a.resid = resid_dev;
    HIPC(launch_classify(a, reinterpret_cast<hipStream_t>(hip_stream)));
    return BMPL_OK;
}

bmpl_status bmpl_autotune(bmpl_ctx* c, int32_t p, int32_t* shapes, double* ms, void* hip_stream)
{
    if (!c) return fail(BMPL_E_INVALID, "bmpl_autotune: NULL context");
    if (p < 1) return fail(BMPL_E_INVALID, "bmpl_autotune: p must be >= 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int rho = c->opt.rho;
    bmpl_status st = ensure_workspace(c, std::max(p, c->p_cap), std::max(c->selcap, rho));
    if (st != BMPL_OK) return st;
    Workspace& w = c->w;
    HIPC(hipMemsetAsync(w.R, 0, (size_t)p * c->kpad * sizeof(float), s));
    if (w.R16) HIPC(hipMemsetAsync(w.R16, 0, (size_t)p * c->kpad * sizeof(uint16_t), s));
    if (w.R8) HIPC(hipMemsetAsync(w.R8, 0, (size_t)p * c->kpad, s));
    if (w.rscale8) {
        std::vector<float> ones(p, 1.0f);
        HIPC(hipMemcpyAsync(w.rscale8, ones.data(), sizeof(float) * p, hipMemcpyHostToDevice, s));
        HIPC(hipStreamSynchronize(s));
    }
    auto gemm = [&](int v, int nb) -> hipError_t {
        if (c->A8)   // the product of every outer iteration after the first
            return launch_corr_gemm_fp8(v, c->A8, c->kpad, c->m, c->kpad, w.R8, c->kpad, nullptr, nullptr, nb,
                                        c->Gc, c->ldg, c->p_cap, 0, 1 << 30, c->ascale8, w.rscale8, s);
        if (c->A16)
            return launch_corr_gemm_bf16(v, c->A16, c->A16p, c->kpad, c->m, c->kpad, w.R16, c->kpad, nullptr, nullptr, nb,
                                         c->Gc, c->ldg, c->p_cap, 0, 1 << 30, s);
        return launch_corr_gemm_f32(v, c->At, c->kpad, c->m, c->kpad, w.R, c->kpad, nullptr, nullptr, nb, c->Gc,
                                    c->ldg, c->p_cap, 0, 1 << 30, s);
    };
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    const int reps[3] = {std::min(p, 4096), std::min(p, 128), std::min(p, 32)};
    const int lo[3] = {512, 64, 1};
    for (int b = 0; b < 3; ++b) {
        const int nb = reps[b];
        double best = 1e30;
        for (int v = 0; v < CORR_VARIANTS; ++v) {
            double t = -1.0;
            if (nb >= lo[b]) {
                hipError_t e = gemm(v, nb);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                for (int r = 0; r < 3 && e == hipSuccess; ++r)
                    e = gemm(v, nb);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float f = 0.f;
                if (e == hipSuccess && hipEventElapsedTime(&f, e0, e1) == hipSuccess) t = f / 3.0;
                (void)hipGetLastError();
                if (t > 0.0 && t < best) {
                    best = t;
                    c->corr_shape[b] = v;
                }
            }
            if (ms) ms[b * CORR_VARIANTS + v] = t;
        }
        if (shapes) shapes[b] = c->corr_shape[b];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(hipStreamSynchronize(s));
    return BMPL_OK;
}

bmpl_status bmpl_set_tuning(bmpl_ctx* c, const int32_t* shapes)
{
    if (!c || !shapes) return fail(BMPL_E_INVALID, "bmpl_set_tuning: NULL argument");
    const bool bf16_only = c->A16 && !c->A8;   // shapes 8..10 exist for bfloat16 only
    for (int b = 0; b < 3; ++b)
        if (shapes[b] < 0 || shapes[b] >= CORR_VARIANTS || (shapes[b] >= 8 && shapes[b] <= 10 && !bf16_only))
            return fail(BMPL_E_INVALID, "bmpl_set_tuning: shape %d out of range for this precision", shapes[b]);
    for (int b = 0; b < 3; ++b) c->corr_shape[b] = shapes[b];
    return BMPL_OK;
}

bmpl_status bmpl_gram_table(const bmpl_ctx* c, const double** Q_dev, int64_t* ldq)
{
    if (!c || !Q_dev || !ldq) return fail(BMPL_E_INVALID, "bmpl_gram_table: NULL argument");
    *Q_dev = c->Q;
    *ldq = c->Q ? c->m : 0;
    return BMPL_OK;
}

bmpl_status bmpl_get_timing(const bmpl_ctx* c, bmpl_timing* t)
{
    if (!c || !t) return fail(BMPL_E_INVALID, "bmpl_get_timing: NULL argument");
    *t = c->timing;
    if (c->phase_dev && c->wall_khz > 0) {
        uint64_t ticks[PHASE_SLOTS];
        HIPC(hipMemcpy(ticks, c->phase_dev, sizeof ticks, hipMemcpyDeviceToHost));
        for (int i = 0; i < 6; ++i) t->solve_phase_us[i] = (double)ticks[i] * 1e3 / c->wall_khz;
        for (int i = 0; i < 6; ++i) t->solve_step_us[i] = (double)ticks[9 + i] * 1e3 / c->wall_khz;
        t->factor_appends = (int64_t)ticks[6];
        t->factor_drops = (int64_t)ticks[7];
        t->sign_fixed_solves = (int64_t)ticks[8];
    }
    return BMPL_OK;
}

bmpl_status bmpl_reset_timing(bmpl_ctx* c)
{
    if (!c) return fail(BMPL_E_INVALID, "bmpl_reset_timing: NULL context");
    c->timing = bmpl_timing{};
    if (c->phase_dev) HIPC(hipMemset(c->phase_dev, 0, PHASE_SLOTS * sizeof(uint64_t)));
    return BMPL_OK;
}

}  // extern "C"
