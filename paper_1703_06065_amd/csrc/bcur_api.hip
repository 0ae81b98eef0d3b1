// Host runtime of the Block CUR library: context, workspace, the stage
// drivers and the C ABI declared in include/bcur.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bcur.h"
#include "bcur_internal.h"

using namespace bcur;

// Scratch of the entry point that allocates nothing (bcur_decompose_noalloc):
// one array per GPU, held from the library's first use on that GPU until the
// process ends.  In host code its name is only a stand-in: the device address
// comes from hipGetSymbolAddress, taken once per device in bcur_create.
constexpr size_t kScratchBytes = (size_t)128 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 16;
constexpr size_t kHostStageBytes = (size_t)1 << 20;
void* g_scratch[kMaxDevices];                                   // device address of scratch, per device
alignas(64) char g_host_stage[kMaxDevices][kHostStageBytes];    // host staging of those calls, per device
std::mutex g_scratch_mu;
}  // namespace

// Per-stage device timing: event pairs are recorded on the context's stream
// and resolved (elapsed time added to the stage total) on the next read.
struct StageTimer {
    bool on = false;
    uint32_t mask = 0;                            // stages that record events
    std::vector<hipEvent_t> pool;                 // free events
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double ms[BCUR_NUM_STAGES] = {};
    int64_t count[BCUR_NUM_STAGES] = {};
};

// Host copies of an asynchronous decomposition's inputs (bcur_decompose_async).
struct AsyncJob {
    const float* A = nullptr;
    int64_t m = 0, n = 0, lda = 0, G = 0, Gr = 0;
    std::vector<int64_t> col_off, row_off, col_map, row_map;
    std::vector<uint64_t> draws;
    bcur_params p{};
    const float* omega = nullptr;
    bcur_result* res = nullptr;
};

struct bcur_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;         // most device workspace the context may hold (0: no limit)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* pinned = nullptr;
    size_t pinned_bytes = 0;
    bool pinned_busy = false;  // a call left copies into `pinned` without synchronizing
    bool noalloc = false;      // workspace and staging are handed in: nothing may be allocated
    char err[512] = {0};       // message of the last error (a fixed buffer: reporting allocates nothing)
    StageTimer timer;
    // asynchronous decomposition: its host thread, its stream (default
    // priority) and the event that orders it after the caller's stream
    std::thread worker;
    bool inflight = false;
    bcur_status job_status = BCUR_OK;
    hipStream_t astream = nullptr;
    hipEvent_t ev_in = nullptr;
    AsyncJob job;
};

namespace {

constexpr int64_t kMaxSketch = 128;
constexpr int64_t kMaxTrials = 64;   // boosting trials per call

inline int64_t round4(int64_t x) { return (x + 3) & ~(int64_t)3; }

bcur_status fail(bcur_ctx* ctx, bcur_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
bcur_status fail(bcur_ctx* ctx, bcur_status st, const char* fmt, ...) {
    if (!ctx) return st;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
    va_end(ap);
    return st;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, BCUR_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                         \
    } while (0)

#define STCHK(expr)                           \
    do {                                      \
        bcur_status s_ = (expr);              \
        if (s_ != BCUR_OK) return s_;         \
    } while (0)

// Entry points other than bcur_wait refuse to run while an asynchronous
// decomposition uses the context (its host thread owns the context's state,
// the error message included, until bcur_wait).
#define GUARD(ctx)                                  \
    do {                                            \
        if (!(ctx)) return BCUR_E_ARG;              \
        if ((ctx)->inflight) return BCUR_E_STATE;   \
    } while (0)

// Bump allocator over the context workspace.  Layout functions run twice:
// once with a null base to size the workspace, once to hand out pointers.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

bcur_status reserve(bcur_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return BCUR_OK;
    if (ctx->noalloc)
        return fail(ctx, BCUR_E_NOMEM, "the call needs %zu bytes of scratch, above the %zu available", bytes,
                    ctx->ws_bytes);
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, BCUR_E_NOMEM, "the call needs %zu bytes of device workspace, over the context's budget of %zu",
                    bytes, ctx->budget);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->ws) HIPCHK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    size_t want = bytes + bytes / 8;
    if (ctx->budget) want = std::min(want, ctx->budget);
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        ctx->ws = nullptr;
        return fail(ctx, BCUR_E_NOMEM, "device workspace of %zu bytes", want);
    }
    ctx->ws_bytes = want;
    return BCUR_OK;
}

bcur_status reserve_pinned(bcur_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->pinned_bytes) return BCUR_OK;
    if (ctx->noalloc)
        return fail(ctx, BCUR_E_NOMEM, "the call needs %zu bytes of host staging, above the %zu available", bytes,
                    ctx->pinned_bytes);
    if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    if (hipHostMalloc((void**)&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
        ctx->pinned = nullptr;
        return fail(ctx, BCUR_E_NOMEM, "pinned host buffer of %zu bytes", bytes);
    }
    ctx->pinned_bytes = bytes;
    return BCUR_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

hipEvent_t timer_event(bcur_ctx* ctx) {
    StageTimer& t = ctx->timer;
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records the start of a stage; the matching stage_end closes it.
struct StageScope {
    bcur_ctx* ctx;
    int stage;
    hipEvent_t a = nullptr;
    StageScope(bcur_ctx* c, int s) : ctx(c), stage(s) {
        if (!ctx->timer.on || !((ctx->timer.mask >> s) & 1u)) return;
        a = timer_event(ctx);
        if (a && hipEventRecord(a, ctx->stream) != hipSuccess) a = nullptr;
    }
    ~StageScope() {
        if (!a) return;
        hipEvent_t b = timer_event(ctx);
        if (!b || hipEventRecord(b, ctx->stream) != hipSuccess) {
            ctx->timer.pool.push_back(a);
            if (b) ctx->timer.pool.push_back(b);
            return;
        }
        ctx->timer.pending.push_back({stage, {a, b}});
    }
};

void timer_resolve(bcur_ctx* ctx) {
    StageTimer& t = ctx->timer;
    for (auto& p : t.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            t.ms[p.first] += ms;
            t.count[p.first] += 1;
        }
        t.pool.push_back(p.second.first);
        t.pool.push_back(p.second.second);
    }
    t.pending.clear();
}

bcur_status check_matrix(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const char* name) {
    if (!A) return fail(ctx, BCUR_E_ARG, "%s is null", name);
    if (m < 1 || n < 1) return fail(ctx, BCUR_E_ARG, "%s has shape %lld x %lld", name, (long long)m, (long long)n);
    if (lda < n) return fail(ctx, BCUR_E_ARG, "%s: leading dimension %lld < %lld", name, (long long)lda, (long long)n);
    if (!aligned16(A) || (lda & 3))
        return fail(ctx, BCUR_E_ARG, "%s must be 16-byte aligned with a leading dimension that is a multiple of 4", name);
    return BCUR_OK;
}

bcur_status check_offsets(bcur_ctx* ctx, const int64_t* off, int64_t G, int64_t n, const char* name) {
    if (!off || G < 1) return fail(ctx, BCUR_E_ARG, "%s: need G >= 1 offsets", name);
    if (off[0] != 0 || off[G] != n) return fail(ctx, BCUR_E_ARG, "%s must start at 0 and end at %lld", name, (long long)n);
    for (int64_t g = 0; g < G; ++g)
        if (off[g + 1] <= off[g]) return fail(ctx, BCUR_E_ARG, "%s must be strictly increasing (block %lld)", name, (long long)g);
    return BCUR_OK;
}

// Column (or row) indices of the chosen blocks in selection order, each block
// once; with a map, block j holds map[off[j] .. off[j+1]-1].
std::vector<int64_t> expand_blocks(const int64_t* off, const int64_t* idx, int64_t s, const int64_t* map = nullptr) {
    std::vector<int64_t> out;
    std::vector<int64_t> seen;
    for (int64_t t = 0; t < s; ++t) {
        const int64_t j = idx[t];
        if (std::find(seen.begin(), seen.end(), j) != seen.end()) continue;
        seen.push_back(j);
        for (int64_t c = off[j]; c < off[j + 1]; ++c) out.push_back(map ? map[c] : c);
    }
    return out;
}

// The same list written to out (capacity cap), without allocating; returns its length.
int64_t expand_blocks_into(const int64_t* off, const int64_t* idx, int64_t s, const int64_t* map, int64_t* out,
                           int64_t cap) {
    int64_t n = 0;
    for (int64_t t = 0; t < s; ++t) {
        const int64_t j = idx[t];
        bool dup = false;
        for (int64_t u = 0; u < t && !dup; ++u) dup = idx[u] == j;
        if (dup) continue;
        for (int64_t c = off[j]; c < off[j + 1] && n < cap; ++c) out[n++] = map ? map[c] : c;
    }
    return n;
}

// The common width of all blocks, or 0 when they differ.
int64_t uniform_width(const int64_t* off, int64_t G) {
    const int64_t b = off[1] - off[0];
    for (int64_t g = 1; g < G; ++g)
        if (off[g + 1] - off[g] != b) return 0;
    return b;
}

// A block map must be a permutation of 0 .. count-1 (or null).
bcur_status check_map(bcur_ctx* ctx, const int64_t* map, int64_t count, const char* name) {
    if (!map) return BCUR_OK;
    std::vector<char> seen(count, 0);
    for (int64_t i = 0; i < count; ++i) {
        if (map[i] < 0 || map[i] >= count || seen[map[i]])
            return fail(ctx, BCUR_E_ARG, "%s is not a permutation of 0 .. %lld (entry %lld)", name,
                        (long long)(count - 1), (long long)i);
        seen[map[i]] = 1;
    }
    return BCUR_OK;
}

// ---- range finder ---------------------------------------------------------

inline int64_t round8(int64_t x) { return (x + 7) & ~(int64_t)7; }

struct RFBufs {
    float *Q, *Y, *Z, *part;
    double *gpart, *T, *Rinv, *Wk, *Wks, *lam, *sqpart;
    void* jws;
    int* info;
    // BF16 operands (k contiguous): A, A^T, Q^T, Z^T
    uint16_t *Abf, *AbfT, *QT, *ZT;
};

size_t rf_partial_floats(int64_t m, int64_t n, int64_t l, bool bf16) {
    const GemmPlan p1 = plan_sgemm(m, l, n, false, true);
    const GemmPlan p2 = plan_sgemm(n, l, m, true, true);
    size_t s = std::max(sgemm_partial_floats(p1, m, l), sgemm_partial_floats(p2, n, l));
    if (bf16) {
        const GemmPlan b1 = plan_bgemm(m, l, n), b2 = plan_bgemm(n, l, m);
        s = std::max(s, std::max(sgemm_partial_floats(b1, m, l), sgemm_partial_floats(b2, n, l)));
    }
    return s;
}

void rf_layout(Arena& a, RFBufs& b, int64_t m, int64_t n, int64_t l, int64_t k, bool bf16 = false) {
    const int64_t lp = round4(l);
    b.Q = a.take<float>(n * lp);
    b.Y = a.take<float>(n * lp);
    b.Z = a.take<float>(m * lp);
    b.part = a.take<float>(std::max<size_t>(rf_partial_floats(m, n, l, bf16), 4));
    b.Abf = bf16 ? a.take<uint16_t>(m * round8(n)) : nullptr;
    b.AbfT = bf16 ? a.take<uint16_t>(n * round8(m)) : nullptr;
    b.QT = bf16 ? a.take<uint16_t>(l * round8(n)) : nullptr;
    b.ZT = bf16 ? a.take<uint16_t>(l * round8(m)) : nullptr;
    const int w = std::max(gram_wgs(n), gram_wgs(m));
    b.gpart = a.take<double>((size_t)w * l * l);
    b.T = a.take<double>(l * l);
    b.Rinv = a.take<double>(l * l);
    b.Wk = a.take<double>(l * k);
    b.Wks = a.take<double>(l * k);
    b.lam = a.take<double>(l);
    b.info = a.take<int>(4);  // right after lam: the host fetches both with one copy
    b.sqpart = a.take<double>(plan_sgemm(m, l, n, false, true).wgs);
    b.jws = a.take<double>((jacobi_ws_bytes(l) + 7) / 8);
}

// A GEMM whose main kernel is timed as `stage` and its split-K sum as `rstage`.
bcur_status gemm_timed(bcur_ctx* ctx, int stage, int rstage, const GemmPlan& p, int64_t M, int64_t N, int64_t K,
                       bool tA, const float* A, int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd,
                       float* part, int epi = EPI_STORE, const float* X = nullptr, int64_t ldx = 0,
                       const float* Y = nullptr, int64_t ldy = 0, double* wsum = nullptr, const int* ncol = nullptr) {
    {
        StageScope ts(ctx, stage);
        HIPCHK(launch_sgemm_main(p, M, N, K, tA, A, lda, B, ldb, D, ldd, part, epi, X, ldx, Y, ldy, wsum, ctx->stream,
                                 ncol));
    }
    if (p.splits > 1) {
        StageScope ts(ctx, rstage);
        HIPCHK(launch_splitk_reduce(p, M, N, part, D, ldd, ctx->stream));
    }
    return BCUR_OK;
}

// One Cholesky QR pass: out = X R^-1 with R^T R = X^T X (+ a tiny shift),
// Gram in FP64, factor and inverse in FP64, product accumulated in FP64.
// gate (device, or null): the pass runs only when *gate != 0; need2 (device,
// or null) receives whether a second pass would still improve orthogonality.
bcur_status cholqr(bcur_ctx* ctx, const RFBufs& b, const float* X, int64_t rows, int64_t l, float* out,
                   const int* gate = nullptr, int* need2 = nullptr) {
    const int64_t lp = round4(l);
    const int w = gram_wgs(rows);
    HIPCHK(launch_gram64(X, rows, l, lp, b.gpart, w, ctx->stream, gate));
    HIPCHK(launch_gram_reduce(b.gpart, w, l, b.T, ctx->stream, gate));
    HIPCHK(launch_chol_rinv_small(b.T, l, b.Rinv, b.info, ctx->stream, gate, need2));
    HIPCHK(launch_apply_small(X, rows, l, lp, b.Rinv, l, l, out, lp, ctx->stream, gate));
    return BCUR_OK;
}

// Q <- omega; q+1 times Q <- orth(A^T (A Q)); Rayleigh-Ritz.  Vk (n x k, ld k),
// Uk (m x k, ld k) if non-null, lam (device, l).
// Y = A^T (A Q) in BF16: Z = A_bf Q_bf, Y = A_bf^T Z_bf (FP32 accumulation).
// The BF16 copies of A must already be in b.Abf / b.AbfT.
bcur_status sketch_pass_bf16(bcur_ctx* ctx, const RFBufs& b, int64_t m, int64_t n, const float* Q, int64_t ldq,
                             int64_t l, float* Y) {
    hipStream_t st = ctx->stream;
    const int64_t lp = round4(l);
    const GemmPlan pz = plan_bgemm(m, l, n), py = plan_bgemm(n, l, m);
    {
        StageScope ts(ctx, BCUR_STAGE_RF_CAST);
        HIPCHK(launch_cast_bf16_both(Q, n, l, ldq, nullptr, 0, b.QT, round8(n), st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_RF_AQ);
        HIPCHK(launch_bgemm_nt(pz, m, l, n, b.Abf, round8(n), b.QT, round8(n), b.Z, lp, b.part, st));
    }
    if (pz.splits > 1) {
        StageScope ts(ctx, BCUR_STAGE_RF_REDUCE);
        HIPCHK(launch_splitk_reduce(pz, m, l, b.part, b.Z, lp, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_RF_CAST);
        HIPCHK(launch_cast_bf16_both(b.Z, m, l, lp, nullptr, 0, b.ZT, round8(m), st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_RF_ATZ);
        HIPCHK(launch_bgemm_nt(py, n, l, m, b.AbfT, round8(m), b.ZT, round8(m), Y, lp, b.part, st));
    }
    if (py.splits > 1) {
        StageScope ts(ctx, BCUR_STAGE_RF_REDUCE);
        HIPCHK(launch_splitk_reduce(py, n, l, b.part, Y, lp, st));
    }
    return BCUR_OK;
}

bcur_status cast_a_bf16(bcur_ctx* ctx, const RFBufs& b, const float* A, int64_t m, int64_t n, int64_t lda) {
    StageScope ts(ctx, BCUR_STAGE_RF_CAST);
    HIPCHK(launch_cast_bf16_both(A, m, n, lda, b.Abf, round8(n), b.AbfT, round8(m), ctx->stream));
    return BCUR_OK;
}

// precision BCUR_PREC_BF16: iterations 0 .. q-1 in BF16, iteration q and the
// Rayleigh-Ritz pass in FP32 (the final FP32 power pass).
//
// frob2 (device, or null): with an FP32 first pass, ||A||_F^2 is summed from
// that pass's loads of A (each element is loaded once) into frob2[0]; the
// caller computes it separately where the range finder has no FP32 pass
// (range_finder_fuses_frob).  On the BF16 path the first FP32 pass is that of
// the last power iteration.
bool range_finder_fuses_frob(int64_t q, int precision) { (void)q; (void)precision; return true; }

// omega: device n x l (dense), or null: the test matrix of `seed` is drawn into Q.
bcur_status range_finder_run(bcur_ctx* ctx, const RFBufs& b, const float* A, int64_t m, int64_t n, int64_t lda,
                             const float* omega, uint64_t seed, int64_t l, int64_t k, int64_t q, float* Vk, float* Uk,
                             int precision = BCUR_PREC_FP32, double* frob2 = nullptr) {
    hipStream_t st = ctx->stream;
    const int64_t lp = round4(l);
    HIPCHK(hipMemsetAsync(b.info, 0, 4 * sizeof(int), st));
    if (omega)
        HIPCHK(hipMemcpy2DAsync(b.Q, lp * sizeof(float), omega, l * sizeof(float), l * sizeof(float), n,
                                hipMemcpyDeviceToDevice, st));
    else
        HIPCHK(launch_test_matrix(seed, n, l, lp, b.Q, lp, st));
    const GemmPlan pz = plan_sgemm(m, l, n, false, true);
    const GemmPlan py = plan_sgemm(n, l, m, true, true);
    const bool bf16 = precision == BCUR_PREC_BF16 && q > 0;
    if (bf16) STCHK(cast_a_bf16(ctx, b, A, m, n, lda));
    for (int64_t it = 0; it <= q; ++it) {
        if (bf16 && it < q) {
            STCHK(sketch_pass_bf16(ctx, b, m, n, b.Q, lp, l, b.Y));
        } else {
            const bool sqa = frob2 && it == (bf16 ? q : 0);
            STCHK(gemm_timed(ctx, BCUR_STAGE_RF_AQ, BCUR_STAGE_RF_REDUCE, pz, m, l, n, false, A, lda, b.Q, lp, b.Z,
                             lp, b.part, sqa ? EPI_STORE_SQA : EPI_STORE, nullptr, 0, nullptr, 0,
                             sqa ? b.sqpart : nullptr));
            if (sqa) HIPCHK(launch_sum_f64(b.sqpart, pz.wgs, frob2, st));
            STCHK(gemm_timed(ctx, BCUR_STAGE_RF_ATZ, BCUR_STAGE_RF_REDUCE, py, n, l, m, true, A, lda, b.Z, lp, b.Y,
                             lp, b.part));
        }
        // Intermediate bases only need to be well conditioned: one Cholesky QR
        // pass (FP64 Gram and factor) leaves an orthogonality error of about
        // 2^-52 cond(Y)^2 + 2^-24.  The basis handed to Rayleigh-Ritz gets a
        // second pass (Cholesky QR2) unless the first factor certifies that
        // its error is already below 2^-26 (decided on the device: the second
        // pass's kernels return at once).
        StageScope ts(ctx, BCUR_STAGE_RF_ORTH);
        STCHK(cholqr(ctx, b, b.Y, n, l, b.Q, nullptr, it == q ? b.info + 1 : nullptr));
        if (it == q) STCHK(cholqr(ctx, b, b.Q, n, l, b.Q, b.info + 1));
    }
    STCHK(gemm_timed(ctx, BCUR_STAGE_RF_AQ, BCUR_STAGE_RF_REDUCE, pz, m, l, n, false, A, lda, b.Q, lp, b.Z, lp,
                     b.part));
    StageScope ts(ctx, BCUR_STAGE_RF_RR);
    const int wz = gram_wgs(m);
    HIPCHK(launch_gram64(b.Z, m, l, lp, b.gpart, wz, st));
    HIPCHK(launch_gram_reduce(b.gpart, wz, l, b.T, st));
    HIPCHK(launch_jacobi_eigh(b.T, l, k, b.lam, b.Wk, b.Wks, b.jws, b.info + 2, st));
    HIPCHK(launch_apply_small(b.Q, n, l, lp, b.Wk, k, k, Vk, k, st));
    if (Uk) HIPCHK(launch_apply_small(b.Z, m, l, lp, b.Wks, k, k, Uk, k, st));
    return BCUR_OK;
}

// ---- fit ------------------------------------------------------------------

constexpr int64_t kFbPanel = 1024;  // columns of A per FP64 fallback panel

struct FitBufs {
    float *H, *F, *X32, *G32, *Gi32, *part, *Gtmp;
    double *G, *spdws, *wsE, *wsD, *wsF, *errv, *piv;
    // FP64 Cholesky QR2 fallback for a numerically rank-deficient or
    // ill-conditioned C: its Gram matrix, L1^-1, Q1 = C L1^-T, two c x kFbPanel panels
    double *Gc64, *L1, *Q1, *T1, *T2;
    int64_t nwsE, nwsD;
    size_t npart;   // floats of split-K partials in part
    int* info;
    int* ncol;   // the columns of A outside C, for the residual pass
};

void fit_layout(Arena& a, FitBufs& b, int64_t m, int64_t n, int64_t c, bool need_gtmp) {
    const int64_t np = round4(n), cp = round4(c);
    b.H = a.take<float>(c * np);
    b.F = a.take<float>(c * np);
    b.X32 = a.take<float>(c * cp);
    b.G32 = a.take<float>(c * cp);
    b.Gi32 = a.take<float>(c * cp);
    const GemmPlan ph = plan_sgemm(c, n, m, true, true);
    const GemmPlan pg = plan_sgemm(c, c, m, true, true);
    const GemmPlan pi = plan_sgemm(c, c, c, true, true);
    const GemmPlan pu = plan_sgemm(c, n, c, false, true);
    size_t part = std::max(std::max(sgemm_partial_floats(ph, c, n), sgemm_partial_floats(pg, c, c)),
                           std::max(sgemm_partial_floats(pu, c, n), sgemm_partial_floats(pi, c, c)));
    b.npart = std::max<size_t>(part, 4);
    b.part = a.take<float>(b.npart);
    b.Gtmp = need_gtmp ? a.take<float>(c * cp) : nullptr;
    b.G = a.take<double>(c * c);
    b.spdws = a.take<double>(spd_inverse_ws_doubles(c));
    // c is the most columns a call may fit; the partial counts of a call with
    // fewer (repeated or narrower blocks) can be larger: a smaller product can
    // take the smaller tile
    b.nwsE = resid_parts_max(m, n);
    b.nwsD = add_dot_parts_max(c, n);
    b.wsE = a.take<double>(b.nwsE);
    b.wsD = a.take<double>(b.nwsD);
    b.wsF = a.take<double>(resid_store_parts(c, n));
    b.errv = a.take<double>(8);
    b.piv = a.take<double>(2 * ((c + 63) / 64));
    b.info = a.take<int>(4);
    b.ncol = a.take<int>(n <= kComplementMaxN ? n : 1);
    b.Gc64 = a.take<double>(c * c);
    b.L1 = a.take<double>(c * c);
    b.Q1 = a.take<double>(m * c);
    b.T1 = a.take<double>(c * std::min<int64_t>(n, kFbPanel));
    b.T2 = a.take<double>(c * std::min<int64_t>(n, kFbPanel));
}

// U = C^+ A through the normal equations with one optional refinement step:
// G = C^T C = L L^T (FP64), X = L^-1 rounded to FP32, G^-1 = X^T X formed in
// FP32 (one c x c x c product), U = G^-1 H and dU = G^-1 F, with the
// refinement's right-hand side F = C^T (A - C U) formed as H - G U (G as
// factored, in FP32).
// When d_cols (device, c) gives C's columns within A (C = A[:, cols]), C^T C
// is read off H = C^T A; otherwise (d_cols null, d_ident = 0..c-1) it is
// formed by its own GEMM into Gtmp.  After the caller synchronizes,
// b.errv[0] = ||E||^2 - <F, dU> (err^2 after the refinement), b.errv[1] =
// ||E||^2 (before it), b.info[0] bit 0 = pivots dropped, b.piv = pivot ranges.
// Hpre: H = C^T A already computed by the caller (c x n, ld round4(n)); b.H is
// then unused.
// With d_cols (distinct columns, as every caller that passes them guarantees),
// C e_k is column cols[k] of A exactly, so U[:, cols] = I leaves those columns
// a residual of exactly zero; it is their least-squares solution when C has
// full column rank, the case this path keeps (otherwise fit_collect redoes U
// whole in FP64).  The residual pass then covers the other n - c columns
// only, through their list, and with a refinement step F[:, cols] = 0, so
// dU leaves those columns at I and adds nothing for them to <F, dU>.  Taken
// where the shorter pass runs fewer rounds of workgroups than the whole one
// (otherwise the two small launches it needs would cost more than it saves).
// b.info[3] = 1 if the list of columns repeats one.
bcur_status fit_run(bcur_ctx* ctx, const FitBufs& b, const float* A, int64_t m, int64_t n, int64_t lda, const float* C,
                    int64_t c, int64_t ldc, const int64_t* d_cols, const int64_t* d_ident, int refine, float* U,
                    int64_t ldu, const float* Hpre = nullptr) {
    hipStream_t st = ctx->stream;
    const int64_t np = round4(n), cp = round4(c);
    HIPCHK(hipMemsetAsync(b.info, 0, 4 * sizeof(int), st));
    const int64_t nr = n - c;
    const bool skip = d_cols && nr > 0 && n <= kComplementMaxN && resid_cols_ok(m, nr, c) &&
                      resid_rounds(m, nr, c) < resid_rounds(m, n, c);
    if (skip) HIPCHK(launch_complement_cols(d_cols, c, n, b.ncol, b.info + 3, st));
    // (the buffers are laid out for the most columns a call may fit; a call
    // with fewer can split its products into more parts than part holds)
    const GemmPlan ph = plan_sgemm_within(c, n, m, true, b.npart);
    // H = C^T A, or the caller's precomputed rows of it (ld np)
    const float* H = Hpre ? Hpre : b.H;
    if (!Hpre)
        STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_H, BCUR_STAGE_FIT_REDUCE, ph, c, n, m, true, C, ldc, A, lda, b.H, np,
                         b.part));
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_INV);
        if (d_cols) {
            HIPCHK(launch_gram_from_cols(H, np, d_cols, c, b.G, st, refine ? b.G32 : nullptr, cp));
        } else {
            if (!b.Gtmp || !d_ident) return fail(ctx, BCUR_E_ARG, "internal: no Gram buffer");
            const GemmPlan pg = plan_sgemm_within(c, c, m, true, b.npart);
            HIPCHK(launch_sgemm(pg, c, c, m, true, C, ldc, C, ldc, b.Gtmp, cp, b.part, EPI_STORE, nullptr, 0, nullptr,
                                0, nullptr, st));
            HIPCHK(launch_gram_from_cols(b.Gtmp, cp, d_ident, c, b.G, st, refine ? b.G32 : nullptr, cp));
        }
        // (with a refinement step, G32 holds G as factored, rounded to FP32, for
        // its F = H - G U)
        double* Linv = nullptr;
        HIPCHK(launch_chol_linv(b.G, c, b.spdws, b.info, b.piv, ldexp(1.0, -24), &Linv, st));
        HIPCHK(launch_f64_to_f32_2d(Linv, c, c, c, b.X32, cp, true, st));
        // G^-1 = X^T X (X is zero above its diagonal)
        const GemmPlan pi = plan_sgemm_within(c, c, c, true, b.npart);
        HIPCHK(launch_sgemm(pi, c, c, c, true, b.X32, cp, b.X32, cp, b.Gi32, cp, b.part, EPI_STORE, nullptr, 0,
                            nullptr, 0, nullptr, st));
    }
    // U = G^-1 H
    const GemmPlan pu = plan_sgemm_within(c, n, c, false, b.npart);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_U, BCUR_STAGE_FIT_REDUCE, pu, c, n, c, false, b.Gi32, cp, H, np, U, ldu,
                     b.part));
    if (skip && !refine) HIPCHK(launch_pin_selected(d_cols, c, U, ldu, nullptr, 0, st));
    // ||A - C U||_F^2 (the residual itself is never stored)
    const int64_t ne = skip ? nr : n;
    const GemmPlan pe = plan_sgemm(m, ne, c, false, false);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_E, BCUR_STAGE_FIT_REDUCE, pe, m, ne, c, false, C, ldc, U, ldu, nullptr, 0,
                     nullptr, EPI_RESID_NORM, A, lda, nullptr, 0, b.wsE, skip ? b.ncol : nullptr));
    if (refine) {
        // F = C^T (A - C U) = H - G U from the products already formed: a c x n x c
        // GEMM in place of a second 2 m c n pass over the m x n residual
        {
            StageScope ts(ctx, BCUR_STAGE_FIT_F);
            const GemmPlan pf = plan_sgemm_within(c, n, c, false, b.npart);
            HIPCHK(launch_sgemm(pf, c, n, c, false, b.G32, cp, U, ldu, b.F, np, b.part, EPI_RESID, H, np, nullptr, 0,
                                b.wsF, st));
            if (skip) HIPCHK(launch_pin_selected(d_cols, c, U, ldu, b.F, np, st));
        }
        // U += G^-1 F with <G^-1 F, F>
        StageScope ts(ctx, BCUR_STAGE_FIT_DU);
        HIPCHK(launch_sgemm_add_dot(pu, c, n, c, false, b.Gi32, cp, b.F, np, U, ldu, b.part, U, ldu, b.F, np, b.wsD,
                                    st));
    }
    // one partial per workgroup of the residual GEMM, and of the dU sum
    HIPCHK(launch_fit_err(b.wsE, resid_parts(m, ne, c), b.wsD, refine ? add_dot_parts(pu, c, n, c) : 0, b.errv, st));
    return BCUR_OK;
}

// Reads the fit's scalars after the stream has been synchronized.
struct FitOut {
    double err2;
    uint32_t flags;
    double cond_est;   // sqrt(largest / smallest Cholesky pivot of C^T C): a lower bound on cond(C)
};

// U = C^+ A by Cholesky QR2 in FP64 (the scheme of the row-block variant):
// L1 L1^T = C^T C from FP32 C with FP64 sums, Q1 = C L1^-T, L2 L2^T = Q1^T Q1,
// U = L1^-T L2^-T L2^-1 Q1^T A, with pivots below 2^-50 of the largest dropped
// (a basic least-squares solution on the kept columns).  Then ||A - C U||_F^2
// for the returned FP32 U (norm-only residual epilogue): err2 is that U's exact
// residual.
bcur_status fit_fallback64(bcur_ctx* ctx, const FitBufs& b, const float* A, int64_t m, int64_t n, int64_t lda,
                           const float* C, int64_t c, int64_t ldc, float* U, int64_t ldu, double* err2) {
    hipStream_t st = ctx->stream;
    const double rel64 = ldexp(1.0, -50);
    double *L1inv = nullptr, *L2inv = nullptr;
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_INV);
        HIPCHK(launch_dgemm_ff(c, c, m, 1.0, C, ldc, true, C, ldc, false, 0.0, b.Gc64, c, st));
        HIPCHK(launch_chol_linv(b.Gc64, c, b.spdws, b.info + 1, nullptr, rel64, &L1inv, st));
        HIPCHK(hipMemcpyAsync(b.L1, L1inv, c * c * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(launch_dgemm_fd(m, c, c, 1.0, C, ldc, false, b.L1, c, true, 0.0, b.Q1, c, st));
        HIPCHK(launch_dgemm(c, c, m, 1.0, b.Q1, c, true, b.Q1, c, false, 0.0, b.Gc64, c, st));
        HIPCHK(launch_chol_linv(b.Gc64, c, b.spdws, b.info + 2, nullptr, rel64, &L2inv, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_U);
        for (int64_t j0 = 0; j0 < n; j0 += kFbPanel) {
            const int64_t w = std::min(kFbPanel, n - j0);
            HIPCHK(launch_dgemm_df(c, w, m, 1.0, b.Q1, c, true, A + j0, lda, false, 0.0, b.T1, w, st));  // Q1^T A
            HIPCHK(launch_dgemm(c, w, c, 1.0, L2inv, c, false, b.T1, w, false, 0.0, b.T2, w, st));       // L2^-1 .
            HIPCHK(launch_dgemm(c, w, c, 1.0, L2inv, c, true, b.T2, w, false, 0.0, b.T1, w, st));        // L2^-T .
            HIPCHK(launch_dgemm(c, w, c, 1.0, b.L1, c, true, b.T1, w, false, 0.0, b.T2, w, st));         // L1^-T .
            HIPCHK(launch_f64_to_f32_2d(b.T2, c, w, w, U + j0, ldu, false, st));
        }
    }
    const GemmPlan pe = plan_sgemm(m, n, c, false, false);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_E, BCUR_STAGE_FIT_REDUCE, pe, m, n, c, false, C, ldc, U, ldu, nullptr, 0,
                     nullptr, EPI_RESID_NORM, A, lda, nullptr, 0, b.wsE));
    HIPCHK(launch_fit_err(b.wsE, resid_parts(m, n, c), b.wsD, 0, b.errv, st));
    double hv[3];
    HIPCHK(hipMemcpyAsync(hv, b.errv, sizeof hv, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *err2 = hv[0];
    return BCUR_OK;
}

// Bytes of host staging fit_collect reads its small results into.
size_t fit_collect_bytes(const FitBufs& b) {
    return (size_t)(reinterpret_cast<const char*>(b.info + 4) - reinterpret_cast<const char*>(b.errv));
}

// hstage: host buffer of fit_collect_bytes(b) bytes, or null (one is allocated).
bcur_status fit_collect(bcur_ctx* ctx, const FitBufs& b, const float* A, int64_t m, int64_t n, int64_t lda,
                        const float* C, int64_t c, int64_t ldc, float* U, int64_t ldu, FitOut* out,
                        char* hstage = nullptr) {
    const int64_t nblk = (c + 63) / 64;
    // errv, piv and info are consecutive in the workspace: one copy
    const char* d0 = reinterpret_cast<const char*>(b.errv);
    const size_t span = fit_collect_bytes(b);
    std::vector<char> own;
    if (!hstage) {
        own.resize(span);
        hstage = own.data();
    }
    HIPCHK(hipMemcpyAsync(hstage, d0, span, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double* hv = reinterpret_cast<const double*>(hstage);
    const double* piv = reinterpret_cast<const double*>(hstage + (reinterpret_cast<const char*>(b.piv) - d0));
    const int* hinfo = reinterpret_cast<const int*>(hstage + (reinterpret_cast<const char*>(b.info) - d0));
    if (hinfo[3]) return fail(ctx, BCUR_E_HIP, "internal: the chosen columns repeat or fall outside A");
    uint32_t fl = 0;
    if (hinfo[0] & 1) fl |= BCUR_FLAG_RANKDEF_C;
    double pmin = INFINITY, pmax = 0.0;
    for (int64_t i = 0; i < nblk; ++i) {
        pmin = std::min(pmin, piv[2 * i]);
        pmax = std::max(pmax, piv[2 * i + 1]);
    }
    // cond(C)^2 is at least the spread of the Cholesky pivots
    if (pmin > 0.0 && pmax / pmin * ldexp(1.0, -24) > 0.1) fl |= BCUR_FLAG_ILLCOND_C;
    double err2 = hv[0];
    if (fl & (BCUR_FLAG_RANKDEF_C | BCUR_FLAG_ILLCOND_C)) {
        // the FP32 normal equations lose about u32 cond(C)^2: redo the fit in FP64
        STCHK(fit_fallback64(ctx, b, A, m, n, lda, C, c, ldc, U, ldu, &err2));
    }
    out->err2 = std::max(err2, 0.0);
    out->flags = fl;
    out->cond_est = (pmin > 0.0 && pmax > 0.0) ? sqrt(pmax / pmin) : INFINITY;
    return BCUR_OK;
}


// ---- row-block variant: U = C^+ A R^+ -------------------------------------

struct CurBufs {
    float *R, *W32;
    double *Gc, *Gr, *Grinv, *B, *X, *Q1, *L1, *H2, *T1, *U0, *Wd, *spc, *spr, *wsE, *errv, *pivc, *pivr;
    int* info;
};

void cur_layout(Arena& a, CurBufs& b, int64_t m, int64_t n, int64_t c, int64_t r) {
    b.R = a.take<float>(r * round4(n));
    b.W32 = a.take<float>(m * round4(r));
    b.Gc = a.take<double>(c * c);
    b.Gr = a.take<double>(r * r);
    b.Grinv = a.take<double>(r * r);
    b.B = a.take<double>(m * r);
    b.X = a.take<double>(m * r);
    b.Q1 = a.take<double>(m * c);
    b.L1 = a.take<double>(c * c);
    b.H2 = a.take<double>(c * r);
    b.T1 = a.take<double>(c * r);
    b.U0 = a.take<double>(c * r);
    b.Wd = a.take<double>(m * r);
    b.spc = a.take<double>(spd_inverse_ws_doubles(c));
    b.spr = a.take<double>(spd_inverse_ws_doubles(r));
    b.wsE = a.take<double>(resid_parts_max(m, n));
    b.errv = a.take<double>(4);
    b.pivc = a.take<double>(2 * ((c + 63) / 64));
    b.pivr = a.take<double>(2 * ((r + 63) / 64));
    b.info = a.take<int>(4);
}

// U = C^+ A R^+ and err^2 = ||A - C U R||_F^2 (in b.errv[0] after a sync).
// FP64 arithmetic on the FP32 data (products of FP32 values are exact in
// FP64) for the c- and r-sized pieces:
//   R side (normal equations): G_r = R R^T, B = A R^T, X = B G_r^-1 = A R^+;
//   C side (Cholesky QR2): C = Q R_C with R_C = (L_2^T)(L_1^T), from
//   G_c = C^T C = L_1 L_1^T, Q_1 = C L_1^-T, Q_1^T Q_1 = L_2 L_2^T, Q = Q_1 L_2^-T,
//   so C C^+ X = Q (Q^T X) and U = L_1^-T L_2^-T (Q^T X).
// Cholesky QR2 keeps the projection accurate for cond(C) up to about 1e7,
// where the normal equations of C would lose cond(C)^2 u.  The residual
// A - (C U) R is one FP32 MFMA GEMM with the fused squared-norm epilogue.
bcur_status fit_cur_run(bcur_ctx* ctx, const CurBufs& b, const float* A, int64_t m, int64_t n, int64_t lda,
                        const float* C, int64_t c, int64_t ldc, int64_t r, float* U, int64_t ldu) {
    hipStream_t st = ctx->stream;
    const int64_t ldr = round4(n), rp = round4(r);
    const double rel64 = ldexp(1.0, -50);
    HIPCHK(hipMemsetAsync(b.info, 0, 4 * sizeof(int), st));
    double *L1inv = nullptr, *L2inv = nullptr;
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_H);
        HIPCHK(launch_dgemm_ff(r, r, n, 1.0, b.R, ldr, false, b.R, ldr, true, 0.0, b.Gr, r, st));
        HIPCHK(launch_dgemm_ff(m, r, n, 1.0, A, lda, false, b.R, ldr, true, 0.0, b.B, r, st));
        HIPCHK(launch_dgemm_ff(c, c, m, 1.0, C, ldc, true, C, ldc, false, 0.0, b.Gc, c, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_INV);
        HIPCHK(launch_spd_inverse(b.Gr, r, b.Grinv, b.spr, b.info + 1, b.pivr, rel64, st));
        HIPCHK(launch_chol_linv(b.Gc, c, b.spc, b.info, b.pivc, rel64, &L1inv, st));
        // L1^-1 leaves the factorization workspace, which the second pass reuses
        HIPCHK(hipMemcpyAsync(b.L1, L1inv, c * c * sizeof(double), hipMemcpyDeviceToDevice, st));
        L1inv = b.L1;
        // Q1 = C L1^-T and its Gram (into G_c's storage); L2^-1 (Q = Q1 L2^-T is never formed)
        HIPCHK(launch_dgemm_fd(m, c, c, 1.0, C, ldc, false, L1inv, c, true, 0.0, b.Q1, c, st));
        HIPCHK(launch_dgemm(c, c, m, 1.0, b.Q1, c, true, b.Q1, c, false, 0.0, b.Gc, c, st));
        HIPCHK(launch_chol_linv(b.Gc, c, b.spc, b.info + 2, nullptr, rel64, &L2inv, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_FIT_U);
        // X = A R^+
        HIPCHK(launch_dgemm(m, r, r, 1.0, b.B, r, false, b.Grinv, r, false, 0.0, b.X, r, st));
        // T1 = Q1^T X, H2 = L2^-1 T1 = Q^T X
        HIPCHK(launch_dgemm(c, r, m, 1.0, b.Q1, c, true, b.X, r, false, 0.0, b.T1, r, st));
        HIPCHK(launch_dgemm(c, r, c, 1.0, L2inv, c, false, b.T1, r, false, 0.0, b.H2, r, st));
        // U = L1^-T L2^-T H2
        HIPCHK(launch_dgemm(c, r, c, 1.0, L2inv, c, true, b.H2, r, false, 0.0, b.T1, r, st));
        HIPCHK(launch_dgemm(c, r, c, 1.0, L1inv, c, true, b.T1, r, false, 0.0, b.U0, r, st));
        // W = C U = Q1 (L2^-T H2) = Q1 T1
        HIPCHK(launch_dgemm(m, r, c, 1.0, b.Q1, c, false, b.T1, r, false, 0.0, b.Wd, r, st));
        HIPCHK(launch_f64_to_f32_2d(b.Wd, m, r, r, b.W32, rp, true, st));
        if (U) HIPCHK(launch_f64_to_f32_2d(b.U0, c, r, r, U, ldu, false, st));
    }
    const GemmPlan pe = plan_sgemm(m, n, r, false, false);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_E, BCUR_STAGE_FIT_REDUCE, pe, m, n, r, false, b.W32, rp, b.R, ldr, nullptr,
                     0, nullptr, EPI_RESID_NORM, A, lda, nullptr, 0, b.wsE));
    HIPCHK(launch_fit_err(b.wsE, resid_parts(m, n, r), b.wsE, 0, b.errv, st));
    return BCUR_OK;
}

// Sampling buffers for one side (columns or rows).
struct SampleBufs {
    int64_t *off, *idx, *list;
    double *sc, *w, *mg;
    uint64_t *dr, *qb, *pr;
    int* st;
};

// The sampler's results (idx, w, mg, st, sc) are laid out last and in one
// stretch so the host fetches them with a single copy; `tail` (bytes, may
// be 0) extends the stretch for the caller's own results.
void sample_layout(Arena& a, SampleBufs& b, int64_t G, int64_t s, int64_t listmax) {
    b.off = a.take<int64_t>(G + 1);
    b.dr = a.take<uint64_t>(s);
    b.qb = a.take<uint64_t>(G);
    b.pr = a.take<uint64_t>(G);
    b.list = a.take<int64_t>(std::max<int64_t>(listmax, 1));
    b.idx = a.take<int64_t>(s);
    b.w = a.take<double>(s);
    b.mg = a.take<double>(s);
    b.st = a.take<int>(4);
    b.sc = a.take<double>(G);
}

// Device workspace of one decomposition, from the shapes alone (the same
// layout bcur_decompose uses).  need_ubuf: the library holds U itself.
size_t decompose_ws_bytes(int64_t m, int64_t n, int64_t G, int64_t maxw, int64_t Gr, int64_t maxh,
                          const bcur_params* p, bool need_ubuf) {
    const int64_t k = p->k, l = p->l, s = p->s;
    const bool bf16 = p->precision == BCUR_PREC_BF16;
    const bool rowv = Gr > 0 && p->s_r > 0;
    const int64_t s_r = rowv ? p->s_r : 0;
    const int64_t cmax = std::min(s * maxw, n);
    const int64_t rmax = rowv ? std::min(s_r * maxh, m) : 0;
    const int64_t ucols = rowv ? rmax : n;
    Arena a;
    RFBufs rb;
    FitBufs fb;
    CurBufs cb;
    SampleBufs sc, sr;
    rf_layout(a, rb, m, n, l, k, bf16);
    sample_layout(a, sc, G, s, cmax);
    if (rowv) sample_layout(a, sr, Gr, s_r, rmax);
    a.take<double>(2);
    a.take<double>(frob2_grid(m, n));
    a.take<float>(n * k);
    if (rowv) a.take<float>(m * k);
    if (p->col_map) {
        a.take<int64_t>(n);
        a.take<float>(n * k);
    }
    if (rowv && p->row_map) {
        a.take<int64_t>(m);
        a.take<float>(m * k);
    }
    a.take<float>(m * round4(cmax));
    if (need_ubuf) a.take<float>(cmax * round4(ucols));
    if (rowv) cur_layout(a, cb, m, n, cmax, rmax);
    else fit_layout(a, fb, m, n, cmax, false);
    return a.off + a.off / 8;   // what reserve() allocates for this request
}

}  // namespace

// ---- C ABI ------------------------------------------------------------------

extern "C" {

const char* bcur_status_str(int status) {
    switch (status) {
        case BCUR_OK: return "ok";
        case BCUR_E_ARG: return "invalid argument";
        case BCUR_E_NONFINITE: return "matrix holds NaN or Inf";
        case BCUR_E_NOMEM: return "out of memory";
        case BCUR_E_HIP: return "HIP runtime error";
        case BCUR_E_RANKDEF: return "numerically singular factorization";
        case BCUR_E_ADMIT: return "request exceeds the memory budget";
        case BCUR_PENDING: return "pending";
        case BCUR_E_STATE: return "unknown ticket";
        default: return "unknown status";
    }
}

const char* bcur_last_error(const bcur_ctx* ctx) { return ctx ? ctx->err : ""; }

size_t bcur_workspace_bytes(const bcur_ctx* ctx) { return ctx ? ctx->ws_bytes : 0; }

bcur_status bcur_release_workspace(bcur_ctx* ctx) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->ws) HIPCHK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    return BCUR_OK;
}

bcur_status bcur_footprint(int64_t m, int64_t n, const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                           const bcur_params* p, int32_t library_holds_u, size_t* bytes) {
    if (!p || !col_off || !bytes || G < 1 || m < 1 || n < 1) return BCUR_E_ARG;
    int64_t maxw = 0, maxh = 0;
    for (int64_t g = 0; g < G; ++g) maxw = std::max(maxw, col_off[g + 1] - col_off[g]);
    if (row_off)
        for (int64_t g = 0; g < Gr; ++g) maxh = std::max(maxh, row_off[g + 1] - row_off[g]);
    *bytes = decompose_ws_bytes(m, n, G, maxw, row_off ? Gr : 0, maxh, p, library_holds_u != 0);
    return BCUR_OK;
}

bcur_status bcur_create(bcur_ctx** out, int device, void* stream, size_t scratch_budget) {
    if (!out) return BCUR_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BCUR_E_ARG;
    bcur_ctx* ctx = new (std::nothrow) bcur_ctx;
    if (!ctx) return BCUR_E_NOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return BCUR_E_HIP;
    }
    ctx->stream = (hipStream_t)stream;   // NULL: the device's null stream
    ctx->budget = scratch_budget;
    if (device < kMaxDevices) {
        // the scratch array's address on this device (the device is current here)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
                delete ctx;
                return BCUR_E_HIP;
            }
            g_scratch[device] = ptr;
        }
    }
    *out = ctx;
    return BCUR_OK;
}

bcur_status bcur_destroy(bcur_ctx* ctx) {
    if (!ctx) return BCUR_E_ARG;
    (void)bcur_wait(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    timer_resolve(ctx);
    for (hipEvent_t e : ctx->timer.pool) (void)hipEventDestroy(e);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->astream) (void)hipStreamDestroy(ctx->astream);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    delete ctx;
    return BCUR_OK;
}

bcur_status bcur_synchronize(bcur_ctx* ctx) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BCUR_OK;
}

bcur_status bcur_timing_enable(bcur_ctx* ctx, int32_t on) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    timer_resolve(ctx);
    ctx->timer.on = on != 0;
    ctx->timer.mask = (uint32_t)on;
    for (int i = 0; i < BCUR_NUM_STAGES; ++i) {
        ctx->timer.ms[i] = 0.0;
        ctx->timer.count[i] = 0;
    }
    return BCUR_OK;
}

bcur_status bcur_timing_read(bcur_ctx* ctx, double* ms, int64_t* count) {
    GUARD(ctx);
    if (!ctx || !ms || !count) return BCUR_E_ARG;
    timer_resolve(ctx);
    for (int i = 0; i < BCUR_NUM_STAGES; ++i) {
        ms[i] = ctx->timer.ms[i];
        count[i] = ctx->timer.count[i];
    }
    return BCUR_OK;
}

bcur_status bcur_test_matrix(bcur_ctx* ctx, int64_t n, int64_t l, uint64_t seed, float* omega, int64_t ldo) {
    GUARD(ctx);
    if (!omega) return fail(ctx, BCUR_E_ARG, "omega is required");
    if (n < 1 || l < 1 || l > 256 || ldo < l) return fail(ctx, BCUR_E_ARG, "need n >= 1, 1 <= l <= 256, ldo >= l");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_test_matrix(seed, n, l, l, omega, ldo, ctx->stream));
    return BCUR_OK;
}

bcur_status bcur_frob2(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, double* out_frob2,
                       int32_t* out_finite) {
    GUARD(ctx);
    if (!ctx || !out_frob2) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    HIPCHK(hipSetDevice(ctx->device));
    const int grid = frob2_grid(m, n);
    Arena a;
    a.take<double>(grid);
    a.take<double>(1);
    STCHK(reserve(ctx, a.off));
    Arena b{ctx->ws, 0};
    double* part = b.take<double>(grid);
    double* out = b.take<double>(1);
    HIPCHK(launch_frob2(A, m, n, lda, part, grid, out, ctx->stream));
    STCHK(reserve_pinned(ctx, 64));
    HIPCHK(hipMemcpyAsync(ctx->pinned, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double v = *reinterpret_cast<double*>(ctx->pinned);
    *out_frob2 = v;
    if (out_finite) *out_finite = isfinite(v) ? 1 : 0;
    return BCUR_OK;
}

bcur_status bcur_range_finder(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* omega,
                              int64_t l, int64_t k, int64_t q, int32_t precision, float* Vk, float* Uk, double* ritz) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    if (!omega || !Vk) return fail(ctx, BCUR_E_ARG, "omega and Vk are required");
    if (k < 1 || l < k || l > std::min(std::min(m, n), kMaxSketch))
        return fail(ctx, BCUR_E_ARG, "need 1 <= k <= l <= min(m, n, %lld)", (long long)kMaxSketch);
    if (q < 0 || q > 64) return fail(ctx, BCUR_E_ARG, "q out of range");
    if (precision != BCUR_PREC_FP32 && precision != BCUR_PREC_BF16)
        return fail(ctx, BCUR_E_ARG, "unknown precision %d", precision);
    HIPCHK(hipSetDevice(ctx->device));
    const bool bf16 = precision == BCUR_PREC_BF16;
    Arena a;
    RFBufs b;
    rf_layout(a, b, m, n, l, k, bf16);
    STCHK(reserve(ctx, a.off));
    Arena r{ctx->ws, 0};
    rf_layout(r, b, m, n, l, k, bf16);
    STCHK(range_finder_run(ctx, b, A, m, n, lda, omega, 0, l, k, q, Vk, Uk, precision));
    if (ritz) {
        STCHK(reserve_pinned(ctx, l * sizeof(double)));
        HIPCHK(hipMemcpyAsync(ctx->pinned, b.lam, l * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const double* lam = reinterpret_cast<const double*>(ctx->pinned);
        for (int64_t i = 0; i < l; ++i) ritz[i] = lam[i] > 0.0 ? sqrt(lam[i]) : 0.0;
    }
    return BCUR_OK;
}

bcur_status bcur_sketch_pass(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* Q,
                             int64_t l, int64_t ldq, int32_t precision, float* Y, int64_t ldy) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_matrix(ctx, Q, n, l, ldq, "Q"));
    if (!Y || ldy < l || (ldy & 3) || !aligned16(Y)) return fail(ctx, BCUR_E_ARG, "Y: bad pointer or leading dimension");
    if (l > 128) return fail(ctx, BCUR_E_ARG, "l must be <= 128");
    if (precision != BCUR_PREC_FP32 && precision != BCUR_PREC_BF16)
        return fail(ctx, BCUR_E_ARG, "unknown precision %d", precision);
    HIPCHK(hipSetDevice(ctx->device));
    const bool bf16 = precision == BCUR_PREC_BF16;
    Arena a;
    RFBufs b;
    rf_layout(a, b, m, n, l, l, bf16);
    STCHK(reserve(ctx, a.off));
    Arena r{ctx->ws, 0};
    rf_layout(r, b, m, n, l, l, bf16);
    const int64_t lp = round4(l);
    HIPCHK(hipMemcpy2DAsync(b.Q, lp * sizeof(float), Q, ldq * sizeof(float), l * sizeof(float), n,
                            hipMemcpyDeviceToDevice, ctx->stream));
    if (bf16) {
        STCHK(cast_a_bf16(ctx, b, A, m, n, lda));
        STCHK(sketch_pass_bf16(ctx, b, m, n, b.Q, lp, l, b.Y));
    } else {
        const GemmPlan pz = plan_sgemm(m, l, n, false, true);
        const GemmPlan py = plan_sgemm(n, l, m, true, true);
        STCHK(gemm_timed(ctx, BCUR_STAGE_RF_AQ, BCUR_STAGE_RF_REDUCE, pz, m, l, n, false, A, lda, b.Q, lp, b.Z, lp,
                         b.part));
        STCHK(gemm_timed(ctx, BCUR_STAGE_RF_ATZ, BCUR_STAGE_RF_REDUCE, py, n, l, m, true, A, lda, b.Z, lp, b.Y, lp,
                         b.part));
    }
    HIPCHK(hipMemcpy2DAsync(Y, ldy * sizeof(float), b.Y, lp * sizeof(float), l * sizeof(float), n,
                            hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BCUR_OK;
}

bcur_status bcur_block_scores(bcur_ctx* ctx, const float* V, int64_t n, int64_t k, int64_t ldv, const int64_t* offsets,
                              int64_t G, double* scores) {
    GUARD(ctx);
    if (!ctx || !V || !scores) return fail(ctx, BCUR_E_ARG, "null argument");
    if (n < 1 || k < 1 || ldv < k) return fail(ctx, BCUR_E_ARG, "bad V shape");
    STCHK(check_offsets(ctx, offsets, G, n, "offsets"));
    HIPCHK(hipSetDevice(ctx->device));
    Arena a;
    a.take<int64_t>(G + 1);
    a.take<double>(G);
    STCHK(reserve(ctx, a.off));
    Arena b{ctx->ws, 0};
    int64_t* d_off = b.take<int64_t>(G + 1);
    double* d_sc = b.take<double>(G);
    HIPCHK(hipMemcpyAsync(d_off, offsets, (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    {
        StageScope ts(ctx, BCUR_STAGE_SCORES);
        HIPCHK(launch_block_scores(V, k, ldv, d_off, G, d_sc, ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(scores, d_sc, G * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BCUR_OK;
}

bcur_status bcur_block_stable_rank(bcur_ctx* ctx, const float* V, int64_t n, int64_t k, int64_t ldv,
                                   const int64_t* offsets, int64_t G, const int64_t* col_map, double* ratios,
                                   int32_t* steps, double* alpha) {
    GUARD(ctx);
    if (!ctx || !V || !alpha) return fail(ctx, BCUR_E_ARG, "null argument");
    if (n < 1 || k < 1 || ldv < k) return fail(ctx, BCUR_E_ARG, "bad V shape");
    STCHK(check_offsets(ctx, offsets, G, n, "offsets"));
    STCHK(check_map(ctx, col_map, n, "col_map"));
    for (int64_t g = 0; g < G; ++g)
        if (std::min(offsets[g + 1] - offsets[g], k) > kDiagMaxD)
            return fail(ctx, BCUR_E_ARG, "block %lld: min(width, k) exceeds %d", (long long)g, kDiagMaxD);
    HIPCHK(hipSetDevice(ctx->device));
    Arena a;
    a.take<int64_t>(G + 1);
    a.take<double>(G);
    a.take<int>(G);
    if (col_map) {
        a.take<int64_t>(n);
        a.take<float>(n * k);
    }
    STCHK(reserve(ctx, a.off));
    Arena b{ctx->ws, 0};
    int64_t* d_off = b.take<int64_t>(G + 1);
    double* d_r = b.take<double>(G);
    int* d_steps = b.take<int>(G);
    int64_t* d_map = col_map ? b.take<int64_t>(n) : nullptr;
    float* Vp = col_map ? b.take<float>(n * k) : nullptr;
    std::vector<double> hr(G);
    std::vector<int> hs(G);
    HIPCHK(hipMemcpyAsync(d_off, offsets, (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    if (col_map) {
        // the rows of V in map order, so every block is a contiguous slice
        HIPCHK(hipMemcpyAsync(d_map, col_map, n * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(launch_gather_rows(V, ldv, k, d_map, n, Vp, k, ctx->stream));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_DIAG_ALPHA);
        HIPCHK(launch_block_stable_rank(col_map ? Vp : V, k, col_map ? k : ldv, d_off, G, d_r, d_steps,
                                        ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(hr.data(), d_r, G * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(hs.data(), d_steps, G * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (steps)
        for (int64_t g = 0; g < G; ++g) steps[g] = hs[g];
    double mn = NAN;
    for (int64_t g = 0; g < G; ++g)
        if (!isnan(hr[g]) && !(hr[g] >= mn)) mn = hr[g];
    if (ratios) memcpy(ratios, hr.data(), G * sizeof(double));
    *alpha = mn;
    return BCUR_OK;
}

bcur_status bcur_incoherence(bcur_ctx* ctx, const float* U, int64_t m, int64_t k, int64_t ldu, double* mu) {
    GUARD(ctx);
    if (!ctx || !U || !mu) return fail(ctx, BCUR_E_ARG, "null argument");
    if (m < 1 || k < 1 || ldu < k) return fail(ctx, BCUR_E_ARG, "bad U shape");
    HIPCHK(hipSetDevice(ctx->device));
    Arena a;
    a.take<double>(row_norm_grid(m));
    a.take<double>(1);
    STCHK(reserve(ctx, a.off));
    Arena b{ctx->ws, 0};
    double* part = b.take<double>(row_norm_grid(m));
    double* d_mu = b.take<double>(1);
    double h = 0.0;
    {
        StageScope ts(ctx, BCUR_STAGE_DIAG_MU);
        HIPCHK(launch_incoherence(U, m, k, ldu, part, d_mu, ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(&h, d_mu, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *mu = h;
    return BCUR_OK;
}

bcur_status bcur_sample_blocks(bcur_ctx* ctx, const double* scores, int64_t G, const uint64_t* draws, int64_t s,
                               int32_t replace, int64_t* idx, double* weights, double* margins) {
    GUARD(ctx);
    if (!ctx || !scores || !draws || !idx) return fail(ctx, BCUR_E_ARG, "null argument");
    if (G < 1 || s < 1 || (!replace && s > G)) return fail(ctx, BCUR_E_ARG, "need 1 <= s <= G (without replacement)");
    HIPCHK(hipSetDevice(ctx->device));
    Arena a;
    a.take<double>(G);
    a.take<uint64_t>(s);
    a.take<uint64_t>(G);
    a.take<uint64_t>(G);
    a.take<int64_t>(s);
    a.take<double>(s);
    a.take<double>(s);
    a.take<int>(4);
    STCHK(reserve(ctx, a.off));
    Arena b{ctx->ws, 0};
    double* d_sc = b.take<double>(G);
    uint64_t* d_dr = b.take<uint64_t>(s);
    uint64_t* qb = b.take<uint64_t>(G);
    uint64_t* pr = b.take<uint64_t>(G);
    int64_t* d_idx = b.take<int64_t>(s);
    double* d_w = b.take<double>(s);
    double* d_mg = b.take<double>(s);
    int* d_st = b.take<int>(4);
    hipStream_t st = ctx->stream;
    HIPCHK(hipMemcpyAsync(d_sc, scores, G * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_dr, draws, s * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(d_st, 0, 4 * sizeof(int), st));
    HIPCHK(launch_sample(d_sc, G, d_dr, s, replace, qb, pr, d_idx, d_w, d_mg, d_st, st));
    int hst[4];
    std::vector<int64_t> hidx(s);
    std::vector<double> hw(s), hm(s);
    HIPCHK(hipMemcpyAsync(hst, d_st, sizeof hst, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hidx.data(), d_idx, s * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hw.data(), d_w, s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hm.data(), d_mg, s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hst[0] != 0) return fail(ctx, BCUR_E_ARG, "scores must be finite and non-negative");
    memcpy(idx, hidx.data(), s * sizeof(int64_t));
    if (weights) memcpy(weights, hw.data(), s * sizeof(double));
    if (margins) memcpy(margins, hm.data(), s * sizeof(double));
    return BCUR_OK;
}

bcur_status bcur_gather_columns(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* offsets,
                                int64_t G, const int64_t* idx, int64_t s, float* C, int64_t ldc, int64_t* c_out) {
    GUARD(ctx);
    if (!ctx || !idx || !C || !c_out) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_offsets(ctx, offsets, G, n, "offsets"));
    if (s < 1) return fail(ctx, BCUR_E_ARG, "s < 1");
    for (int64_t t = 0; t < s; ++t)
        if (idx[t] < 0 || idx[t] >= G) return fail(ctx, BCUR_E_ARG, "idx[%lld] out of range", (long long)t);
    const std::vector<int64_t> cols = expand_blocks(offsets, idx, s);
    const int64_t c = (int64_t)cols.size();
    if (ldc < c) return fail(ctx, BCUR_E_ARG, "ldc %lld < c = %lld", (long long)ldc, (long long)c);
    HIPCHK(hipSetDevice(ctx->device));
    STCHK(reserve(ctx, c * sizeof(int64_t) + 256));
    int64_t* d_cols = reinterpret_cast<int64_t*>(ctx->ws);
    STCHK(reserve_pinned(ctx, c * sizeof(int64_t)));
    HIPCHK(hipStreamSynchronize(ctx->stream));   // the pinned staging buffer may still be read by a copy
    memcpy(ctx->pinned, cols.data(), c * sizeof(int64_t));
    HIPCHK(hipMemcpyAsync(d_cols, ctx->pinned, c * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    ctx->pinned_busy = true;  // the copy may still read the staging buffer when this returns
    HIPCHK(launch_gather_cols(A, lda, m, d_cols, c, C, ldc, ctx->stream));
    *c_out = c;
    return BCUR_OK;
}

bcur_status bcur_fit_columns(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* C, int64_t c,
                             int64_t ldc, int32_t refine, float* U, int64_t ldu, double* err, uint32_t* flags) {
    GUARD(ctx);
    if (!ctx || !U || !err) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_matrix(ctx, C, m, c, ldc, "C"));
    if (ldu < n || (ldu & 3) || !aligned16(U)) return fail(ctx, BCUR_E_ARG, "U: bad leading dimension or alignment");
    if (refine < 0 || refine > 1) return fail(ctx, BCUR_E_ARG, "refine must be 0 or 1");
    HIPCHK(hipSetDevice(ctx->device));
    FitBufs b;
    int64_t* d_id = nullptr;
    {
        Arena a;
        fit_layout(a, b, m, n, c, true);
        a.take<int64_t>(c);
        STCHK(reserve(ctx, a.off));
        Arena r{ctx->ws, 0};
        fit_layout(r, b, m, n, c, true);
        d_id = r.take<int64_t>(c);
    }
    STCHK(reserve_pinned(ctx, c * sizeof(int64_t)));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int64_t* h_id = reinterpret_cast<int64_t*>(ctx->pinned);
    for (int64_t i = 0; i < c; ++i) h_id[i] = i;
    HIPCHK(hipMemcpyAsync(d_id, h_id, c * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    STCHK(fit_run(ctx, b, A, m, n, lda, C, c, ldc, nullptr, d_id, refine, U, ldu));
    FitOut fo;
    STCHK(fit_collect(ctx, b, A, m, n, lda, C, c, ldc, U, ldu, &fo));
    *err = sqrt(fo.err2);
    if (flags) *flags = fo.flags;
    return BCUR_OK;
}

}  // extern "C"

namespace {

bcur_status decompose_impl(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* col_off,
                           int64_t G, const int64_t* row_off, int64_t Gr, const bcur_params* p, const float* omega,
                           const uint64_t* draws, bcur_result* res) {
    if (!p || !res || !draws || !res->idx) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_offsets(ctx, col_off, G, n, "col_off"));
    const int64_t k = p->k, l = p->l, s = p->s, q = p->q;
    if (k < 1 || l < k || l > std::min(std::min(m, n), kMaxSketch))
        return fail(ctx, BCUR_E_ARG, "need 1 <= k <= l <= min(m, n, %lld)", (long long)kMaxSketch);
    if (q < 0 || q > 64) return fail(ctx, BCUR_E_ARG, "q out of range");
    if (s < 1 || (!p->replace && s > G)) return fail(ctx, BCUR_E_ARG, "need 1 <= s <= G without replacement");
    if (p->precision != BCUR_PREC_FP32 && p->precision != BCUR_PREC_BF16)
        return fail(ctx, BCUR_E_ARG, "unknown precision %d", p->precision);
    const bool bf16 = p->precision == BCUR_PREC_BF16;
    if (p->refine < 0 || p->refine > 1) return fail(ctx, BCUR_E_ARG, "refine must be 0 or 1");
    const bool rowv = row_off != nullptr && p->s_r > 0;
    const int64_t s_r = rowv ? p->s_r : 0;
    if (rowv) {
        STCHK(check_offsets(ctx, row_off, Gr, m, "row_off"));
        if (!p->replace && s_r > Gr) return fail(ctx, BCUR_E_ARG, "s_r > Gr without replacement");
        if (!res->idx_r) return fail(ctx, BCUR_E_ARG, "idx_r is required for the row-block variant");
    }
    STCHK(check_map(ctx, p->col_map, n, "col_map"));
    const int64_t* rmap_h = rowv ? p->row_map : nullptr;
    STCHK(check_map(ctx, rmap_h, m, "row_map"));
    int64_t maxw = 0, maxh = 0;
    for (int64_t g = 0; g < G; ++g) maxw = std::max(maxw, col_off[g + 1] - col_off[g]);
    if (rowv)
        for (int64_t g = 0; g < Gr; ++g) maxh = std::max(maxh, row_off[g + 1] - row_off[g]);
    const int64_t cmax = std::min(s * maxw, n);
    const int64_t rmax = rowv ? std::min(s_r * maxh, m) : 0;
    const int64_t ucols = rowv ? rmax : n;
    if (res->U && (res->ldu < ucols || (res->ldu & 3) || !aligned16(res->U) || res->u_rows_cap < cmax))
        return fail(ctx, BCUR_E_ARG, "U needs ldu >= %lld (a multiple of 4, 16-byte aligned) and %lld rows",
                    (long long)ucols, (long long)cmax);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;

    // workspace: range finder | sampling (columns, rows) | C, V_k, U_k | fit
    RFBufs rb;
    FitBufs fb;
    CurBufs cb;
    SampleBufs sc, sr;
    double *d_frob, *d_fpart;
    float *Vk, *Uk, *Cbuf, *Ubuf, *Vp = nullptr, *Up = nullptr;
    int64_t *d_cmap = nullptr, *d_rmap = nullptr;
    auto layout = [&](Arena& a) {
        rf_layout(a, rb, m, n, l, k, bf16);
        sample_layout(a, sc, G, s, cmax);
        d_frob = a.take<double>(2);
        if (rowv) sample_layout(a, sr, Gr, s_r, rmax);
        d_fpart = a.take<double>(frob2_grid(m, n));
        Vk = a.take<float>(n * k);
        Uk = rowv ? a.take<float>(m * k) : nullptr;
        if (p->col_map) {
            d_cmap = a.take<int64_t>(n);
            Vp = a.take<float>(n * k);
        }
        if (rmap_h) {
            d_rmap = a.take<int64_t>(m);
            Up = a.take<float>(m * k);
        }
        Cbuf = a.take<float>(m * round4(cmax));
        Ubuf = res->U ? nullptr : a.take<float>(cmax * round4(ucols));
        if (rowv) cur_layout(a, cb, m, n, cmax, rmax);
        else fit_layout(a, fb, m, n, cmax, false);
    };
    {
        Arena a;
        layout(a);
        STCHK(reserve(ctx, a.off));
        Arena b{ctx->ws, 0};
        layout(b);
    }
    // pinned staging: offsets | draws | frob2 | status | idx, w, mg | scores | lam | list
    // (for the rows the same again after the columns)
    auto side_bytes = [](int64_t g, int64_t ss, int64_t lm) {
        return 8 * (g + 1) + 8 * ss + (24 * ss + 16 + 8 * g + 16 + 5 * 256) + 8 * lm + 16;
    };
    // (+256 per merged span: offsets | draws, lam | info keep their workspace padding)
    const size_t pin_need = side_bytes(G, s, cmax) + (rowv ? side_bytes(Gr, s_r, rmax) : 0) + 16 + 8 * l + 64 +
                            (p->col_map ? 8 * n + 8 : 0) + (rmap_h ? 8 * m + 8 : 0) + 3 * 256 +
                            (rowv ? 0 : fit_collect_bytes(fb) + 8);
    STCHK(reserve_pinned(ctx, pin_need));
    if (ctx->pinned_busy) HIPCHK(hipStreamSynchronize(st));
    ctx->pinned_busy = true;
    char* pin = ctx->pinned;
    auto ptake = [&pin](size_t bytes) {
        char* p0 = pin;
        pin += (bytes + 7) & ~(size_t)7;
        return p0;
    };
    // offsets and draws (consecutive in the workspace) go up in one copy per side
    auto upload_side = [&](const SampleBufs& b, const int64_t* off_src, int64_t g, const uint64_t* dr_src,
                           int64_t ss) -> int64_t* {
        const char* d0 = reinterpret_cast<const char*>(b.off);
        const size_t span = (size_t)(reinterpret_cast<const char*>(b.dr + ss) - d0);
        char* h0 = ptake(span);
        int64_t* h_off = reinterpret_cast<int64_t*>(h0);
        memcpy(h_off, off_src, (g + 1) * sizeof(int64_t));
        memcpy(h0 + (reinterpret_cast<const char*>(b.dr) - d0), dr_src, ss * sizeof(uint64_t));
        return hipMemcpyAsync(b.off, h0, span, hipMemcpyHostToDevice, st) == hipSuccess ? h_off : nullptr;
    };
    if (!upload_side(sc, col_off, G, draws, s)) return fail(ctx, BCUR_E_HIP, "upload of the offsets failed");
    HIPCHK(hipMemsetAsync(sc.st, 0, 4 * sizeof(int), st));
    int64_t* h_roff = nullptr;
    if (rowv) {
        h_roff = upload_side(sr, row_off, Gr, draws + s, s_r);
        if (!h_roff) return fail(ctx, BCUR_E_HIP, "upload of the row offsets failed");
        HIPCHK(hipMemsetAsync(sr.st, 0, 4 * sizeof(int), st));
    }
    if (p->col_map) {
        int64_t* h_cm = reinterpret_cast<int64_t*>(ptake(8 * n));
        memcpy(h_cm, p->col_map, n * sizeof(int64_t));
        HIPCHK(hipMemcpyAsync(d_cmap, h_cm, n * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    if (rmap_h) {
        int64_t* h_rm = reinterpret_cast<int64_t*>(ptake(8 * m));
        memcpy(h_rm, rmap_h, m * sizeof(int64_t));
        HIPCHK(hipMemcpyAsync(d_rmap, h_rm, m * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }

    // 1. ||A||_F^2 (summed by the range finder's first FP32 pass over A when it has one)
    const bool fused_frob = range_finder_fuses_frob(q, p->precision);
    if (!fused_frob) {
        StageScope ts(ctx, BCUR_STAGE_FROB);
        HIPCHK(launch_frob2(A, m, n, lda, d_fpart, frob2_grid(m, n), d_frob, st));
    }
    // 2. sketched top-k right subspace (and left vectors for the row blocks)
    STCHK(range_finder_run(ctx, rb, A, m, n, lda, omega, p->seed, l, k, q, Vk, Uk, p->precision,
                           fused_frob ? d_frob : nullptr));
    // 3. block scores (with a map, over the rows of V_k (U_k) listed in map
    // order, so each block's rows are contiguous), 4. sampling
    {
        StageScope ts(ctx, BCUR_STAGE_SCORES);
        if (d_cmap) HIPCHK(launch_gather_rows(Vk, k, k, d_cmap, n, Vp, k, st));
        if (d_rmap) HIPCHK(launch_gather_rows(Uk, k, k, d_rmap, m, Up, k, st));
        HIPCHK(launch_block_scores(d_cmap ? Vp : Vk, k, k, sc.off, G, sc.sc, st));
        if (rowv) HIPCHK(launch_block_scores(d_rmap ? Up : Uk, k, k, sr.off, Gr, sr.sc, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_SAMPLE);
        HIPCHK(launch_sample(sc.sc, G, sc.dr, s, p->replace, sc.qb, sc.pr, sc.idx, sc.w, sc.mg, sc.st, st));
        if (rowv)
            HIPCHK(launch_sample(sr.sc, Gr, sr.dr, s_r, p->replace, sr.qb, sr.pr, sr.idx, sr.w, sr.mg, sr.st, st));
    }
    // results needed on the host to lay out C (and R)
    struct HostSide {
        int* st;
        int64_t* idx;
        double *w, *mg, *sc;
        int64_t* list;
    };
    // one copy per side: the device results from idx to the end of sc (for
    // the columns also d_frob, laid out right after), mirrored on the host
    auto stage_side = [&](const SampleBufs& b, int64_t lm, const char* dev_end, HostSide& h) -> bcur_status {
        const char* d0 = reinterpret_cast<const char*>(b.idx);
        const size_t span = (size_t)(dev_end - d0);
        char* h0 = ptake(span);
        auto mirror = [&](const void* dp) { return h0 + (reinterpret_cast<const char*>(dp) - d0); };
        h.idx = reinterpret_cast<int64_t*>(mirror(b.idx));
        h.w = reinterpret_cast<double*>(mirror(b.w));
        h.mg = reinterpret_cast<double*>(mirror(b.mg));
        h.st = reinterpret_cast<int*>(mirror(b.st));
        h.sc = reinterpret_cast<double*>(mirror(b.sc));
        h.list = reinterpret_cast<int64_t*>(ptake(8 * std::max<int64_t>(lm, 1)));
        HIPCHK(hipMemcpyAsync(h0, d0, span, hipMemcpyDeviceToHost, st));
        return BCUR_OK;
    };
    HostSide hc{}, hr{};
    STCHK(stage_side(sc, cmax, reinterpret_cast<const char*>(d_frob + 1), hc));
    const double* h_frob = reinterpret_cast<const double*>(reinterpret_cast<const char*>(hc.idx) +
                                                           (reinterpret_cast<const char*>(d_frob) -
                                                            reinterpret_cast<const char*>(sc.idx)));
    if (rowv) STCHK(stage_side(sr, rmax, reinterpret_cast<const char*>(sr.sc + Gr), hr));
    // lam and info (consecutive in the workspace) come back in one copy
    const char* rf0 = reinterpret_cast<const char*>(rb.lam);
    const size_t rf_span = (size_t)(reinterpret_cast<const char*>(rb.info + 4) - rf0);
    char* h_rf = ptake(rf_span);
    double* h_lam = reinterpret_cast<double*>(h_rf);
    int* rinfo = reinterpret_cast<int*>(h_rf + (reinterpret_cast<const char*>(rb.info) - rf0));
    // The checks of the draws, once their results are on the host.
    auto check_draws = [&]() -> bcur_status {
        if (!isfinite(h_frob[0])) return fail(ctx, BCUR_E_NONFINITE, "A holds NaN or Inf");
        if (hc.st[0] != 0 || (rowv && hr.st[0] != 0)) return fail(ctx, BCUR_E_HIP, "block scores are not finite");
        for (int64_t t = 0; t < s; ++t)
            if (hc.idx[t] < 0 || hc.idx[t] >= G) return fail(ctx, BCUR_E_HIP, "sampler returned an invalid block");
        for (int64_t t = 0; t < s_r; ++t)
            if (hr.idx[t] < 0 || hr.idx[t] >= Gr)
                return fail(ctx, BCUR_E_HIP, "sampler returned an invalid row block");
        return BCUR_OK;
    };
    // Blocks of one width drawn without replacement: c = s b (and r = s_r h) is
    // known, so the lists are expanded on the device and the path runs to its
    // end without a host round trip; the draws are checked after the fit's
    // synchronization.  Otherwise the host expands the chosen blocks (dropping
    // repeats) before the gather.
    const int64_t bw = uniform_width(col_off, G), bh = rowv ? uniform_width(row_off, Gr) : 0;
    const bool on_device = !p->replace && bw > 0 && (!rowv || bh > 0);
    int64_t c = 0, r = 0;
    if (on_device) {
        c = s * bw;
        HIPCHK(launch_expand_blocks(sc.idx, s, sc.off, G, d_cmap, bw, sc.list, st));
        if (rowv) {
            r = s_r * bh;
            HIPCHK(launch_expand_blocks(sr.idx, s_r, sr.off, Gr, d_rmap, bh, sr.list, st));
        }
    } else {
        HIPCHK(hipStreamSynchronize(st));
        STCHK(check_draws());
        c = expand_blocks_into(col_off, hc.idx, s, p->col_map, hc.list, cmax);
        HIPCHK(hipMemcpyAsync(sc.list, hc.list, c * sizeof(int64_t), hipMemcpyHostToDevice, st));
        if (rowv) {
            r = expand_blocks_into(row_off, hr.idx, s_r, rmap_h, hr.list, rmax);
            HIPCHK(hipMemcpyAsync(sr.list, hr.list, r * sizeof(int64_t), hipMemcpyHostToDevice, st));
        }
    }
    // 5. C = A S (unscaled) and R = S_R^T A
    const int64_t ldc = round4(c);
    {
        StageScope ts(ctx, BCUR_STAGE_GATHER);
        HIPCHK(launch_gather_cols(A, lda, m, sc.list, c, Cbuf, ldc, st));
        if (rowv) HIPCHK(launch_gather_rows(A, lda, n, sr.list, r, cb.R, round4(n), st));
    }
    // results the host reads after the fit's synchronization
    HIPCHK(hipMemcpyAsync(h_rf, rf0, rf_span, hipMemcpyDeviceToHost, st));
    // 6. U and the residual
    float* U = res->U ? res->U : Ubuf;
    const int64_t ldu = res->U ? res->ldu : round4(ucols);
    double err2 = 0.0;
    uint32_t fl = 0;
    double cond_est = 0.0;
    if (rowv) {
        STCHK(fit_cur_run(ctx, cb, A, m, n, lda, Cbuf, c, ldc, r, U, ldu));
        double hv[4];
        int hinfo[4];
        HIPCHK(hipMemcpyAsync(hv, cb.errv, sizeof hv, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hinfo, cb.info, sizeof hinfo, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        err2 = std::max(hv[0], 0.0);
        if ((hinfo[0] | hinfo[2]) & 1) fl |= BCUR_FLAG_RANKDEF_C;
        if (hinfo[1] & 1) fl |= BCUR_FLAG_RANKDEF_R;
    } else {
        STCHK(fit_run(ctx, fb, A, m, n, lda, Cbuf, c, ldc, sc.list, nullptr, p->refine, U, ldu));
        FitOut fo;
        char* h_fit = ptake(fit_collect_bytes(fb));
        STCHK(fit_collect(ctx, fb, A, m, n, lda, Cbuf, c, ldc, U, ldu, &fo, h_fit));
        err2 = fo.err2;
        fl = fo.flags;
        cond_est = fo.cond_est;
    }
    ctx->pinned_busy = false;  // the fit's synchronization completed every copy
    if (on_device) STCHK(check_draws());
    if (rinfo[0] & 1) fl |= BCUR_FLAG_RANKDEF_Y;
    if (hc.st[1] || (rowv && hr.st[1])) fl |= BCUR_FLAG_ZERO_SCORE;
    memcpy(res->idx, hc.idx, s * sizeof(int64_t));
    if (res->weights) memcpy(res->weights, hc.w, s * sizeof(double));
    if (res->scores) memcpy(res->scores, hc.sc, G * sizeof(double));
    if (rowv) {
        memcpy(res->idx_r, hr.idx, s_r * sizeof(int64_t));
        if (res->row_scores) memcpy(res->row_scores, hr.sc, Gr * sizeof(double));
    }
    if (res->ritz)
        for (int64_t i = 0; i < l; ++i) res->ritz[i] = h_lam[i] > 0.0 ? sqrt(h_lam[i]) : 0.0;
    double mm = INFINITY;
    for (int64_t t = 0; t < s; ++t) mm = std::min(mm, hc.mg[t]);
    res->c = c;
    res->r = r;
    res->frob2 = h_frob[0];
    res->err = sqrt(err2);
    res->rel_err = h_frob[0] > 0.0 ? res->err / sqrt(h_frob[0]) : 0.0;
    res->min_margin = mm;
    res->flags = fl;
    res->rr_sweeps = (uint32_t)rinfo[2];
    // lam_1 / (lam_k - lam_{k+1}) of the Ritz values: the sensitivity of the
    // top-k subspace, and so of the scores, to perturbations of A
    const double gap = k < l ? h_lam[k - 1] - h_lam[k] : 0.0;
    res->kappa = k >= l ? 1.0 : (gap > 0.0 ? h_lam[0] / gap : INFINITY);
    res->cond_c = cond_est;
    return BCUR_OK;
}

}  // namespace

extern "C" {

bcur_status bcur_decompose(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* col_off,
                           int64_t G, const int64_t* row_off, int64_t Gr, const bcur_params* p, const float* omega,
                           const uint64_t* draws, bcur_result* res) {
    GUARD(ctx);
    return decompose_impl(ctx, A, m, n, lda, col_off, G, row_off, Gr, p, omega, draws, res);
}

bcur_status bcur_decompose_async(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                 const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                                 const bcur_params* p, const float* omega, const uint64_t* draws, bcur_result* res) {
    GUARD(ctx);
    if (!p || !res || !draws || !res->idx || !col_off) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_offsets(ctx, col_off, G, n, "col_off"));
    const bool rowv = row_off != nullptr && p->s_r > 0;
    if (rowv) STCHK(check_offsets(ctx, row_off, Gr, m, "row_off"));
    if (p->s < 1 || p->s_r < 0) return fail(ctx, BCUR_E_ARG, "need s >= 1 and s_r >= 0");
    AsyncJob& j = ctx->job;
    j.A = A;
    j.m = m;
    j.n = n;
    j.lda = lda;
    j.G = G;
    j.Gr = rowv ? Gr : 0;
    j.col_off.assign(col_off, col_off + G + 1);
    if (rowv) j.row_off.assign(row_off, row_off + Gr + 1);
    else j.row_off.clear();
    j.draws.assign(draws, draws + p->s + (rowv ? p->s_r : 0));
    j.p = *p;
    if (p->col_map) j.col_map.assign(p->col_map, p->col_map + n);
    else j.col_map.clear();
    if (rowv && p->row_map) j.row_map.assign(p->row_map, p->row_map + m);
    else j.row_map.clear();
    j.p.col_map = j.col_map.empty() ? nullptr : j.col_map.data();
    j.p.row_map = j.row_map.empty() ? nullptr : j.row_map.data();
    j.omega = omega;
    j.res = res;
    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->astream) HIPCHK(hipStreamCreateWithFlags(&ctx->astream, hipStreamNonBlocking));
    if (!ctx->ev_in) HIPCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ctx->ev_in, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->astream, ctx->ev_in, 0));
    ctx->inflight = true;
    ctx->worker = std::thread([ctx]() {
        AsyncJob& jb = ctx->job;
        if (hipSetDevice(ctx->device) != hipSuccess) {
            ctx->job_status = fail(ctx, BCUR_E_HIP, "hipSetDevice failed on the context's host thread");
            return;
        }
        hipStream_t caller = ctx->stream;
        ctx->stream = ctx->astream;
        ctx->job_status = decompose_impl(ctx, jb.A, jb.m, jb.n, jb.lda, jb.col_off.data(), jb.G,
                                         jb.row_off.empty() ? nullptr : jb.row_off.data(), jb.Gr, &jb.p, jb.omega,
                                         jb.draws.data(), jb.res);
        // a failed call may have left work queued: finish it before the stream is handed back
        (void)hipStreamSynchronize(ctx->astream);
        ctx->stream = caller;
    });
    return BCUR_OK;
}

bcur_status bcur_wait(bcur_ctx* ctx) {
    if (!ctx) return BCUR_E_ARG;
    if (!ctx->inflight) return BCUR_OK;
    ctx->worker.join();
    ctx->inflight = false;
    return ctx->job_status;
}

bcur_status bcur_decompose_noalloc(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                   const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                                   const bcur_params* p, const float* omega, const uint64_t* draws, bcur_result* res) {
    GUARD(ctx);
    if (!p || !res) return fail(ctx, BCUR_E_ARG, "null argument");
    if (p->col_map || (row_off && p->s_r > 0 && p->row_map))
        return fail(ctx, BCUR_E_ARG, "block maps are not taken without allocation: use bcur_decompose");
    if (!res->U) return fail(ctx, BCUR_E_ARG, "U must be a caller buffer without allocation");
    if (ctx->device >= kMaxDevices || !g_scratch[ctx->device])
        return fail(ctx, BCUR_E_HIP, "no scratch array on device %d", ctx->device);
    // the device's scratch array and host staging stand in for the context's
    // workspace and pinned buffer for this call; nothing is allocated
    char* const ws = ctx->ws;
    const size_t ws_bytes = ctx->ws_bytes;
    char* const pinned = ctx->pinned;
    const size_t pinned_bytes = ctx->pinned_bytes;
    const bool pinned_busy = ctx->pinned_busy, timing = ctx->timer.on;
    ctx->ws = static_cast<char*>(g_scratch[ctx->device]);
    ctx->ws_bytes = kScratchBytes;
    ctx->pinned = g_host_stage[ctx->device];
    ctx->pinned_bytes = kHostStageBytes;
    ctx->pinned_busy = false;
    ctx->timer.on = false;   // stage events are not recorded by this call
    ctx->noalloc = true;
    const bcur_status st = decompose_impl(ctx, A, m, n, lda, col_off, G, row_off, Gr, p, omega, draws, res);
    // a failed call may leave copies through the shared staging in flight
    if (st != BCUR_OK) (void)hipStreamSynchronize(ctx->stream);
    ctx->noalloc = false;
    ctx->ws = ws;
    ctx->ws_bytes = ws_bytes;
    ctx->pinned = pinned;
    ctx->pinned_bytes = pinned_bytes;
    ctx->pinned_busy = pinned_busy;
    ctx->timer.on = timing;
    return st;
}

bcur_status bcur_decompose_boost(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                 const int64_t* col_off, int64_t G, const bcur_params* p, const float* omega,
                                 int64_t t, const uint64_t* draws, bcur_result* res, double* errs, int64_t* best_out) {
    if (!ctx) return BCUR_E_ARG;
    GUARD(ctx);
    if (!p || !res || !draws || !res->idx || !errs) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_offsets(ctx, col_off, G, n, "col_off"));
    const int64_t k = p->k, l = p->l, s = p->s, q = p->q;
    if (t < 1 || t > kMaxTrials) return fail(ctx, BCUR_E_ARG, "need 1 <= t <= %lld", (long long)kMaxTrials);
    if (k < 1 || l < k || l > std::min(std::min(m, n), kMaxSketch))
        return fail(ctx, BCUR_E_ARG, "need 1 <= k <= l <= min(m, n, %lld)", (long long)kMaxSketch);
    if (q < 0 || q > 64) return fail(ctx, BCUR_E_ARG, "q out of range");
    if (s < 1 || (!p->replace && s > G)) return fail(ctx, BCUR_E_ARG, "need 1 <= s <= G without replacement");
    if (p->precision != BCUR_PREC_FP32 && p->precision != BCUR_PREC_BF16)
        return fail(ctx, BCUR_E_ARG, "unknown precision %d", p->precision);
    if (p->refine < 0 || p->refine > 1) return fail(ctx, BCUR_E_ARG, "refine must be 0 or 1");
    if (p->s_r != 0) return fail(ctx, BCUR_E_ARG, "boosting covers the column-block path only (s_r = 0)");
    STCHK(check_map(ctx, p->col_map, n, "col_map"));
    const bool bf16 = p->precision == BCUR_PREC_BF16;
    int64_t maxw = 0;
    for (int64_t g = 0; g < G; ++g) maxw = std::max(maxw, col_off[g + 1] - col_off[g]);
    const int64_t cmax = std::min(s * maxw, n), cseg = round4(cmax), ctot_max = t * cseg;
    if (res->U && (res->ldu < n || (res->ldu & 3) || !aligned16(res->U) || res->u_rows_cap < cmax))
        return fail(ctx, BCUR_E_ARG, "U needs ldu >= %lld (a multiple of 4, 16-byte aligned) and %lld rows",
                    (long long)n, (long long)cmax);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t np = round4(n);

    // workspace: range finder | scores and the trials' draws and results | C of all trials, H of all
    // trials | one fit's buffers | two U buffers
    RFBufs rb;
    FitBufs fb;
    double *d_frob, *d_fpart, *d_sc, *d_w, *d_mg;
    int64_t *d_off, *d_idx, *d_list;
    uint64_t *d_dr, *d_qb, *d_pr;
    int* d_st;
    float *Vk, *Call, *Hall, *hpart, *Ua, *Ub, *Vp = nullptr;
    int64_t* d_cmap = nullptr;
    // split-K partials of the all-trials H GEMM: the largest over the column
    // counts it can have (multiples of 4 up to ctot_max)
    size_t hpart_floats = 4;
    for (int64_t cc = 4; cc <= ctot_max; cc += 4)
        hpart_floats = std::max(hpart_floats, sgemm_partial_floats(plan_sgemm(cc, n, m, true, true), cc, n));
    auto layout = [&](Arena& a) {
        rf_layout(a, rb, m, n, l, k, bf16);
        d_off = a.take<int64_t>(G + 1);
        d_dr = a.take<uint64_t>(t * s);
        d_qb = a.take<uint64_t>(G);
        d_pr = a.take<uint64_t>(G);
        d_list = a.take<int64_t>(ctot_max);
        // read back in one copy: idx .. frob
        d_idx = a.take<int64_t>(t * s);
        d_w = a.take<double>(t * s);
        d_mg = a.take<double>(t * s);
        d_st = a.take<int>(4 * t);
        d_sc = a.take<double>(G);
        d_frob = a.take<double>(2);
        d_fpart = a.take<double>(frob2_grid(m, n));
        Vk = a.take<float>(n * k);
        if (p->col_map) {
            d_cmap = a.take<int64_t>(n);
            Vp = a.take<float>(n * k);
        }
        Call = a.take<float>(m * ctot_max);
        Hall = a.take<float>(ctot_max * np);
        hpart = a.take<float>(hpart_floats);
        fit_layout(a, fb, m, n, cmax, false);
        Ua = a.take<float>(cmax * np);
        Ub = res->U ? nullptr : a.take<float>(cmax * np);
    };
    {
        Arena a;
        layout(a);
        STCHK(reserve(ctx, a.off));
        Arena b{ctx->ws, 0};
        layout(b);
    }
    const char* span0 = reinterpret_cast<const char*>(d_idx);
    const size_t span = (size_t)(reinterpret_cast<const char*>(d_frob + 1) - span0);
    const size_t pin_need =
        8 * (G + 1) + 8 * t * s + 8 * ctot_max + span + 8 * l + 64 + (p->col_map ? 8 * n : 0) + 2 * 256;
    STCHK(reserve_pinned(ctx, pin_need));
    if (ctx->pinned_busy) HIPCHK(hipStreamSynchronize(st));
    ctx->pinned_busy = true;
    char* pin = ctx->pinned;
    auto ptake = [&pin](size_t bytes) {
        char* p0 = pin;
        pin += (bytes + 7) & ~(size_t)7;
        return p0;
    };
    // offsets and draws (consecutive in the workspace) go up in one copy
    const char* in0 = reinterpret_cast<const char*>(d_off);
    const size_t in_span = (size_t)(reinterpret_cast<const char*>(d_dr + t * s) - in0);
    char* h_in = ptake(in_span);
    int64_t* h_off = reinterpret_cast<int64_t*>(h_in);
    uint64_t* h_dr = reinterpret_cast<uint64_t*>(h_in + (reinterpret_cast<const char*>(d_dr) - in0));
    int64_t* h_list = reinterpret_cast<int64_t*>(ptake(8 * ctot_max));
    char* h0 = ptake(span);
    // lam and info (consecutive in the workspace) come back in one copy
    const char* rf0 = reinterpret_cast<const char*>(rb.lam);
    const size_t rf_span = (size_t)(reinterpret_cast<const char*>(rb.info + 4) - rf0);
    char* h_rf = ptake(rf_span);
    double* h_lam = reinterpret_cast<double*>(h_rf);
    int* rinfo = reinterpret_cast<int*>(h_rf + (reinterpret_cast<const char*>(rb.info) - rf0));
    auto mirror = [&](const void* dp) { return h0 + (reinterpret_cast<const char*>(dp) - span0); };
    memcpy(h_off, col_off, (G + 1) * sizeof(int64_t));
    memcpy(h_dr, draws, t * s * sizeof(uint64_t));
    HIPCHK(hipMemcpyAsync(d_off, h_in, in_span, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(d_st, 0, 4 * t * sizeof(int), st));
    if (p->col_map) {
        int64_t* h_cm = reinterpret_cast<int64_t*>(ptake(8 * n));
        memcpy(h_cm, p->col_map, n * sizeof(int64_t));
        HIPCHK(hipMemcpyAsync(d_cmap, h_cm, n * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    const bool fused_frob = range_finder_fuses_frob(q, p->precision);
    if (!fused_frob) {
        StageScope ts(ctx, BCUR_STAGE_FROB);
        HIPCHK(launch_frob2(A, m, n, lda, d_fpart, frob2_grid(m, n), d_frob, st));
    }
    // one top-k subspace and one set of scores for every trial
    STCHK(range_finder_run(ctx, rb, A, m, n, lda, omega, p->seed, l, k, q, Vk, nullptr, p->precision,
                           fused_frob ? d_frob : nullptr));
    {
        StageScope ts(ctx, BCUR_STAGE_SCORES);
        if (d_cmap) HIPCHK(launch_gather_rows(Vk, k, k, d_cmap, n, Vp, k, st));
        HIPCHK(launch_block_scores(d_cmap ? Vp : Vk, k, k, d_off, G, d_sc, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_SAMPLE);
        for (int64_t i = 0; i < t; ++i)
            HIPCHK(launch_sample(d_sc, G, d_dr + i * s, s, p->replace, d_qb, d_pr, d_idx + i * s, d_w + i * s,
                                 d_mg + i * s, d_st + 4 * i, st));
    }
    HIPCHK(hipMemcpyAsync(h0, span0, span, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_rf, rf0, rf_span, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t* hidx = reinterpret_cast<const int64_t*>(mirror(d_idx));
    const double* hw = reinterpret_cast<const double*>(mirror(d_w));
    const double* hmg = reinterpret_cast<const double*>(mirror(d_mg));
    const int* hst = reinterpret_cast<const int*>(mirror(d_st));
    const double* hsc = reinterpret_cast<const double*>(mirror(d_sc));
    const double* hfrob = reinterpret_cast<const double*>(mirror(d_frob));
    if (!isfinite(hfrob[0])) return fail(ctx, BCUR_E_NONFINITE, "A holds NaN or Inf");
    uint32_t zero_drawn = 0;
    for (int64_t i = 0; i < t; ++i) {
        if (hst[4 * i] != 0) return fail(ctx, BCUR_E_HIP, "block scores are not finite");
        zero_drawn |= hst[4 * i + 1] ? 1u : 0u;
    }
    for (int64_t e = 0; e < t * s; ++e)
        if (hidx[e] < 0 || hidx[e] >= G) return fail(ctx, BCUR_E_HIP, "sampler returned an invalid block");
    // the trials' columns side by side, each segment starting at a multiple of 4
    // (padded with copies of its first column)
    std::vector<int64_t> seg_off(t), seg_c(t);
    int64_t ctot = 0;
    for (int64_t i = 0; i < t; ++i) {
        const std::vector<int64_t> cols = expand_blocks(col_off, hidx + i * s, s, p->col_map);
        const int64_t ci = (int64_t)cols.size();
        seg_off[i] = ctot;
        seg_c[i] = ci;
        for (int64_t j = 0; j < round4(ci); ++j) h_list[ctot + j] = cols[j < ci ? j : 0];
        ctot += round4(ci);
    }
    HIPCHK(hipMemcpyAsync(d_list, h_list, ctot * sizeof(int64_t), hipMemcpyHostToDevice, st));
    {
        StageScope ts(ctx, BCUR_STAGE_GATHER);
        HIPCHK(launch_gather_cols(A, lda, m, d_list, ctot, Call, ctot, st));
    }
    // H = C^T A for every trial at once: one GEMM over the concatenated columns
    const GemmPlan ph = plan_sgemm(ctot, n, m, true, true);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_H, BCUR_STAGE_FIT_REDUCE, ph, ctot, n, m, true, Call, ctot, A, lda, Hall, np,
                     hpart));
    float* Ubest = res->U ? res->U : Ub;
    const int64_t ldb = res->U ? res->ldu : np;
    float* Ucur = Ua;
    int64_t best = -1;
    double best_err2 = INFINITY;
    uint32_t best_flags = 0;
    double best_cond = 0.0;
    for (int64_t i = 0; i < t; ++i) {
        const float* Ci = Call + seg_off[i];
        STCHK(fit_run(ctx, fb, A, m, n, lda, Ci, seg_c[i], ctot, d_list + seg_off[i], nullptr, p->refine, Ucur, np,
                      Hall + seg_off[i] * np));
        FitOut fo;
        STCHK(fit_collect(ctx, fb, A, m, n, lda, Ci, seg_c[i], ctot, Ucur, np, &fo));
        errs[i] = sqrt(fo.err2);
        if (fo.err2 < best_err2) {
            best_err2 = fo.err2;
            best = i;
            best_flags = fo.flags;
            best_cond = fo.cond_est;
            HIPCHK(hipMemcpy2DAsync(Ubest, ldb * sizeof(float), Ucur, np * sizeof(float), n * sizeof(float),
                                    seg_c[i], hipMemcpyDeviceToDevice, st));
        }
    }
    if (best < 0) best = 0;   // every error was NaN: report the first trial
    HIPCHK(hipStreamSynchronize(st));
    ctx->pinned_busy = false;
    uint32_t fl = best_flags;
    if (rinfo[0] & 1) fl |= BCUR_FLAG_RANKDEF_Y;
    if (zero_drawn) fl |= BCUR_FLAG_ZERO_SCORE;
    memcpy(res->idx, hidx + best * s, s * sizeof(int64_t));
    if (res->weights) memcpy(res->weights, hw + best * s, s * sizeof(double));
    if (res->scores) memcpy(res->scores, hsc, G * sizeof(double));
    if (res->ritz)
        for (int64_t i = 0; i < l; ++i) res->ritz[i] = h_lam[i] > 0.0 ? sqrt(h_lam[i]) : 0.0;
    double mm = INFINITY;
    for (int64_t u = 0; u < s; ++u) mm = std::min(mm, hmg[best * s + u]);
    res->c = seg_c[best];
    res->r = 0;
    res->frob2 = hfrob[0];
    res->err = errs[best];
    res->rel_err = hfrob[0] > 0.0 ? res->err / sqrt(hfrob[0]) : 0.0;
    res->min_margin = mm;
    res->flags = fl;
    res->rr_sweeps = (uint32_t)rinfo[2];
    const double gap = k < l ? h_lam[k - 1] - h_lam[k] : 0.0;
    res->kappa = k >= l ? 1.0 : (gap > 0.0 ? h_lam[0] / gap : INFINITY);
    res->cond_c = best_cond;
    if (best_out) *best_out = best;
    return BCUR_OK;
}

// One run of Algorithm 1.  The workspace layout ends with ntail buffers of
// cmax x round4(r) floats; with tail_slot >= 0 the core goes to that buffer
// (ld round4(r)) instead of res->U, and *tail returns the first buffer.
static bcur_status alg1_impl(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                             const int64_t* col_off, int64_t G, const bcur_alg1_params* p, const uint64_t* draws,
                             bcur_alg1_result* res, int ntail, int tail_slot, float** tail) {
    if (!ctx) return BCUR_E_ARG;
    if (!p || !res || !draws || !res->rows || !res->idx) return fail(ctx, BCUR_E_ARG, "null argument");
    STCHK(check_matrix(ctx, A, m, n, lda, "A"));
    STCHK(check_offsets(ctx, col_off, G, n, "col_off"));
    const int64_t r = p->r, kr = p->kr, s = p->s, rank_k = p->rank_k;
    if (r < 1 || r > std::min(m, kMaxSketch))
        return fail(ctx, BCUR_E_ARG, "need 1 <= r <= min(m, %lld)", (long long)kMaxSketch);
    if (kr < 1 || kr > std::min(r, n)) return fail(ctx, BCUR_E_ARG, "need 1 <= kr <= min(r, n)");
    if (s < 1 || (!p->replace && s > G)) return fail(ctx, BCUR_E_ARG, "need 1 <= s <= G without replacement");
    if (rank_k < 0) return fail(ctx, BCUR_E_ARG, "rank_k < 0");
    if (p->replace < 0 || p->replace > 1 || p->pinv_eig < 0 || p->pinv_eig > 1)
        return fail(ctx, BCUR_E_ARG, "replace and pinv_eig must be 0 or 1");
    STCHK(check_map(ctx, p->col_map, n, "col_map"));
    int64_t maxw = 0;
    for (int64_t g = 0; g < G; ++g) maxw = std::max(maxw, col_off[g + 1] - col_off[g]);
    const int64_t cmax = std::min(s * maxw, n);
    if (res->U && (res->ldu < r || (res->ldu & 3) || !aligned16(res->U) || res->u_rows_cap < cmax))
        return fail(ctx, BCUR_E_ARG, "U needs ldu >= %lld (a multiple of 4, 16-byte aligned) and %lld rows",
                    (long long)r, (long long)cmax);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t rp = round4(r), np = round4(n), tmax = std::min(r, cmax);

    // workspace: columns' sampler | first-sync results | R, R^T, its eigensystem | C, W, W^+ | residual
    SampleBufs sc;
    double *d_frob, *d_fpart, *lamR, *gpart, *TR, *WkR, *WksR, *dscale, *Wx, *gpartW, *Gw, *Rw, *lamW, *Vw, *Mw, *P64,
        *wsE, *errv;
    int64_t* d_rows;
    uint64_t* d_rdr;
    int *infoR, *infoW;
    float *R0, *RT, *Vk, *Cbuf, *Ubuf, *P32, *Vp = nullptr;
    int64_t* d_cmap = nullptr;
    const bool chol_scores = kr == r;
    const int gwW = gram_wgs(std::max(r, cmax));
    void *jwsR, *jwsW;
    const int gw = gram_wgs(n);
    const int64_t nwsE = resid_parts(m, n, r);
    auto layout = [&](Arena& a) {
        d_rdr = a.take<uint64_t>(r);
        sample_layout(a, sc, G, s, cmax);
        // read back in one copy, from sc.idx to the end of infoR
        d_frob = a.take<double>(2);
        lamR = a.take<double>(r);
        d_rows = a.take<int64_t>(r);
        infoR = a.take<int>(4);
        d_fpart = a.take<double>(frob2_grid(m, n));
        R0 = a.take<float>(r * np);
        RT = a.take<float>(n * rp);
        gpart = a.take<double>((size_t)gw * r * r);
        TR = a.take<double>(r * r);
        WkR = a.take<double>(r * kr);
        WksR = a.take<double>(r * kr);
        jwsR = a.take<double>((jacobi_ws_bytes(r) + 7) / 8);
        Vk = a.take<float>(n * kr);
        if (p->col_map) {
            d_cmap = a.take<int64_t>(n);
            Vp = a.take<float>(n * kr);
        }
        Cbuf = a.take<float>(m * round4(cmax));
        dscale = a.take<double>(cmax);
        Wx = a.take<double>(cmax * r);
        gpartW = a.take<double>((size_t)gwW * tmax * tmax);
        Gw = a.take<double>(tmax * tmax);
        Rw = a.take<double>(tmax * tmax);
        Vw = a.take<double>(tmax * tmax);
        Mw = a.take<double>(tmax * tmax);
        jwsW = a.take<double>((jacobi_ws_bytes(tmax) + 7) / 8);
        Ubuf = ntail > 0 ? a.take<float>((size_t)ntail * cmax * rp) : nullptr;
        P64 = a.take<double>(m * r);
        P32 = a.take<float>(m * rp);
        wsE = a.take<double>(nwsE);
        // read back in one copy at the end
        errv = a.take<double>(8);
        lamW = a.take<double>(tmax);
        infoW = a.take<int>(8);
    };
    {
        Arena a;
        layout(a);
        STCHK(reserve(ctx, a.off));
        Arena b{ctx->ws, 0};
        layout(b);
    }
    const char* span1_0 = reinterpret_cast<const char*>(sc.idx);
    const size_t span1 = (size_t)(reinterpret_cast<const char*>(infoR + 4) - span1_0);
    const char* span2_0 = reinterpret_cast<const char*>(errv);
    const size_t span2 = (size_t)(reinterpret_cast<const char*>(infoW + 8) - span2_0);
    // pinned staging: offsets | draws | columns and their scales | the two read-back spans
    const size_t pin_need = 8 * (G + 1) + 8 * (r + s) + 16 * cmax + span1 + span2 + 64 + (p->col_map ? 8 * n : 0);
    STCHK(reserve_pinned(ctx, pin_need));
    if (ctx->pinned_busy) HIPCHK(hipStreamSynchronize(st));
    ctx->pinned_busy = true;
    char* pin = ctx->pinned;
    auto ptake = [&pin](size_t bytes) {
        char* p0 = pin;
        pin += (bytes + 7) & ~(size_t)7;
        return p0;
    };
    int64_t* h_off = reinterpret_cast<int64_t*>(ptake(8 * (G + 1)));
    uint64_t* h_dr = reinterpret_cast<uint64_t*>(ptake(8 * (r + s)));
    int64_t* h_cols = reinterpret_cast<int64_t*>(ptake(8 * cmax));
    double* h_scale = reinterpret_cast<double*>(ptake(8 * cmax));
    char* h1 = ptake(span1);
    char* h2 = ptake(span2);
    auto mirror1 = [&](const void* dp) { return h1 + (reinterpret_cast<const char*>(dp) - span1_0); };
    auto mirror2 = [&](const void* dp) { return h2 + (reinterpret_cast<const char*>(dp) - span2_0); };
    memcpy(h_off, col_off, (G + 1) * sizeof(int64_t));
    memcpy(h_dr, draws, (r + s) * sizeof(uint64_t));
    HIPCHK(hipMemcpyAsync(sc.off, h_off, (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_rdr, h_dr, r * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sc.dr, h_dr + r, s * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(sc.st, 0, 4 * sizeof(int), st));
    HIPCHK(hipMemsetAsync(infoR, 0, 4 * sizeof(int), st));
    HIPCHK(hipMemsetAsync(infoW, 0, 8 * sizeof(int), st));
    if (p->col_map) {
        int64_t* h_cm = reinterpret_cast<int64_t*>(ptake(8 * n));
        memcpy(h_cm, p->col_map, n * sizeof(int64_t));
        HIPCHK(hipMemcpyAsync(d_cmap, h_cm, n * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }

    // ||A||_F^2
    {
        StageScope ts(ctx, BCUR_STAGE_FROB);
        HIPCHK(launch_frob2(A, m, n, lda, d_fpart, frob2_grid(m, n), d_frob, st));
    }
    // step 1: r uniform rows, R = A[rows, :] (the scaling sqrt(m/r) is applied in W and U)
    {
        StageScope ts(ctx, BCUR_STAGE_A1_ROWS);
        HIPCHK(launch_uniform_rows(m, d_rdr, r, d_rows, st));
        HIPCHK(launch_gather_rows(A, lda, n, d_rows, r, R0, np, st));
        HIPCHK(launch_gather_rows_t(A, lda, n, d_rows, r, RT, rp, st));
    }
    // step 2: top-kr right singular vectors of R (a uniform row scale changes
    // neither V nor the scores).  With kr = r they span the row space of R and
    // any orthonormal basis of it gives the same scores: V = R^T L^-T from the
    // FP64 factor R R^T = L L^T (orthonormal up to about u64 cond(R)^2, the
    // accuracy of the scores themselves).  Otherwise from the eigensystem
    // R R^T = U_R Lambda U_R^T: V_kr = R^T U_kr Lambda_kr^-1/2.
    {
        StageScope ts(ctx, BCUR_STAGE_A1_SVDR);
        if (chol_scores) {
            HIPCHK(launch_gram64(RT, n, r, rp, gpart, gw, st));
            HIPCHK(launch_gram_reduce(gpart, gw, r, TR, st));
            HIPCHK(launch_chol_rinv_small(TR, r, WkR, infoR + 2, st));
            HIPCHK(launch_apply_small(RT, n, r, rp, WkR, r, r, Vk, kr, st));
        } else {
            HIPCHK(launch_gram64(RT, n, r, rp, gpart, gw, st));
            HIPCHK(launch_gram_reduce(gpart, gw, r, TR, st));
            HIPCHK(launch_jacobi_eigh(TR, r, kr, lamR, WkR, WksR, jwsR, infoR, st));
            HIPCHK(launch_apply_small(RT, n, r, rp, WksR, kr, kr, Vk, kr, st));
        }
    }
    {
        StageScope ts(ctx, BCUR_STAGE_SCORES);
        if (d_cmap) HIPCHK(launch_gather_rows(Vk, kr, kr, d_cmap, n, Vp, kr, st));
        HIPCHK(launch_block_scores(d_cmap ? Vp : Vk, kr, kr, sc.off, G, sc.sc, st));
    }
    {
        StageScope ts(ctx, BCUR_STAGE_SAMPLE);
        HIPCHK(launch_sample(sc.sc, G, sc.dr, s, p->replace, sc.qb, sc.pr, sc.idx, sc.w, sc.mg, sc.st, st));
    }
    HIPCHK(hipMemcpyAsync(h1, span1_0, span1, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t* hidx = reinterpret_cast<const int64_t*>(mirror1(sc.idx));
    const double* hw = reinterpret_cast<const double*>(mirror1(sc.w));
    const double* hmg = reinterpret_cast<const double*>(mirror1(sc.mg));
    const int* hst = reinterpret_cast<const int*>(mirror1(sc.st));
    const double* hsc = reinterpret_cast<const double*>(mirror1(sc.sc));
    const double* hfrob = reinterpret_cast<const double*>(mirror1(d_frob));
    const double* hlamR = reinterpret_cast<const double*>(mirror1(lamR));
    const int64_t* hrows = reinterpret_cast<const int64_t*>(mirror1(d_rows));
    if (!isfinite(hfrob[0])) return fail(ctx, BCUR_E_NONFINITE, "A holds NaN or Inf");
    if (hst[0] != 0) return fail(ctx, BCUR_E_HIP, "block scores are not finite");
    for (int64_t t = 0; t < s; ++t)
        if (hidx[t] < 0 || hidx[t] >= G) return fail(ctx, BCUR_E_HIP, "sampler returned an invalid block");
    // columns of C and the scale of each (the first draw's weight of its block;
    // scale 1 for a block drawn at zero weight)
    int64_t c = 0;
    for (int64_t t = 0; t < s; ++t) {
        const int64_t j = hidx[t];
        bool dup = false;
        for (int64_t u = 0; u < t; ++u) dup |= hidx[u] == j;
        if (dup) continue;
        const double wj = isfinite(hw[t]) ? hw[t] : 1.0;
        for (int64_t col = col_off[j]; col < col_off[j + 1]; ++col) {
            h_cols[c] = p->col_map ? p->col_map[col] : col;
            h_scale[c] = wj;
            ++c;
        }
    }
    HIPCHK(hipMemcpyAsync(sc.list, h_cols, c * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dscale, h_scale, c * sizeof(double), hipMemcpyHostToDevice, st));
    const int64_t ldc = round4(c), t_w = std::min(r, c);
    const double alpha = sqrt((double)m / (double)r);
    // C = A S unscaled
    {
        StageScope ts(ctx, BCUR_STAGE_GATHER);
        HIPCHK(launch_gather_cols(A, lda, m, sc.list, c, Cbuf, ldc, st));
    }
    // step 3: W = alpha R S, U = W^+ through the pseudoinverse M of the smaller
    // Gram matrix G = X^T X, where X = W (r x c) when c <= r and X = W^T (c x r)
    // otherwise: W^+ = M W^T = (X M)^T, or W^+ = W^T M = X M.  The core for the
    // unscaled factors is alpha D W^+.  M = G^-1 from a Cholesky factor when its
    // inverse certifies that no singular value of W is near the cutoff and no
    // truncation is asked for; otherwise (decided on the device) M from the
    // eigensystem of G with the cutoff and the rank-k truncation.
    // infoW: [0..1] eigensolver, [2] Cholesky, [3] 1 = eigensystem used, [4..5] kept counts
    if (tail) *tail = Ubuf;
    float* U = tail_slot >= 0 ? Ubuf + (size_t)tail_slot * cmax * rp : res->U;
    const int64_t ldu = tail_slot >= 0 ? rp : res->ldu;
    {
        StageScope ts(ctx, BCUR_STAGE_A1_PINV);
        const bool wide = c > r;   // X = W^T
        const int64_t K = wide ? c : r;
        HIPCHK(launch_alg1_w(RT, rp, r, sc.list, dscale, c, alpha, wide ? 1 : 0, Wx, st));
        const int gk = gram_wgs(K);
        HIPCHK(launch_gram64(Wx, K, t_w, t_w, gpartW, gk, st));
        HIPCHK(launch_gram_reduce(gpartW, gk, t_w, Gw, st));
        const double cut = ldexp((double)std::max(r, c), -24);
        const int force_eig = p->pinv_eig || (rank_k > 0 && rank_k < t_w);
        HIPCHK(launch_chol_rinv_small(Gw, t_w, Rw, infoW + 2, st));
        HIPCHK(launch_pinv_certify(Gw, Rw, t_w, infoW + 2, cut * cut, force_eig, infoW + 3, infoW + 4, st));
        HIPCHK(launch_gram_inv_rinv(Rw, t_w, Mw, infoW + 3, st));
        HIPCHK(launch_jacobi_eigh(Gw, t_w, t_w, lamW, Vw, nullptr, jwsW, infoW, st, infoW + 3));
        HIPCHK(launch_pinv_eig(lamW, Vw, t_w, cut * cut, rank_k, Mw, infoW + 4, infoW + 3, st));
        HIPCHK(launch_pinv_apply(Wx, K, t_w, Mw, dscale, alpha, wide ? 0 : 1, U, ldu, st));
    }
    // err = ||A - (C U) R||_F for the FP32 U: C U with FP64 accumulation, rounded
    // to FP32, then the residual GEMM with its fused squared norm
    {
        StageScope ts(ctx, BCUR_STAGE_A1_CU);
        HIPCHK(launch_dgemm_ff(m, r, c, 1.0, Cbuf, ldc, false, U, ldu, false, 0.0, P64, r, st));
        HIPCHK(launch_f64_to_f32_2d(P64, m, r, r, P32, rp, true, st));
    }
    const GemmPlan pe = plan_sgemm(m, n, r, false, false);
    STCHK(gemm_timed(ctx, BCUR_STAGE_FIT_E, BCUR_STAGE_FIT_REDUCE, pe, m, n, r, false, P32, rp, R0, np, nullptr, 0,
                     nullptr, EPI_RESID_NORM, A, lda, nullptr, 0, wsE));
    HIPCHK(launch_fit_err(wsE, nwsE, wsE, 0, errv, st));
    HIPCHK(hipMemcpyAsync(h2, span2_0, span2, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->pinned_busy = false;
    const double* herr = reinterpret_cast<const double*>(mirror2(errv));
    const int* hinfoW = reinterpret_cast<const int*>(mirror2(infoW));
    uint32_t fl = 0;
    if (hst[1]) fl |= BCUR_FLAG_ZERO_SCORE;
    if (hinfoW[4] < t_w) fl |= BCUR_FLAG_RANKDEF_W;
    if (hinfoW[3]) fl |= BCUR_FLAG_PINV_EIG;
    const int* hinfoR = reinterpret_cast<const int*>(mirror1(infoR));
    if (chol_scores) {
        if (hinfoR[2] & 1) fl |= BCUR_FLAG_RANKDEF_R;
    } else {
        const double cutR = ldexp((double)std::max(r, n), -24);
        if (!(hlamR[kr - 1] > cutR * cutR * hlamR[0])) fl |= BCUR_FLAG_RANKDEF_R;
    }
    memcpy(res->rows, hrows, r * sizeof(int64_t));
    memcpy(res->idx, hidx, s * sizeof(int64_t));
    if (res->weights) memcpy(res->weights, hw, s * sizeof(double));
    if (res->scores) memcpy(res->scores, hsc, G * sizeof(double));
    double mm = INFINITY;
    for (int64_t t = 0; t < s; ++t) mm = std::min(mm, hmg[t]);
    res->c = c;
    res->rank_w = hinfoW[5];
    res->frob2 = hfrob[0];
    res->err = sqrt(std::max(herr[0], 0.0));
    res->rel_err = hfrob[0] > 0.0 ? res->err / sqrt(hfrob[0]) : 0.0;
    res->min_margin = mm;
    res->flags = fl;
    res->sweeps = (uint32_t)hinfoW[0];
    return BCUR_OK;
}


bcur_status bcur_decompose_alg1(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                const int64_t* col_off, int64_t G, const bcur_alg1_params* p, const uint64_t* draws,
                                bcur_alg1_result* res) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    if (!res) return fail(ctx, BCUR_E_ARG, "null argument");
    return alg1_impl(ctx, A, m, n, lda, col_off, G, p, draws, res, res->U ? 0 : 1, res->U ? -1 : 0, nullptr);
}

bcur_status bcur_decompose_alg1_boost(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                      const int64_t* col_off, int64_t G, const bcur_alg1_params* p, int64_t t,
                                      const uint64_t* draws, bcur_alg1_result* res, double* errs,
                                      int64_t* best_out) {
    GUARD(ctx);
    if (!ctx) return BCUR_E_ARG;
    if (!p || !res || !draws || !res->rows || !res->idx || !errs) return fail(ctx, BCUR_E_ARG, "null argument");
    if (t < 1 || t > kMaxTrials) return fail(ctx, BCUR_E_ARG, "need 1 <= t <= %lld", (long long)kMaxTrials);
    STCHK(check_offsets(ctx, col_off, G, n, "col_off"));
    const int64_t r = p->r, s = p->s;
    if (r < 1 || s < 1) return fail(ctx, BCUR_E_ARG, "need r >= 1 and s >= 1");
    int64_t maxw = 0;
    for (int64_t g = 0; g < G; ++g) maxw = std::max(maxw, col_off[g + 1] - col_off[g]);
    const int64_t cmax = std::min(s * maxw, n), rp = round4(r);
    if (res->U && (res->ldu < r || (res->ldu & 3) || !aligned16(res->U) || res->u_rows_cap < cmax))
        return fail(ctx, BCUR_E_ARG, "U needs ldu >= %lld (a multiple of 4, 16-byte aligned) and %lld rows",
                    (long long)r, (long long)cmax);
    // every trial keeps its host results; the cores alternate between two
    // workspace buffers so the best one so far is never overwritten
    std::vector<int64_t> rows((size_t)t * r), idx((size_t)t * s);
    std::vector<double> w((size_t)t * s), sc((size_t)t * G);
    std::vector<bcur_alg1_result> runs(t);
    int64_t best = -1;
    int best_slot = 1;
    float* tail = nullptr;
    for (int64_t i = 0; i < t; ++i) {
        bcur_alg1_result& ri = runs[i];
        ri = bcur_alg1_result{};
        ri.rows = rows.data() + i * r;
        ri.idx = idx.data() + i * s;
        ri.weights = w.data() + i * s;
        ri.scores = sc.data() + i * G;
        const int slot = best_slot ^ 1;
        STCHK(alg1_impl(ctx, A, m, n, lda, col_off, G, p, draws + i * (r + s), &ri, 2, slot, &tail));
        errs[i] = ri.err;
        if (best < 0 || ri.err < runs[best].err) {
            best = i;
            best_slot = slot;
        }
    }
    const bcur_alg1_result& rb = runs[best];
    if (res->U)
        HIPCHK(hipMemcpy2DAsync(res->U, res->ldu * sizeof(float), tail + (size_t)best_slot * cmax * rp,
                                rp * sizeof(float), r * sizeof(float), rb.c, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    memcpy(res->rows, rb.rows, r * sizeof(int64_t));
    memcpy(res->idx, rb.idx, s * sizeof(int64_t));
    if (res->weights) memcpy(res->weights, rb.weights, s * sizeof(double));
    if (res->scores) memcpy(res->scores, rb.scores, G * sizeof(double));
    res->c = rb.c;
    res->rank_w = rb.rank_w;
    res->frob2 = rb.frob2;
    res->err = rb.err;
    res->rel_err = rb.rel_err;
    res->min_margin = rb.min_margin;
    res->flags = rb.flags;
    res->sweeps = rb.sweeps;
    if (best_out) *best_out = best;
    return BCUR_OK;
}

}  // extern "C"
