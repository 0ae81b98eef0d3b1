/*
 * bcur.h - C ABI of the Block CUR hot path on AMD Instinct MI355X (gfx950).
 *
 * Block CUR (Oswal, Jain, Xu, Eriksson, "Block CUR: Decomposing Matrices
 * using Groups of Columns", arXiv 1703.06065) approximates A (m x n) from a
 * few predefined blocks of its columns (and, optionally, rows) chosen by block
 * leverage scores.  The library computes, on one GPU:
 *
 *   1. ||A||_F^2 and a finiteness check                       (Sec. 2.1)
 *   2. a top-k right singular subspace V_k of A with a randomized range
 *      finder (the sketching replacement for the score step, Sec. 3.1)
 *   3. block leverage scores l_g = ||V_k^T E_g||_F^2            (Def. 2)
 *   4. s blocks sampled with probability proportional to l_g  (Alg. 1, step 2)
 *   5. C = A S, the chosen column blocks                      (Sec. 3.1)
 *   6. U = C^+ A and the residual ||A - C C^+ A||_F           (Remark, Sec. 3.3)
 *      or, for the row-block variant, U = C^+ A R^+ and ||A - C U R||_F.
 *
 * Conventions for every call:
 *   - Matrices are row-major float32 with a leading dimension (elements
 *     between consecutive rows) >= the number of columns.  Device matrices
 *     handed to the library must be 16-byte aligned with a leading dimension
 *     that is a multiple of 4.
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary host memory.  The library never takes
 *     ownership of caller memory and never frees it.
 *   - Work is issued on the context's stream.  Calls that return host values
 *     synchronize that stream before returning; the others are stream-ordered
 *     and return at once.
 *   - Every call returns a bcur_status.  On an error nothing is written to
 *     host outputs; device outputs may be partly written.  The message of the
 *     last error of a context is available from bcur_last_error.
 *   - A context is not thread safe: use one context per host thread.
 */
#ifndef BCUR_H
#define BCUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bcur_status {
    BCUR_OK = 0,
    BCUR_E_ARG = 1,        /* invalid argument: shape, offsets, k, s, null pointer, alignment */
    BCUR_E_NONFINITE = 2,  /* A holds a NaN or an Inf */
    BCUR_E_NOMEM = 3,      /* a device or host allocation failed */
    BCUR_E_HIP = 4,        /* a HIP runtime call or kernel launch failed */
    BCUR_E_RANKDEF = 5,    /* a Cholesky factorization met a pivot below its threshold */
    BCUR_E_ADMIT = 6,      /* serving: the request can never fit the memory budget */
    BCUR_PENDING = 7,      /* serving: the request has not finished yet */
    BCUR_E_STATE = 8       /* serving: unknown or already collected ticket; context: a call was made
                              while an asynchronous decomposition is in flight (see bcur_wait) */
} bcur_status;

/* Arithmetic used by the range finder's passes over A.
 *
 * FP32 products (every product of BCUR_PREC_FP32, the fit, and the last
 * power pass of BCUR_PREC_BF16) accumulate in FP32.  Small products run on
 * the FP32 matrix cores.  Products with M, K >= 256 and either N >= 256 and
 * at least 8e9 multiply-adds, or a sketch width 32 < N <= 128 and at least
 * 1e9, split each FP32 operand
 * exactly into three BF16 terms, a = a0 + a1 + a2, and form a b from the
 * six largest of the nine term products on the BF16 matrix cores.  The
 * three dropped terms are below 2^-23 |a b|, two FP32 unit roundoffs, which
 * is less than the FP32 accumulation's own rounding; the results meet the
 * same tolerances as FP32 MFMA products.  The split needs |a| < 3.38e38 (a
 * larger finite value rounds to infinity in BF16); non-finite operands give
 * NaN. */
enum {
    BCUR_PREC_FP32 = 0,    /* FP32 products as above */
    BCUR_PREC_BF16 = 1     /* first q power iterations: A and the basis rounded to BF16, BF16 MFMA with
                              FP32 accumulation; then one FP32 power pass */
};

/* Bits of bcur_result.flags. */
enum {
    BCUR_FLAG_RANKDEF_C = 1u << 0,   /* C^T C was numerically singular: pivots dropped */
    BCUR_FLAG_ILLCOND_C = 1u << 1,   /* estimated cond(C)^2 * 2^-24 > 0.1: U is inaccurate */
    BCUR_FLAG_ZERO_SCORE = 1u << 2,  /* a block of zero score was drawn (all remaining scores were 0) */
    BCUR_FLAG_RANKDEF_Y = 1u << 3,   /* a Gram matrix of the range finder needed a diagonal shift */
    BCUR_FLAG_RANKDEF_R = 1u << 4,   /* R R^T was numerically singular (row-block variant; Algorithm 1:
                                        fewer than kr singular values of R above the cutoff) */
    BCUR_FLAG_RANKDEF_W = 1u << 5,   /* Algorithm 1: singular values of W at or below the cutoff were dropped */
    BCUR_FLAG_PINV_EIG = 1u << 6     /* Algorithm 1 (informational): W^+ came from the eigensystem of W's Gram
                                        matrix, not from its certified Cholesky factor */
};

typedef struct bcur_ctx bcur_ctx;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` that issues all work on `stream`
 * (a hipStream_t owned by the caller; NULL means the device's null stream).
 * The context owns a grow-only device workspace and a pinned host staging
 * buffer.  scratch_budget: the most device workspace, in bytes, the context
 * may hold (0: no limit); a call whose workspace would exceed it fails with
 * BCUR_E_NOMEM before allocating anything (bcur_footprint gives a
 * decomposition's need from its shapes). */
bcur_status bcur_create(bcur_ctx** out, int device, void* stream, size_t scratch_budget);

/* Destroy a context, freeing only what the library allocated. */
bcur_status bcur_destroy(bcur_ctx* ctx);

/* Wait for all work issued by the context. */
bcur_status bcur_synchronize(bcur_ctx* ctx);

/* Static text for a status code, and the message of the context's last error
 * ("" if none).  The returned strings stay valid until the next call. */
const char* bcur_status_str(int status);
const char* bcur_last_error(const bcur_ctx* ctx);

/* Bytes of device workspace currently held by the context. */
size_t bcur_workspace_bytes(const bcur_ctx* ctx);

/* Give the context's device workspace back (it is reallocated on demand). */
bcur_status bcur_release_workspace(bcur_ctx* ctx);

/* ---- stage calls -------------------------------------------------------- */

/* The Rademacher test matrix of the range finder (its random input; Sec. 3.1
 * allows the score step to be sketched) drawn on the device from a seed:
 * omega[i][j] = +1 or -1 from bit j of the Philox4x64-10 block (Salmon et
 * al., SC 2011) with counter (i, 0, 0, 0) and key (seed, 0); bit j is bit
 * j % 64 of output word j / 64, and a 0 bit gives +1.  The matrix of a
 * narrower sketch is the leading columns of a wider one.
 * omega: device n x l float32 (leading dimension ldo >= l); columns l ..
 * ldo-1 are not written.  Requires 1 <= l <= 256.  Stream-ordered. */
bcur_status bcur_test_matrix(bcur_ctx* ctx, int64_t n, int64_t l, uint64_t seed, float* omega, int64_t ldo);

/* ||A||_F^2 = sum_ij A_ij^2 (Sec. 2.1, Frobenius norm), accumulated in float64
 * in a fixed order (bitwise reproducible on one device).
 * A: device, m x n, leading dimension lda.  out_frob2: host, one double.
 * out_finite: host, set to 1 when every entry is finite, else 0.
 * Synchronous. */
bcur_status bcur_frob2(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                       double* out_frob2, int32_t* out_finite);

/* Randomized range finder: an orthonormal basis V_k (n x k) of the top-k
 * right singular subspace of A, the sketch that Sec. 3.1 allows in place of
 * an SVD.  Q starts as the test matrix omega (n x l, l = k + oversampling);
 * q+1 times Q <- orth(A^T (A Q)) (Cholesky QR with float64 Gram matrices);
 * then Rayleigh-Ritz: Z = A Q, T = Z^T Z, T = W diag(lam) W^T (float64
 * Jacobi), V_k = Q W[:, :k], Ritz values sqrt(lam).
 * A: device m x n (lda).  omega: device n x l float32, row-major, dense.
 * precision: BCUR_PREC_FP32, or BCUR_PREC_BF16 (iterations 0 .. q-1 as BF16
 * sketch passes, iteration q and the Rayleigh-Ritz pass in FP32).
 * Vk: device n x k float32 (leading dimension k), written.
 * Uk: device m x k (leading dimension k) or NULL; when given, receives
 *     Z W[:, :k] diag(1/sqrt(lam_k)), the matching left vectors.
 * ritz: host, l doubles, or NULL (Ritz singular values, descending).
 * Requires 1 <= k <= l <= min(m, n, 128).  Synchronous when ritz != NULL. */
bcur_status bcur_range_finder(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                              const float* omega, int64_t l, int64_t k, int64_t q, int32_t precision,
                              float* Vk, float* Uk, double* ritz);

/* One sketch pass of the range finder: Y = A^T (A Q), the power step that
 * multiplies a basis by A^T A.  BCUR_PREC_FP32: FP32 products (see BCUR_PREC_FP32).
 * BCUR_PREC_BF16: A and Q rounded to BF16 (nearest even), BF16 MFMA with
 * FP32 accumulation, A Q rounded to BF16 before the second product.
 * A: device m x n (lda).  Q: device n x l (ldq).  Y: device n x l (ldy,
 * multiple of 4), written.  Requires l <= 128.  Synchronous. */
bcur_status bcur_sketch_pass(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* Q,
                             int64_t l, int64_t ldq, int32_t precision, float* Y, int64_t ldy);

/* Block leverage scores l_g = ||V^T E_g||_F^2 (Def. 2): the sum of squares of
 * rows offsets[g] .. offsets[g+1]-1 of V, accumulated in float64.
 * V: device n x k (ldv).  offsets: host, G+1 int64, offsets[0] = 0,
 * strictly increasing, offsets[G] = n.  scores: host, G doubles.
 * Synchronous. */
bcur_status bcur_block_scores(bcur_ctx* ctx, const float* V, int64_t n, int64_t k, int64_t ldv,
                              const int64_t* offsets, int64_t G, double* scores);

/* Sample s blocks with probability proportional to their scores (Alg. 1,
 * step 2), on the device.  Scores are quantized exactly to integers
 * q_g = floor(l_g 2^sh) with one power-of-two scale sh = 62 - ceil(log2 G)
 * - E, where max_g l_g = f 2^E, f in [0.5, 1).  Draw t maps the 64-bit word
 * r_t to x = floor(r_t W / 2^64) on [0, W), W the total weight of the
 * remaining blocks (all blocks when replace != 0, the not yet chosen ones
 * otherwise), and picks the block whose interval, laid out in index order,
 * holds x.  When every remaining weight is zero the smallest remaining index
 * is taken.  weights_t = 1/sqrt(s p_j), p_j = q_j / sum(q) (the scaling of
 * S, Sec. 3.1), +inf for a zero-weight block.
 * scores: host, G finite non-negative doubles.  draws: host, s words.
 * idx: host, s int64.  weights: host, s doubles or NULL.  margins: host, s
 * doubles or NULL (distance of x to the nearer edge of its interval, in score
 * units).  Needs s <= G when replace == 0.  Synchronous. */
bcur_status bcur_sample_blocks(bcur_ctx* ctx, const double* scores, int64_t G, const uint64_t* draws,
                               int64_t s, int32_t replace, int64_t* idx, double* weights, double* margins);

/* C = A S without scaling (Sec. 3.1): the column blocks idx[0..s-1] of A side
 * by side in selection order; a block listed twice is copied once.
 * A: device m x n (lda).  offsets: host G+1.  idx: host s.
 * C: device m x c (ldc >= c), written.  c_out: host, receives c.
 * Stream-ordered (returns before the copy completes). */
bcur_status bcur_gather_columns(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                const int64_t* offsets, int64_t G, const int64_t* idx, int64_t s,
                                float* C, int64_t ldc, int64_t* c_out);

/* U = C^+ A (Sec. 2.1 pseudoinverse; the block column-subset-selection fit
 * of the Remark in Sec. 3.3) by the normal equations: H = C^T A and
 * C^T C on the MFMA units, a float64 Cholesky inverse of C^T C, then
 * `refine` (0 or 1) steps of iterative refinement whose right-hand side
 * C^T (A - C U) is formed as H - (C^T C) U.  err = ||A - C U||_F.  The accuracy of U is about
 * u32 cond(C)^2 relative.  When pivots of C^T C are dropped
 * (BCUR_FLAG_RANKDEF_C: C numerically rank-deficient) or their spread says
 * the FP32 normal equations are inaccurate (BCUR_FLAG_ILLCOND_C), the fit is
 * redone by Cholesky QR2 in FP64 (a basic least-squares solution on the
 * columns kept at 2^-50) and err is the exact residual of the returned U.
 * A: device m x n (lda).  C: device m x c (ldc).  U: device c x n (ldu);
 * only those c x n elements are written.  err: host double.  flags: host uint32 (BCUR_FLAG_*), or NULL.
 * Synchronous. */
bcur_status bcur_fit_columns(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                             const float* C, int64_t c, int64_t ldc, int32_t refine,
                             float* U, int64_t ldu, double* err, uint32_t* flags);

/* ---- diagnostics (Sec. 3.2) ------------------------------------------------ */

/* Block stable rank (Def. 3) of the slices of V (device n x k, ldv; the
 * top-k right singular vectors, e.g. from bcur_range_finder): ratios[g] =
 * ||V^T E_g||_F^2 / ||V^T E_g||_2^2 (host G, or NULL; NaN for a zero slice) and
 * *alpha = their minimum over the nonzero slices.  FP64 from the exact squares
 * of the FP32 entries; the spectral norm of each slice comes from the Gram
 * matrix of its smaller side by repeated squaring to the top eigenspace
 * (steps: host G, or NULL, receives the squaring steps each block took, at
 * most 64).  col_map (host n, or NULL): blocks of arbitrary row sets of V,
 * as in bcur_params.  BCUR_E_ARG when min(block width, k) > 64 for some block.
 * Synchronous. */
bcur_status bcur_block_stable_rank(bcur_ctx* ctx, const float* V, int64_t n, int64_t k, int64_t ldv,
                                   const int64_t* offsets, int64_t G, const int64_t* col_map, double* ratios,
                                   int32_t* steps, double* alpha);

/* Column-space incoherence (Def. 4) of U (device m x k, ldu; the top-k left
 * singular vectors): *mu = (m / k) max_i ||U^T e_i||_2^2, FP64.  Synchronous. */
bcur_status bcur_incoherence(bcur_ctx* ctx, const float* U, int64_t m, int64_t k, int64_t ldu, double* mu);

/* ---- profiling ---------------------------------------------------------- */

/* Device time per stage, measured with HIP events recorded on the context's
 * stream around each stage's kernels (the events bracket exactly the launches
 * named below, so their elapsed time is those kernels' duration). */
enum {
    BCUR_STAGE_FROB = 0,      /* ||A||_F^2 */
    BCUR_STAGE_RF_AQ = 1,     /* Z = A Q, main GEMM kernel (range finder) */
    BCUR_STAGE_RF_ATZ = 2,    /* Y = A^T Z, main GEMM kernel (range finder) */
    BCUR_STAGE_RF_REDUCE = 3, /* split-K sums of the range finder GEMMs */
    BCUR_STAGE_RF_ORTH = 4,   /* Cholesky QR: Gram, factor, apply */
    BCUR_STAGE_RF_RR = 5,     /* Rayleigh-Ritz: Gram, Jacobi, V_k */
    BCUR_STAGE_SCORES = 6,    /* block leverage scores */
    BCUR_STAGE_SAMPLE = 7,    /* block sampling */
    BCUR_STAGE_GATHER = 8,    /* C = A S */
    BCUR_STAGE_FIT_H = 9,     /* H = C^T A, main GEMM kernel */
    BCUR_STAGE_FIT_REDUCE = 10, /* split-K sums of the fit GEMMs */
    BCUR_STAGE_FIT_INV = 11,  /* G = C^T C, its FP64 Cholesky with X = L^-1, G^-1 = X^T X */
    BCUR_STAGE_FIT_U = 12,    /* U = G^-1 H, G^-1 = X^T X, X = L^-1, G = L L^T */
    BCUR_STAGE_FIT_E = 13,    /* ||A - C U||_F^2 (the residual is not stored) */
    BCUR_STAGE_FIT_F = 14,    /* F = C^T (A - C U), formed as H - (C^T C) U */
    BCUR_STAGE_FIT_DU = 15,   /* U += G^-1 F with <G^-1 F, F> */
    BCUR_STAGE_RF_CAST = 16,  /* BF16 copies of A and of the sketch panels */
    BCUR_STAGE_A1_ROWS = 17,  /* Algorithm 1: uniform row draws, R = A[rows, :] and its transpose */
    BCUR_STAGE_A1_SVDR = 18,  /* Algorithm 1: R R^T, its eigensolver, V_kr = R^T U_kr Sigma^-1 */
    BCUR_STAGE_A1_PINV = 19,  /* Algorithm 1: W, its Gram matrix, eigensolver, W^+, scaled U */
    BCUR_STAGE_A1_CU = 20,    /* Algorithm 1: P = C U (FP64 accumulation, rounded to FP32) */
    BCUR_STAGE_DIAG_ALPHA = 21, /* block stable rank */
    BCUR_STAGE_DIAG_MU = 22,  /* incoherence */
    BCUR_NUM_STAGES = 23
};

/* Stage timing: `on` = 0 turns it off; otherwise bit i of `on` times stage
 * i (-1 times every stage).  Each timed stage records two events per
 * launch on the context's stream, so time only the stages needed.
 * Changing the setting clears the totals. */
bcur_status bcur_timing_enable(bcur_ctx* ctx, int32_t on);

/* Totals since timing was enabled: ms[i] milliseconds and count[i] launches
 * of stage i, for i < BCUR_NUM_STAGES (host arrays).  Synchronizes. */
bcur_status bcur_timing_read(bcur_ctx* ctx, double* ms, int64_t* count);

/* ---- the whole path ----------------------------------------------------- */

typedef struct bcur_params {
    int64_t k;          /* target rank, 1 <= k */
    int64_t s;          /* number of column blocks to sample */
    int64_t l;          /* sketch width k + oversampling; l <= min(m, n, 128) */
    int64_t q;          /* power iterations (the range finder applies A^T A q+1 times) */
    int32_t replace;    /* 0: without replacement (default), 1: independent draws */
    int32_t precision;  /* BCUR_PREC_FP32 or BCUR_PREC_BF16 */
    int32_t refine;     /* refinement steps of the least-squares fit: 0 or 1 */
    int32_t reserved;
    int64_t s_r;        /* row blocks to sample for the row-block variant, 0 = columns only */
    /* Blocks of arbitrary column (row) sets: host, n (m) entries forming a
     * permutation, or NULL.  Column block g is then the set of columns
     * col_map[col_off[g] .. col_off[g+1]-1] (row block h: row_map[row_off[h]
     * .. row_off[h+1]-1]); the E_g of Def. 2 may pick any columns.  NULL means
     * the identity (contiguous blocks).  C and R hold the chosen columns and
     * rows in selection order, each block's in map order. */
    const int64_t* col_map;
    const int64_t* row_map;
    /* Seed of the test matrix (bcur_test_matrix) when the call's omega is
     * NULL; ignored otherwise. */
    uint64_t seed;
} bcur_params;

typedef struct bcur_result {
    /* caller-provided buffers (capacities in parentheses) */
    int64_t* idx;        /* host (s): chosen column blocks, selection order */
    double* weights;     /* host (s) or NULL: 1/sqrt(s p) of each draw */
    double* scores;      /* host (G) or NULL: block leverage scores */
    double* ritz;        /* host (l) or NULL: Ritz singular values */
    float* U;            /* device or NULL: U, c x n (columns only) or c x r (row variant) */
    int64_t ldu;         /* leading dimension of U */
    int64_t u_rows_cap;  /* rows U can hold (>= c) */
    int64_t* idx_r;      /* host (s_r) or NULL: chosen row blocks (row variant) */
    double* row_scores;  /* host (Gr) or NULL */
    /* outputs */
    int64_t c;           /* columns of C */
    int64_t r;           /* rows of R (row variant), else 0 */
    double frob2;        /* ||A||_F^2 */
    double err;          /* ||A - C U||_F, or ||A - C U R||_F for the row variant */
    double rel_err;      /* err / ||A||_F */
    double min_margin;   /* smallest sampling margin over the column draws */
    uint32_t flags;      /* BCUR_FLAG_* */
    uint32_t rr_sweeps;  /* Jacobi sweeps of the Rayleigh-Ritz eigensolver */
    /* precision report */
    double kappa;        /* lam_1 / (lam_k - lam_{k+1}) of the Ritz values (lam = Ritz value^2; 1 when k = l,
                            inf without a gap): how strongly rounding of the passes over A can move the top-k
                            subspace and so the scores (their error is below about 4 sqrt(max(m, n)) u32 kappa
                            max(l_g, k / G) in FP32, with u_bf16 in place of u32 on the BF16 passes) */
    double cond_c;       /* columns only: sqrt(largest / smallest pivot) of the Cholesky factor of C^T C, a
                            lower bound on cond(C) (U carries a relative error of about sqrt(m) u32 cond(C)^2
                            err / ||A||_F); 0 for the row-block variant */
} bcur_result;

/* One Block CUR decomposition: stages 1-6 above.
 * A: device m x n (lda).  col_off: host G+1 column-block offsets.
 * row_off: host Gr+1 row-block offsets, or NULL (columns only).
 * omega: device n x l test matrix (dense, leading dimension l), or NULL: the
 * Rademacher matrix of params->seed is drawn on the device (bcur_test_matrix).
 * draws: host, s + s_r 64-bit words (column draws first).
 * Columns only: U on C's own columns is the identity (C e_k is that column of
 * A exactly, so the residual there is zero; it is the least-squares solution
 * there when C has full column rank, the case the FP32 fit keeps, and the
 * FP64 fallback recomputes U whole otherwise).  Where the residual product is
 * large enough for the split-BF16 tile (m, c, n - c >= 256 and
 * m c (n - c) >= 8e9, n <= 262144) and its 256 x 256 tiles over n - c columns
 * take fewer rounds of 256 workgroups than over n, the residual pass covers
 * only the other n - c columns.  Synchronous. */
bcur_status bcur_decompose(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                           const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                           const bcur_params* params, const float* omega, const uint64_t* draws,
                           bcur_result* result);

/* bcur_decompose without waiting for it: the call checks its pointers, copies
 * the host inputs (offsets, draws, maps, parameters) and returns; the
 * decomposition then runs on the context's own host thread, its device work
 * issued after everything queued on the context's stream before this call
 * (the call records an event there that the work waits for) and on an
 * internal stream of the default priority.  A, omega and result (with the
 * buffers it points to) are borrowed until bcur_wait returns: every output,
 * host and device, is valid only then.  Until then any other call on the
 * context returns BCUR_E_STATE.  Argument errors found after the return are
 * reported by bcur_wait. */
bcur_status bcur_decompose_async(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                 const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                                 const bcur_params* params, const float* omega, const uint64_t* draws,
                                 bcur_result* result);

/* Wait for the context's asynchronous decomposition and return its status
 * (BCUR_OK at once when none is in flight). */
bcur_status bcur_wait(bcur_ctx* ctx);

/* bcur_decompose for callers that cannot allocate during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * it calls no hipMalloc, hipFree, hipHostMalloc or host allocator.  Its
 * device workspace is a static array of the library, 128 MiB on each GPU the
 * library runs on (held from the first bcur_create on that GPU until the
 * process ends); its host staging is a static 1 MiB buffer per GPU.  A call
 * whose workspace (bcur_footprint with library_holds_u = 0) exceeds 128 MiB,
 * or whose staging exceeds 1 MiB, fails with BCUR_E_NOMEM before any work.
 * result->U must be a caller buffer; block maps (params->col_map, row_map)
 * are refused with BCUR_E_ARG; stage timing is not recorded.  Every call on a
 * GPU shares that GPU's arrays and leaves its contents behind (each call
 * clears what it needs): calls that overlap on one GPU, from any contexts,
 * race.  Results are bitwise those of bcur_decompose.  Synchronous. */
bcur_status bcur_decompose_noalloc(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                   const int64_t* col_off, int64_t G, const int64_t* row_off, int64_t Gr,
                                   const bcur_params* params, const float* omega, const uint64_t* draws,
                                   bcur_result* result);

/* Device workspace one bcur_decompose call needs for these shapes and
 * parameters (bytes; library_holds_u != 0 when result->U will be NULL).
 * Host only, no device access. */
bcur_status bcur_footprint(int64_t m, int64_t n, const int64_t* col_off, int64_t G, const int64_t* row_off,
                           int64_t Gr, const bcur_params* params, int32_t library_holds_u, size_t* bytes);

/* ---- boosting -------------------------------------------------------------
 *
 * Sec. 3.3 turns the constant-probability guarantee of one run into
 * probability 1 - delta by running t = ln(1/delta) independent samplings and
 * keeping the one of smallest error.  Here: one range finder and one set of
 * block scores (stages 1-3 of bcur_decompose) shared by t trials; trial i
 * draws s blocks with draws[i*s .. i*s+s-1], gathers C_i and fits U_i = C_i^+ A
 * with its residual exactly as bcur_decompose does (columns only, params->s_r
 * = 0); the H_i = C_i^T A products of all trials run as one GEMM over their
 * concatenated columns.  omega may be NULL (the test matrix of params->seed).  result describes the kept trial (smallest err, the
 * first on ties) and receives its U; errs (host, t) receives every trial's
 * err; *best (may be NULL) its index.  1 <= t <= 64.  Synchronous. */
bcur_status bcur_decompose_boost(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                 const int64_t* col_off, int64_t G, const bcur_params* params,
                                 const float* omega, int64_t t, const uint64_t* draws, bcur_result* result,
                                 double* errs, int64_t* best);

/* ---- Algorithm 1: uniform rows, U = W^+ ------------------------------------
 *
 * The method as listed in Algorithm 1 of Sec. 3.1:
 *   1. r rows of A drawn uniformly without replacement, R = S_R^T A with the
 *      scaling sqrt(m / r) of the sampling matrix S_R;
 *   2. block scores l_g(R, kr) = ||V_{R,kr}^T E_g||_F^2 (Def. 2 applied to R)
 *      from the exact top-kr right singular vectors of R (for kr = r any
 *      orthonormal basis of the row space of R: Cholesky QR of R^T in FP64;
 *      for kr < r the eigensystem of R R^T in FP64); s column blocks drawn
 *      with p_g = l_g / sum(l), C = A S with S scaled by 1/sqrt(s p_g) per
 *      block;
 *   3. W = R S (r x c), U = W^+ (Sec. 2.1), or U_k = (W_k)^+, the pseudoinverse
 *      of the best rank-k approximation of W (the rank-k variant of Sec. 4.1),
 *      and err = ||A - C U R||_F.
 * Row draw t takes the x-th remaining row in ascending order with
 * x = floor(draws[t] (m - t) / 2^64).  Column draws follow bcur_sample_blocks.
 * W^+ treats singular values of W at or below max(r, c) 2^-24 sigma_1(W) as
 * zero (W holds FP32 data).  It is formed from the Cholesky factor of W's
 * smaller Gram matrix when the factor's inverse certifies that no singular
 * value is near that cutoff, else from the Gram matrix's eigensystem.  A block drawn with zero weight (possible only
 * when every remaining score is zero) enters S with scale 1.  Repeated
 * column blocks (with replacement) are kept once, with their first weight. */

typedef struct bcur_alg1_params {
    int64_t r;          /* rows drawn, 1 <= r <= min(m, 128) */
    int64_t kr;         /* right singular vectors of R behind the scores, 1 <= kr <= min(r, n) */
    int64_t s;          /* column blocks to draw */
    int64_t rank_k;     /* 0: U = W^+;  k >= 1: U_k = (W_k)^+ */
    int32_t replace;    /* column draws: 0 without replacement, 1 independent */
    int32_t pinv_eig;   /* 0: Cholesky route when certified (default); 1: always the eigensystem */
    const int64_t* col_map;  /* host (n) permutation or NULL: blocks of arbitrary column sets, as in
                                bcur_params */
} bcur_alg1_params;

typedef struct bcur_alg1_result {
    /* caller-provided buffers (capacities in parentheses) */
    int64_t* rows;       /* host (r): sampled rows of A, draw order */
    int64_t* idx;        /* host (s): chosen column blocks, selection order */
    double* weights;     /* host (s) or NULL: 1/sqrt(s p) of each column draw */
    double* scores;      /* host (G) or NULL: block scores l_g(R, kr) */
    float* U;            /* device or NULL: c x r (ldu >= r, a multiple of 4, 16-byte aligned), the
                            core for the UNSCALED factors: A ~ A[:, cols] U A[rows, :], i.e.
                            sqrt(m / r) D W^+ with D the per-column scales of S */
    int64_t ldu;
    int64_t u_rows_cap;  /* rows U can hold (>= c) */
    /* outputs */
    int64_t c;           /* columns of C */
    int64_t rank_w;      /* singular values of W kept in U */
    double frob2;        /* ||A||_F^2 */
    double err;          /* ||A - C U R||_F for the returned FP32 U */
    double rel_err;      /* err / ||A||_F */
    double min_margin;   /* smallest sampling margin over the column draws */
    uint32_t flags;      /* BCUR_FLAG_* */
    uint32_t sweeps;     /* Jacobi sweeps of the eigensolver of W's Gram matrix (0 on the Cholesky route) */
} bcur_alg1_result;

/* Algorithm 1 of Sec. 3.1 (with its rank-k variant of Sec. 4.1).
 * A: device m x n (lda).  col_off: host G+1 column-block offsets.
 * draws: host, r + s 64-bit words (row draws first).  Synchronous.
 * BCUR_E_ARG for r, kr, s or rank_k out of range; BCUR_E_NONFINITE when A
 * holds a NaN or an Inf. */
bcur_status bcur_decompose_alg1(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                const int64_t* col_off, int64_t G, const bcur_alg1_params* params,
                                const uint64_t* draws, bcur_alg1_result* result);

/* Boosting as Thm. 2 states it (Sec. 3.3): Algorithm 1 run t times with
 * independent draws, trial i taking words i(r+s) .. i(r+s)+r+s-1 of draws
 * (host, t(r+s) words: its r row draws, then its s column draws); result
 * describes the run of smallest err (the first on ties) and receives its
 * core; errs (host, t) every run's err; *best (may be NULL) its index.
 * 1 <= t <= 64.  Synchronous. */
bcur_status bcur_decompose_alg1_boost(bcur_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                                      const int64_t* col_off, int64_t G, const bcur_alg1_params* params,
                                      int64_t t, const uint64_t* draws, bcur_alg1_result* result, double* errs,
                                      int64_t* best);

/* ---- serving: continuous batching of decompositions ------------------------
 *
 * A server runs up to `max_slots` decompositions at once, each in its own
 * slot (a context with its own HIP stream and host thread), so requests that
 * arrive while others run are admitted as soon as a slot is free and their
 * device-memory footprint (bcur_footprint) fits `hbm_budget`; their work
 * overlaps on the device.  Admission is in arrival order.  Results are
 * bitwise identical to bcur_decompose on the same inputs (the kernels and
 * their tilings depend only on each request's shapes). */

typedef struct bcur_server bcur_server;

typedef struct bcur_request {
    const float* A;          /* device, borrowed until the ticket completes */
    int64_t m, n, lda;
    const int64_t* col_off;  /* host, copied at submission */
    int64_t G;
    const int64_t* row_off;  /* host or NULL, copied */
    int64_t Gr;
    bcur_params params;
    const float* omega;      /* device, borrowed; NULL: the test matrix of params.seed */
    const uint64_t* draws;   /* host, s + s_r words, copied */
    float* U;                /* device output or NULL, borrowed */
    int64_t ldu, u_rows_cap;
    void* stream;            /* hipStream_t that produced A / omega, or NULL: the
                                request waits for the work queued on it so far */
} bcur_request;

typedef struct bcur_stats {
    int64_t completed, failed, queued, running;
    double p50_ms, p99_ms, mean_ms;  /* latency from submission to completion */
    double throughput;               /* completed per second, first submission to last completion */
    uint64_t hbm_held, hbm_peak;     /* device workspace held now / at most */
    int64_t peak_running;            /* most requests running at once */
} bcur_stats;

bcur_status bcur_server_create(bcur_server** out, int device, size_t hbm_budget, int32_t max_slots);
/* Waits for queued and running requests, then frees everything. */
bcur_status bcur_server_destroy(bcur_server* srv);
/* BCUR_E_ADMIT when the request's footprint exceeds the whole budget. */
bcur_status bcur_server_submit(bcur_server* srv, const bcur_request* request, uint64_t* ticket);
/* BCUR_PENDING while running; otherwise the request's status, with the
 * results copied into `out` (host arrays as in bcur_result) and the ticket
 * released.  BCUR_E_STATE for an unknown or collected ticket. */
bcur_status bcur_server_poll(bcur_server* srv, uint64_t ticket, bcur_result* out);
/* As poll, but blocks until the request has finished. */
bcur_status bcur_server_wait(bcur_server* srv, uint64_t ticket, bcur_result* out);
bcur_status bcur_server_stats(bcur_server* srv, bcur_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* BCUR_H */
