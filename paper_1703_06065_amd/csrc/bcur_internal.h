// Internal declarations shared by the Block CUR HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace bcur {

// Launch helpers return hipSuccess or the launch error.

// ---- reductions, scores, sampling, gather (k_basic.hip) -------------------
int frob2_grid(int64_t m, int64_t n);
hipError_t launch_frob2(const float* A, int64_t m, int64_t n, int64_t lda, double* partial, int grid,
                        double* out, hipStream_t st);
hipError_t launch_block_scores(const float* V, int64_t k, int64_t ldv, const int64_t* d_off, int64_t G,
                               double* scores, hipStream_t st);
// status[0] = 0 ok, 1 invalid scores; status[1] = 1 when a zero-weight block was drawn
hipError_t launch_sample(const double* scores, int64_t G, const uint64_t* draws, int64_t s, int replace,
                         uint64_t* qbuf, uint64_t* pref, int64_t* idx, double* weights, double* margins,
                         int* status, hipStream_t st);
hipError_t launch_gather_cols(const float* A, int64_t lda, int64_t m, const int64_t* d_cols, int64_t c,
                              float* C, int64_t ldc, hipStream_t st);
// out[t b + i] = map[off[idx[t]] + i] (identity when map is null) for s blocks of width b; an index
// outside [0, G) is read as 0
hipError_t launch_expand_blocks(const int64_t* idx, int64_t s, const int64_t* off, int64_t G, const int64_t* map,
                                int64_t b, int64_t* out, hipStream_t st);
// Q (n x wcols, ldq) = the Rademacher test matrix of `seed` in columns 0 .. l-1 (l <= 256,
// l <= wcols <= 256), zero in columns l .. wcols-1: row i from the Philox4x64-10 block of
// counter (i, 0, 0, 0) and key (seed, 0), bit j giving +1 (0) or -1 (1)
hipError_t launch_test_matrix(uint64_t seed, int64_t n, int64_t l, int64_t wcols, float* Q, int64_t ldq,
                              hipStream_t st);
hipError_t launch_gather_rows(const float* A, int64_t lda, int64_t n, const int64_t* d_rows, int64_t r,
                              float* R, int64_t ldr, hipStream_t st);
hipError_t launch_sum_f64(const double* x, int64_t count, double* out, hipStream_t st);
// G (c x c, FP64) = symmetrized H[:, cols]; G32 (ld ldg32), when not null, gets the same values in FP32
hipError_t launch_gram_from_cols(const float* H, int64_t ldh, const int64_t* d_cols, int64_t c, double* G,
                                 hipStream_t st, float* G32 = nullptr, int64_t ldg32 = 0);
hipError_t launch_f64_to_f32(const double* x, int64_t count, float* y, hipStream_t st);
// y[:, 0:cols] (row stride ldy) = x (rows x cols, ldx) rounded to FP32; with
// zero_pad, also zero in columns cols..ldy-1 (y then owns whole rows of ldy:
// never for a block of columns inside a wider matrix)
hipError_t launch_f64_to_f32_2d(const double* x, int64_t rows, int64_t cols, int64_t ldx, float* y, int64_t ldy,
                                bool zero_pad, hipStream_t st);
hipError_t launch_cast_bf16(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out, int64_t ldo,
                            hipStream_t st);
hipError_t launch_zero_f32(float* x, int64_t rows, int64_t cols, int64_t ld, hipStream_t st);
// ncol[0 .. n - c) = the columns of 0 .. n-1 that are not in cols (c distinct
// columns in [0, n), n <= kComplementMaxN), ascending.  A list that repeats a
// column or names one outside [0, n) sets *bad = 1 (the first n - c of the
// columns left are still written, nothing past them).
constexpr int64_t kComplementMaxN = 262144;
hipError_t launch_complement_cols(const int64_t* cols, int64_t c, int64_t n, int* ncol, int* bad, hipStream_t st);
// U[i][cols[k]] = (i == k) for i, k < c and, when F is not null, F[i][cols[k]] = 0
hipError_t launch_pin_selected(const int64_t* cols, int64_t c, float* U, int64_t ldu, float* F, int64_t ldf,
                               hipStream_t st);
hipError_t launch_fit_err(const double* parts, int64_t nparts_e, const double* dot_parts, int64_t nparts_d,
                          double* out, hipStream_t st);

// ---- FP32 MFMA GEMM (k_sgemm.hip) ------------------------------------------
enum GemmEpi { EPI_STORE = 0, EPI_RESID = 1, EPI_ADD_DOT = 2, EPI_RESID_NORM = 3, EPI_STORE_SQA = 4 };
struct GemmPlan {
    int splits = 1;
    int64_t kchunk = 0;
    int64_t wgs = 0;     // workgroups of the main kernel
    int cfg = 0;         // tile configuration index
};
// D = op(A) B, op(A) = A (M x K, lda) or A^T (A stored K x M, lda); B is K x N (ldb).
GemmPlan plan_sgemm(int64_t M, int64_t N, int64_t K, bool transA, bool allow_split);
size_t sgemm_partial_floats(const GemmPlan& p, int64_t M, int64_t N);
// plan_sgemm (split-K allowed) with at most cap_floats of split partials: the
// split count is lowered when the plan's would need more (a workspace laid out
// for a larger product than the one run can hold fewer splits of it)
GemmPlan plan_sgemm_within(int64_t M, int64_t N, int64_t K, bool transA, size_t cap_floats);
// EPI_STORE: D = acc.  EPI_RESID: D = X - acc, wsum[wg] = sum (X - acc)^2.
// EPI_RESID_NORM: wsum only, D is not written (may be null).
// EPI_STORE_SQA (A not transposed): as EPI_STORE, and wsum[wg] (one per workgroup of the grid,
// p.wgs in all, split-K included) = the FP64 sum of squares of the A elements that workgroup
// loaded, so that the sum over all of them is ||A||_F^2.
// EPI_ADD_DOT: D = X + acc, wsum[wg] = sum acc * Y.   Epilogues need splits == 1 here;
// launch_sgemm also takes EPI_RESID with split-K (D = X - the split sum, no wsum written).
// main kernel only (partial tiles when split) and the split-K sum
hipError_t launch_sgemm_main(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A,
                             int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd, float* partial,
                             int epi, const float* X, int64_t ldx, const float* Y, int64_t ldy, double* wsum,
                             hipStream_t st, const int* ncol = nullptr);
hipError_t launch_splitk_reduce(const GemmPlan& p, int64_t M, int64_t N, const float* partial, float* D,
                                int64_t ldd, hipStream_t st);
// wsum partials written by the norm-only residual epilogue (EPI_RESID_NORM) of an M x N x K
// product planned with plan_sgemm(M, N, K, false, false): one per workgroup
int64_t resid_parts(int64_t M, int64_t N, int64_t K);
// The most partials any norm-only residual of M x N writes, whatever K (its
// tile depends on M N K: a buffer laid out for the largest K a call may see
// must hold the smaller tile's count)
int64_t resid_parts_max(int64_t M, int64_t N);
// Whether EPI_RESID_NORM of an M x N x K product runs on the split-BF16 tile,
// the one that takes a column list (ncol: output column j is column ncol[j]
// of B and X, j < N; launch_sgemm_main rejects a list anywhere else)
bool resid_cols_ok(int64_t M, int64_t N, int64_t K);
// Rounds of 256 workgroups (one a compute unit on the split-BF16 tile) the
// norm-only residual of M x N x K launches
int64_t resid_rounds(int64_t M, int64_t N, int64_t K);
// wsum partials written by EPI_RESID (the FP32 square tile) of an M x N product
int64_t resid_store_parts(int64_t M, int64_t N);
// D = X + op(A) B and wsum[w] = partial sums of (op(A) B) * Y,
// with split-K when the plan has it (the sum and the epilogue then run in a
// second kernel).  add_dot_parts gives the number of wsum partials written.
int64_t add_dot_parts(const GemmPlan& p, int64_t M, int64_t N, int64_t K);
// the most add_dot_parts gives for M x N, whatever K and plan
int64_t add_dot_parts_max(int64_t M, int64_t N);
hipError_t launch_sgemm_add_dot(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A,
                                int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd, float* partial,
                                const float* X, int64_t ldx, const float* Y, int64_t ldy, double* wsum, hipStream_t st);
hipError_t launch_sgemm(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A,
                        int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd, float* partial,
                        int epi, const float* X, int64_t ldx, const float* Y, int64_t ldy, double* wsum,
                        hipStream_t st);

// ---- BF16 sketch passes (k_bgemm.hip) ----------------------------------------
// out = bf16(A) (m x n, ldo) and outT = bf16(A)^T (n x m, ldt); either may be null.
hipError_t launch_cast_bf16_both(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out, int64_t ldo,
                                 uint16_t* outT, int64_t ldt, hipStream_t st);
// D (M x N, FP32) = A (M x K, bf16, lda) * B^T with B stored N x K (bf16, ldb); leading
// dimensions multiples of 8.  Split partial tiles go to `partial` (sum with launch_splitk_reduce).
GemmPlan plan_bgemm(int64_t M, int64_t N, int64_t K);
hipError_t launch_bgemm_nt(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda,
                           const uint16_t* B, int64_t ldb, float* D, int64_t ldd, float* partial, hipStream_t st);

// ---- small dense FP64 kernels (k_small.hip) --------------------------------
int gram_wgs(int64_t rows);
// partial[w] (l x l) = sum over the w-th row range of X^T X, FP64 accumulation (wgs partials).
// With gate non-null the Gram, reduce, factor and apply kernels return at once when *gate == 0.
hipError_t launch_gram64(const float* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                         hipStream_t st, const int* gate = nullptr);
// the same for an FP64 X
hipError_t launch_gram64(const double* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                         hipStream_t st);
// T (l x l) = sum of the wgs partials in a fixed order, many workgroups.
hipError_t launch_gram_reduce(const double* partial, int parts, int64_t l, double* T, hipStream_t st,
                              const int* gate = nullptr);
// T = sum of the partials; T + shift I = R^T R (R upper), Rinv = R^-1 (l x l upper),
// shift = l 2^-52 trace(T).  info[0] |= 1 when the smallest pivot was below 10 * shift.
// need2 (or null): 0 when ||T||_F ||Rinv||_F^2 < 2^26 and no pivot was small (one Cholesky QR
// pass then leaves an orthogonality error below 2^-26), else 1.
hipError_t launch_chol_rinv_small(const double* T, int64_t l, double* Rinv, int* info, hipStream_t st,
                                  const int* gate = nullptr, int* need2 = nullptr);
// out (rows x lo, FP32, ldo) = X (rows x li, FP32, ldx) * M (li x lo, FP64, ldm)
hipError_t launch_apply_small(const float* X, int64_t rows, int64_t li, int64_t ldx, const double* M,
                              int64_t lo, int64_t ldm, float* out, int64_t ldo, hipStream_t st,
                              const int* gate = nullptr);
// Symmetric eigensolver (cyclic Jacobi) of the l x l matrix T (FP64):
// lam (l, descending), Wk (l x k, FP64), Wks = Wk diag(1/sqrt(lam)) (l x k) or null;
// info[0] = sweeps, info[1] = 1 when converged.  ws: jacobi_ws_bytes(l) bytes.
size_t jacobi_ws_bytes(int64_t l);
// With gate non-null both kernels return at once when *gate == 0 (nothing is written).
hipError_t launch_jacobi_eigh(const double* T, int64_t l, int64_t k, double* lam, double* Wk, double* Wks, void* ws,
                              int* info, hipStream_t st, const int* gate = nullptr);

// ---- blocked FP64 Cholesky inverse (k_dense64.hip) -------------------------
size_t spd_inverse_ws_doubles(int64_t c);
// Ginv = G^-1 for SPD G (c x c, FP64, overwritten by its Cholesky factor).
// info[0] |= 1 when a pivot fell below tau = c rel_tau max diag (rel_tau: the relative
// accuracy of G's entries, 2^-24 for a Gram matrix formed in FP32, 2^-50 for one formed in
// FP64): that column is dropped and its rows and columns of Ginv are zero (the inverse of
// the kept columns' Gram matrix);
// piv[0] = min pivot, piv[1] = max pivot (of the Schur complements).
hipError_t launch_spd_inverse(double* G, int64_t c, double* Ginv, double* ws, int* info, double* piv,
                              double rel_tau, hipStream_t st);
// The same factorization, returning *Linv = L^-1 (c x c, lower, inside ws) instead of G^-1.
hipError_t launch_chol_linv(double* G, int64_t c, double* ws, int* info, double* piv, double rel_tau,
                            double** Linv, hipStream_t st);
// D = alpha op(A) op(B) + beta D in FP64 (op = transpose when the flag is set); the
// _ff / _fd variants read FP32 operands (A and B, or A only), widened exactly.
hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, bool tA,
                        const double* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd,
                        hipStream_t st);
hipError_t launch_dgemm_ff(int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda, bool tA,
                           const float* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd,
                           hipStream_t st);
hipError_t launch_dgemm_fd(int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda, bool tA,
                           const double* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd,
                           hipStream_t st);
hipError_t launch_dgemm_df(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, bool tA,
                           const float* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st);

// ---- diagnostics (k_diag.hip) --------------------------------------------------
constexpr int kDiagMaxD = 64;   // largest min(block width, k) of the stable-rank kernel
// ratios[g] = ||X_g||_F^2 / ||X_g||_2^2 for the slice X_g of V (rows d_off[g] .. d_off[g+1]-1),
// NaN for a zero slice; steps[g] = squaring steps taken; needs min(width, k) <= kDiagMaxD for every block
hipError_t launch_block_stable_rank(const float* V, int64_t k, int64_t ldv, const int64_t* d_off, int64_t G,
                                    double* ratios, int* steps, hipStream_t st);
int row_norm_grid(int64_t m);
// out[0] = (m / k) max_i sum_c U[i][c]^2; partial: row_norm_grid(m) doubles
hipError_t launch_incoherence(const float* U, int64_t m, int64_t k, int64_t ldu, double* partial, double* out,
                              hipStream_t st);

// ---- Algorithm 1 (k_alg1.hip) ------------------------------------------------
// rows[t] (t < r <= min(m, 128)): the x-th row not yet taken, x = floor(draws[t] (m - t) / 2^64)
hipError_t launch_uniform_rows(int64_t m, const uint64_t* draws, int64_t r, int64_t* rows, hipStream_t st);
// RT (n x ldrt) = A[rows, :]^T, columns r .. ldrt-1 zero
hipError_t launch_gather_rows_t(const float* A, int64_t lda, int64_t n, const int64_t* d_rows, int64_t r, float* RT,
                                int64_t ldrt, hipStream_t st);
// W = alpha R S in FP64 with W[i][t] = alpha d_scale[t] RT[d_cols[t]][i]: stored as Wt (c x r, ld r)
// when transposed = 1, else as W (r x c, ld c)
hipError_t launch_alg1_w(const float* RT, int64_t ldrt, int64_t r, const int64_t* d_cols, const double* d_scale,
                         int64_t c, double alpha, int transposed, double* W, hipStream_t st);
// M (t x t) = V diag(1/lam over the kept prefix) V^T (lam descending, V t x t with eigenvectors in
// columns); kept = #{lam_j > cut lam_0}, capped at rank_k when rank_k > 0; cnt = {above cut, kept}.
// Skipped when gate is non-null and *gate == 0.
hipError_t launch_pinv_eig(const double* lam, const double* V, int64_t t, double cut, int64_t rank_k, double* M,
                           int* cnt, const int* gate, hipStream_t st);
// *use_eig = 0 (and cnt = {t, t}) when G's Cholesky inverse factor Rinv certifies that no eigenvalue
// of G is at or below cut2 lam_max and force_eig is 0; else *use_eig = 1
hipError_t launch_pinv_certify(const double* G, const double* Rinv, int64_t t, const int* chol_info, double cut2,
                               int force_eig, int* use_eig, int* cnt, hipStream_t st);
// M = Rinv Rinv^T (t x t), skipped when *use_eig != 0
hipError_t launch_gram_inv_rinv(const double* Rinv, int64_t t, double* M, const int* use_eig, hipStream_t st);
// Y = X M for X (K x t, FP64, ld t) and M (t x t, FP64, symmetric); with row scales s_i = alpha
// d_scale[i]: transposed = 0 stores U[i][j] = s_i Y[i][j] (K x t), transposed = 1 stores
// U[j][i] = s_j Y[i][j] (t x K), rounded to FP32 (ldu)
hipError_t launch_pinv_apply(const double* X, int64_t K, int64_t t, const double* M, const double* d_scale,
                             double alpha, int transposed, float* U, int64_t ldu, hipStream_t st);

}  // namespace bcur
