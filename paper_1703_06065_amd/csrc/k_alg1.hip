// Kernels of Algorithm 1 (Sec. 3.1): uniform row draws, the transposed row
// sample, the scaled intersection W = R S and its pseudoinverse from an
// eigensystem of W's Gram matrix.
#include <limits.h>

#include "bcur_internal.h"

namespace bcur {
namespace {

// Row draws without replacement, each remaining row equally likely (one wave).
// Draw t takes the x-th free row in ascending order, x = floor(d_t (m - t) / 2^64).
// That row j* is the smallest fixed point at or above x of the non-decreasing
// f(j) = x + #{taken rows <= j}: iterating j <- f(j) from j = x climbs to it
// (every iterate stays <= j*), in at most t + 1 steps.  Draw t is kept in
// slot t: lane t % 64, register t / 64.
__global__ __launch_bounds__(64) void k_uniform_rows(int64_t m, const uint64_t* __restrict__ draws, int r,
                                                    int64_t* __restrict__ rows) {
    const int lane = threadIdx.x;
    // x of draws lane and lane + 64, computed up front
    const long long x0 = lane < r ? (long long)__umul64hi(draws[lane], (uint64_t)(m - lane)) : 0;
    const long long x1 = lane + 64 < r ? (long long)__umul64hi(draws[lane + 64], (uint64_t)(m - lane - 64)) : 0;
    long long a0 = LLONG_MAX, a1 = LLONG_MAX;
    for (int t = 0; t < r; ++t) {
        const long long xt = t < 64 ? x0 : x1;
        const int src = t & 63;
        const long long x = (long long)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(xt >> 32), src) << 32) |
                                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)xt, src));
        long long j = x;
        for (;;) {
            const long long jn = x + __popcll(__ballot(a0 <= j)) + __popcll(__ballot(a1 <= j));
            if (jn == j) break;
            j = jn;
        }
        if (lane == src) {
            if (t < 64) a0 = j;
            else a1 = j;
        }
        if (lane == 0) rows[t] = j;
    }
}

// RT (n x ldrt) = A[rows, :]^T, zero in columns r .. ldrt-1; 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_gather_rows_t(const float* __restrict__ A, int64_t lda, int64_t n,
                                                      const int64_t* __restrict__ rows, int r,
                                                      float* __restrict__ RT, int64_t ldrt) {
    __shared__ float tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int i0 = blockIdx.y * 64;
    for (int ii = ty; ii < 64; ii += 4) {
        const int i = i0 + ii;
        float v = 0.0f;
        if (i < r && j0 + tx < n) v = A[rows[i] * lda + j0 + tx];
        tile[ii][tx] = v;
    }
    __syncthreads();
    for (int jj = ty; jj < 64; jj += 4) {
        const int64_t j = j0 + jj;
        const int i = i0 + tx;
        if (j < n && i < ldrt) RT[j * ldrt + i] = tile[tx][jj];
    }
}

// W = alpha R S in FP64, W[i][t] = alpha d[t] RT[cols[t]][i] (i < r, t < c), stored
// transposed (Wt, c x r) or not (W, r x c).  One workgroup per column t of W.
__global__ __launch_bounds__(128) void k_alg1_w(const float* __restrict__ RT, int64_t ldrt, int r,
                                               const int64_t* __restrict__ cols, const double* __restrict__ d,
                                               int64_t c, double alpha, int transposed, double* __restrict__ W) {
    const int64_t t = blockIdx.x;
    const double sc = alpha * d[t];
    const float* src = RT + cols[t] * ldrt;
    for (int i = threadIdx.x; i < r; i += 128) {
        const double v = sc * (double)src[i];
        if (transposed) W[t * r + i] = v;
        else W[(int64_t)i * c + t] = v;
    }
}

// M (t x t) = sum over the kept j of v_j v_j^T / lam_j, with lam descending and
// V (t x t, ld t) holding the eigenvectors v_j in its columns.  Kept: lam_j >
// cut lam_0, then at most rank_k of them when rank_k > 0.  cnt[0] = eigenvalues
// above the cutoff, cnt[1] = kept.  One workgroup per row of M.
__global__ __launch_bounds__(128) void k_pinv_eig(const double* __restrict__ lam, const double* __restrict__ V,
                                                 int t, double cut, int rank_k, double* __restrict__ M,
                                                 int* __restrict__ cnt, const int* __restrict__ gate) {
    __shared__ double va[128];
    if (gate && *gate == 0) return;
    const int a = blockIdx.x, tid = threadIdx.x;
    const double l0 = lam[0];
    const int above = __syncthreads_count(tid < t && l0 > 0.0 && lam[tid < t ? tid : 0] > cut * l0);
    const int kept = rank_k > 0 && rank_k < above ? rank_k : above;
    if (tid < t) va[tid] = tid < kept ? V[(int64_t)a * t + tid] / lam[tid] : 0.0;
    __syncthreads();
    if (tid < t) {
        const double* vb = V + (int64_t)tid * t;
        double acc = 0.0;
        for (int j = 0; j < kept; ++j) acc = fma(va[j], vb[j], acc);
        M[(int64_t)a * t + tid] = acc;
    }
    if (a == 0 && tid == 0) {
        cnt[0] = above;
        cnt[1] = kept;
    }
}

// Decides between the Cholesky route and the eigensystem for the pseudoinverse
// of the Gram matrix G (t x t) of W.  With G + s I = R^T R (s the factor's
// shift) and Rinv = R^-1, lam_min(G) >= 1 / ||Rinv||_F^2 - s and lam_max(G) <=
// trace(G); when the first bound exceeds 4 cut2 times the second, no
// eigenvalue of G can fall at or below the cutoff (cut2 lam_max), G^+ = G^-1,
// and the Cholesky route is exact up to rounding: use_eig = 0, cnt = {t, t}.
// Otherwise (a small pivot, a truncation asked for, or no certificate)
// use_eig = 1.  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_pinv_certify(const double* __restrict__ G, const double* __restrict__ Rinv,
                                                     int t, const int* __restrict__ chol_info, double cut2,
                                                     int force_eig, int* __restrict__ use_eig,
                                                     int* __restrict__ cnt) {
    __shared__ double s_tr[4], s_fr[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double tr = 0.0, fr = 0.0;
    for (int i = tid; i < t; i += 256) tr += G[(int64_t)i * t + i];
    // the upper triangle of Rinv: rows by wave, columns by lane
    for (int i = wave; i < t; i += 4)
        for (int j = i + lane; j < t; j += 64) {
            const double v = Rinv[(int64_t)i * t + j];
            fr = fma(v, v, fr);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o, 64);
        fr += __shfl_xor(fr, o, 64);
    }
    if ((tid & 63) == 0) {
        s_tr[tid >> 6] = tr;
        s_fr[tid >> 6] = fr;
    }
    __syncthreads();
    if (tid == 0) {
        const double trace = (s_tr[0] + s_tr[1]) + (s_tr[2] + s_tr[3]);
        const double fro2 = (s_fr[0] + s_fr[1]) + (s_fr[2] + s_fr[3]);
        const double shift = (double)t * ldexp(1.0, -52) * trace;
        const bool ok = !force_eig && *chol_info == 0 && trace > 0.0 && 1.0 / fro2 - shift > 4.0 * cut2 * trace;
        use_eig[0] = ok ? 0 : 1;
        if (ok) {
            cnt[0] = t;
            cnt[1] = t;
        }
    }
}

// M (t x t) = Rinv Rinv^T = (R^T R)^-1 for upper triangular Rinv; skipped when
// *use_eig is set.  One workgroup per row of M.
__global__ __launch_bounds__(128) void k_gram_inv_rinv(const double* __restrict__ Rinv, int t,
                                                      double* __restrict__ M, const int* __restrict__ use_eig) {
    __shared__ double ra[128];
    if (*use_eig) return;
    const int a = blockIdx.x, tid = threadIdx.x;
    if (tid < t) ra[tid] = tid >= a ? Rinv[(int64_t)a * t + tid] : 0.0;
    __syncthreads();
    if (tid < t) {
        const double* rb = Rinv + (int64_t)tid * t;
        double acc = 0.0;
        for (int k = a > tid ? a : tid; k < t; ++k) acc = fma(ra[k], rb[k], acc);
        M[(int64_t)a * t + tid] = acc;
    }
}

// Y = X M (X: K x t, M: t x t symmetric, FP64), scaled by s_i = alpha d[i] per
// row of the core and rounded to FP32: U[i][j] = s_i Y[i][j], or, transposed,
// U[j][i] = s_j Y[i][j].  A workgroup takes 16 rows of X (staged in LDS) and
// all t columns; thread (j, q) accumulates rows 4q .. 4q+3 of column j.
constexpr int kPaRows = 16;
__global__ __launch_bounds__(256) void k_pinv_apply(const double* __restrict__ X, int64_t K, int t,
                                                   const double* __restrict__ M, const double* __restrict__ d,
                                                   double alpha, int transposed, float* __restrict__ U,
                                                   int64_t ldu) {
    __shared__ double xs[kPaRows][129];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kPaRows;
    const int nrow = (int)(K - i0 < kPaRows ? K - i0 : kPaRows);
    for (int e = tid; e < kPaRows * t; e += 256) {
        const int rr = e / t, k = e - rr * t;
        xs[rr][k] = rr < nrow ? X[(i0 + rr) * t + k] : 0.0;
    }
    __syncthreads();
    // columns j = tid % 64 + 64 h (h = 0, 1), row quarter q = tid / 64
    const int jl = tid & 63, q = tid >> 6;
    for (int h = 0; h < 2; ++h) {
        const int j = jl + 64 * h;
        if (j >= t) break;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < t; ++k) {
            const double mk = M[(int64_t)k * t + j];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(xs[4 * q + u][k], mk, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int rr = 4 * q + u;
            if (rr < nrow) {
                const int64_t i = i0 + rr;
                if (transposed) U[(int64_t)j * ldu + i] = (float)(alpha * d[j] * acc[u]);
                else U[i * ldu + j] = (float)(alpha * d[i] * acc[u]);
            }
        }
    }
}

}  // namespace

hipError_t launch_uniform_rows(int64_t m, const uint64_t* draws, int64_t r, int64_t* rows, hipStream_t st) {
    if (r < 1 || r > 128 || r > m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_uniform_rows, dim3(1), dim3(64), 0, st, m, draws, (int)r, rows);
    return hipGetLastError();
}

hipError_t launch_gather_rows_t(const float* A, int64_t lda, int64_t n, const int64_t* d_rows, int64_t r, float* RT,
                                int64_t ldrt, hipStream_t st) {
    if (r < 1 || ldrt < r || n < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((ldrt + 63) / 64));
    hipLaunchKernelGGL(k_gather_rows_t, grid, dim3(256), 0, st, A, lda, n, d_rows, (int)r, RT, ldrt);
    return hipGetLastError();
}

hipError_t launch_alg1_w(const float* RT, int64_t ldrt, int64_t r, const int64_t* d_cols, const double* d_scale,
                         int64_t c, double alpha, int transposed, double* W, hipStream_t st) {
    if (c < 1 || r < 1 || ldrt < r) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_alg1_w, dim3((unsigned)c), dim3(128), 0, st, RT, ldrt, (int)r, d_cols, d_scale, c, alpha,
                       transposed, W);
    return hipGetLastError();
}

hipError_t launch_pinv_eig(const double* lam, const double* V, int64_t t, double cut, int64_t rank_k, double* M,
                           int* cnt, const int* gate, hipStream_t st) {
    if (t < 1 || t > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pinv_eig, dim3((unsigned)t), dim3(128), 0, st, lam, V, (int)t, cut, (int)rank_k, M, cnt,
                       gate);
    return hipGetLastError();
}

hipError_t launch_pinv_certify(const double* G, const double* Rinv, int64_t t, const int* chol_info, double cut2,
                               int force_eig, int* use_eig, int* cnt, hipStream_t st) {
    if (t < 1 || t > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pinv_certify, dim3(1), dim3(256), 0, st, G, Rinv, (int)t, chol_info, cut2, force_eig,
                       use_eig, cnt);
    return hipGetLastError();
}

hipError_t launch_gram_inv_rinv(const double* Rinv, int64_t t, double* M, const int* use_eig, hipStream_t st) {
    if (t < 1 || t > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_inv_rinv, dim3((unsigned)t), dim3(128), 0, st, Rinv, (int)t, M, use_eig);
    return hipGetLastError();
}

hipError_t launch_pinv_apply(const double* X, int64_t K, int64_t t, const double* M, const double* d_scale,
                             double alpha, int transposed, float* U, int64_t ldu, hipStream_t st) {
    if (K < 1 || t < 1 || t > 128 || ldu < (transposed ? K : t)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pinv_apply, dim3((unsigned)((K + kPaRows - 1) / kPaRows)), dim3(256), 0, st, X, K, (int)t, M,
                       d_scale, alpha, transposed, U, ldu);
    return hipGetLastError();
}

}  // namespace bcur
