// Diagnostics of the sample complexity (Sec. 3.2): the block stable rank of
// Def. 3 (per block the stable rank ||X||_F^2 / ||X||_2^2 of the slice X of
// V_k) and the column-space incoherence of Def. 4 (the largest row norm of
// U_k, scaled by m / k).
#include <math.h>

#include "bcur_internal.h"

namespace bcur {
namespace {

constexpr int kDLd = kDiagMaxD + 1;

// Sum over the workgroup of one double per thread (256 threads), returned to
// every thread.
__device__ __forceinline__ double wg_sum256(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// One workgroup per block g.  X = V[off[g] .. off[g+1]-1, :] (b x k, FP32).
// Y = X X^T (b x b) when b <= k, else X^T X (k x k): d = min(b, k) <= kDiagMaxD,
// in FP64 with exact products.  ||X||_F^2 = trace Y.  ||X||_2^2 = lambda_max(Y)
// by repeated squaring: P = Y / trace Y, then P <- P^2 / trace(P^2), which
// multiplies the ratio of any eigenvalue to the largest by itself each step,
// so P tends to the projector onto the top eigenspace divided by its
// dimension; the iteration stops when P moves by at most 1e-12 in the
// Frobenius norm (at most 64 steps).  lambda_max is then the Rayleigh
// quotient of Y at the column of P with the largest diagonal entry.
// ratios[g] = trace Y / lambda_max, NaN for a zero slice.
__global__ __launch_bounds__(256) void k_block_stable_rank(const float* __restrict__ V, int k, int64_t ldv,
                                                          const int64_t* __restrict__ off,
                                                          double* __restrict__ ratios, int* __restrict__ steps) {
    __shared__ double Y[kDiagMaxD * kDLd], P[kDiagMaxD * kDLd], Q[kDiagMaxD * kDLd];
    __shared__ double red[4];
    __shared__ double s_tr;
    __shared__ int s_col;
    const int g = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = off[g];
    const int b = (int)(off[g + 1] - r0);
    const bool by_rows = b <= k;
    const int d = by_rows ? b : k;
    for (int e = tid; e < d * d; e += 256) {
        const int i = e / d, j = e - i * d;
        double acc = 0.0;
        if (by_rows) {
            const float* xi = V + (r0 + i) * ldv;
            const float* xj = V + (r0 + j) * ldv;
            for (int c = 0; c < k; ++c) acc = fma((double)xi[c], (double)xj[c], acc);
        } else {
            for (int rr = 0; rr < b; ++rr) {
                const float* x = V + (r0 + rr) * ldv;
                acc = fma((double)x[i], (double)x[j], acc);
            }
        }
        Y[i * kDLd + j] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < d; ++i) tr += Y[i * kDLd + i];
        s_tr = tr;
    }
    __syncthreads();
    const double fro2 = s_tr;
    if (!(fro2 > 0.0)) {
        if (tid == 0) {
            ratios[g] = NAN;
            steps[g] = 0;
        }
        return;
    }
    for (int e = tid; e < d * d; e += 256) {
        const int i = e / d, j = e - i * d;
        P[i * kDLd + j] = Y[i * kDLd + j] / fro2;
    }
    __syncthreads();
    int it = 0;
    while (it < 64) {
        ++it;
        for (int e = tid; e < d * d; e += 256) {
            const int i = e / d, j = e - i * d;
            double acc = 0.0;
            for (int l = 0; l < d; ++l) acc = fma(P[i * kDLd + l], P[l * kDLd + j], acc);
            Q[i * kDLd + j] = acc;
        }
        __syncthreads();
        if (tid == 0) {
            double tr = 0.0;
            for (int i = 0; i < d; ++i) tr += Q[i * kDLd + i];
            s_tr = tr;
        }
        __syncthreads();
        const double tq = s_tr;
        double diff = 0.0;
        for (int e = tid; e < d * d; e += 256) {
            const int i = e / d, j = e - i * d;
            const double nv = Q[i * kDLd + j] / tq;
            const double dv = nv - P[i * kDLd + j];
            diff = fma(dv, dv, diff);
            P[i * kDLd + j] = nv;
        }
        const double dsum = wg_sum256(diff, red);
        if (dsum <= 1e-24) break;
    }
    __syncthreads();
    if (tid == 0) {
        int jb = 0;
        for (int j = 1; j < d; ++j)
            if (P[j * kDLd + j] > P[jb * kDLd + jb]) jb = j;
        s_col = jb;
    }
    __syncthreads();
    const int jb = s_col;
    // v = column jb of P; lambda = v^T Y v / v^T v
    double num = 0.0, den = 0.0;
    for (int i = tid; i < d; i += 256) {
        const double vi = P[i * kDLd + jb];
        double yv = 0.0;
        for (int l = 0; l < d; ++l) yv = fma(Y[i * kDLd + l], P[l * kDLd + jb], yv);
        num = fma(vi, yv, num);
        den = fma(vi, vi, den);
    }
    num = wg_sum256(num, red);
    den = wg_sum256(den, red);
    if (tid == 0) {
        ratios[g] = fro2 / (num / den);
        steps[g] = it;
    }
}

// partial[blockIdx] = the largest FP64 sum of squares over this workgroup's rows of U
__global__ __launch_bounds__(256) void k_row_norm_max(const float* __restrict__ U, int64_t m, int k, int64_t ldu,
                                                     double* __restrict__ partial) {
    __shared__ double red[4];
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        const float* u = U + i * ldu;
        double acc = 0.0;
        for (int c = 0; c < k; ++c) acc = fma((double)u[c], (double)u[c], acc);
        mx = fmax(mx, acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// out = scale * max over the partials (one workgroup)
__global__ __launch_bounds__(256) void k_max_scale(const double* __restrict__ partial, int parts, double scale,
                                                  double* __restrict__ out) {
    __shared__ double red[4];
    double mx = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) mx = fmax(mx, partial[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = scale * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

}  // namespace

int row_norm_grid(int64_t m) {
    int64_t g = (m + 255) / 256;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_block_stable_rank(const float* V, int64_t k, int64_t ldv, const int64_t* d_off, int64_t G,
                                    double* ratios, int* steps, hipStream_t st) {
    if (G < 1 || k < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_stable_rank, dim3((unsigned)G), dim3(256), 0, st, V, (int)k, ldv, d_off, ratios,
                       steps);
    return hipGetLastError();
}

hipError_t launch_incoherence(const float* U, int64_t m, int64_t k, int64_t ldu, double* partial, double* out,
                              hipStream_t st) {
    if (m < 1 || k < 1) return hipErrorInvalidValue;
    const int grid = row_norm_grid(m);
    hipLaunchKernelGGL(k_row_norm_max, dim3((unsigned)grid), dim3(256), 0, st, U, m, (int)k, ldu, partial);
    hipLaunchKernelGGL(k_max_scale, dim3(1), dim3(256), 0, st, (const double*)partial, grid,
                       (double)m / (double)k, out);
    return hipGetLastError();
}

}  // namespace bcur
