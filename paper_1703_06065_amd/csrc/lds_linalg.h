// One-workgroup FP64 factorizations on a matrix held in LDS, shared by the
// small-factorization kernels.  Control flow is uniform across the workgroup
// (every loop bound depends only on the matrix size), so no wave serializes
// on divergent lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace bcur {

// Right-looking Cholesky of the w x w symmetric matrix in S (row stride ld),
// in place: on return the lower triangle holds L with S = L L^T.  A pivot
// (Schur complement) not above `thr` marks its column as dropped: drop[j] = 1,
// the column of L is zero below a unit diagonal and it updates nothing.
// Rows and columns w .. wp-1 are set to the identity.  Returns (in every
// thread) the smallest and largest pivot seen.  One barrier per column.
// sq (wp doubles of LDS) receives sqrt of the pivots (1 for dropped ones).
__device__ inline void lds_cholesky(double* S, int ld, int w, int wp, double thr, int* drop, double* sq,
                                    double& pmin, double& pmax) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < wp; e += nt) drop[e] = 0;
    pmin = INFINITY;
    pmax = 0.0;
    for (int j = 0; j < w; ++j) {
        __syncthreads();
        const double d = S[j * ld + j];
        pmin = fmin(pmin, d);
        pmax = fmax(pmax, d);
        if (!(d > thr)) {
            if (tid == 0) drop[j] = 1;
            continue;
        }
        const double rd = 1.0 / d;
        // lower trailing triangle on a 16-wide thread grid (no integer division)
        for (int i = j + 1 + tid / 16; i < w; i += nt / 16) {
            const double lij = S[i * ld + j] * rd;
            for (int p = j + 1 + (tid & 15); p <= i; p += 16) S[i * ld + p] -= lij * S[p * ld + j];
        }
    }
    __syncthreads();
    // the pivots' square roots first: the scaling below overwrites the diagonal
    for (int j = tid; j < wp; j += nt) sq[j] = (j >= w || drop[j]) ? 1.0 : sqrt(S[j * ld + j]);
    __syncthreads();
    // scale the columns: L[i][j] = S[i][j] / sqrt(d_j); pad with the identity
    for (int i = tid / 16; i < wp; i += nt / 16)
        for (int j = tid & 15; j <= i; j += 16) {
            double v;
            if (i >= w || j >= w || drop[j]) v = i == j ? 1.0 : 0.0;
            else v = i == j ? sq[j] : S[i * ld + j] / sq[j];
            S[i * ld + j] = v;
        }
    __syncthreads();
}

// In-place inverse X = L^-1 of the lower-triangular wp x wp matrix in S
// (row stride ld, wp a power of two >= 8), by recursive 2x2 blocking:
// X21 = -X22 (L21 X11).  Diagonal 8x8 blocks are inverted first by forward
// substitution (one column per thread, from a copy in `base`, wp*8 doubles);
// each doubling step forms T = L21 X11 in the unused strict upper triangle
// and then overwrites L21 with X21.  A dropped index d (drop[d] != 0) takes
// 1/L_dd as 0, which zeroes row d and column d of X.  The strict upper
// triangle of S is clobbered.
__device__ inline void lds_tri_inverse(double* S, int ld, int wp, const int* drop, double* base) {
    const int tid = threadIdx.x, nt = blockDim.x;
    // copy the diagonal 8x8 blocks
    for (int e = tid; e < wp * 8; e += nt) {
        const int o = (e >> 6) * 8, i = (e >> 3) & 7, j = e & 7;
        base[e] = S[(o + i) * ld + o + j];
    }
    __syncthreads();
    for (int e = tid; e < wp; e += nt) {
        const int blk = e >> 3, c = e & 7, o = blk * 8;
        const double* L = base + blk * 64;
        for (int i = 0; i < 8; ++i) {
            double x = 0.0;
            if (i == c) {
                x = drop[o + c] ? 0.0 : 1.0 / L[c * 8 + c];
            } else if (i > c && !drop[o + i]) {
                double acc = 0.0;
                for (int p = c; p < i; ++p) acc = fma(L[i * 8 + p], S[(o + p) * ld + o + c], acc);
                x = -acc / L[i * 8 + i];
            }
            if (i >= c) S[(o + i) * ld + o + c] = x;
        }
    }
    __syncthreads();
    for (int lb = 3; (1 << lb) < wp; ++lb) {
        const int b = 1 << lb, total = wp * b / 2;
        // T = L21 X11 (X11 lower): T[i][j] = sum_{q=j}^{b-1} L21[i][q] X11[q][j]
        for (int e = tid; e < total; e += nt) {
            const int o = (e >> (2 * lb)) * 2 * b, i = (e >> lb) & (b - 1), j = e & (b - 1);
            const double* Lr = S + (o + b + i) * ld + o;
            const double* Xc = S + o * ld + o + j;
            // four interleaved partial sums (fixed order) break the FMA latency chain
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int q = j;
            for (; q + 3 < b; q += 4) {
                a0 = fma(Lr[q], Xc[q * ld], a0);
                a1 = fma(Lr[q + 1], Xc[(q + 1) * ld], a1);
                a2 = fma(Lr[q + 2], Xc[(q + 2) * ld], a2);
                a3 = fma(Lr[q + 3], Xc[(q + 3) * ld], a3);
            }
            for (; q < b; ++q) a0 = fma(Lr[q], Xc[q * ld], a0);
            S[(o + i) * ld + o + b + j] = (a0 + a1) + (a2 + a3);
        }
        __syncthreads();
        // X21 = -X22 T (X22 lower): X21[i][j] = -sum_{q=0}^{i} X22[i][q] T[q][j]
        for (int e = tid; e < total; e += nt) {
            const int o = (e >> (2 * lb)) * 2 * b, i = (e >> lb) & (b - 1), j = e & (b - 1);
            const double* Xr = S + (o + b + i) * ld + o + b;
            const double* Tc = S + o * ld + o + b + j;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int q = 0;
            for (; q + 3 <= i; q += 4) {
                a0 = fma(Xr[q], Tc[q * ld], a0);
                a1 = fma(Xr[q + 1], Tc[(q + 1) * ld], a1);
                a2 = fma(Xr[q + 2], Tc[(q + 2) * ld], a2);
                a3 = fma(Xr[q + 3], Tc[(q + 3) * ld], a3);
            }
            for (; q <= i; ++q) a0 = fma(Xr[q], Tc[q * ld], a0);
            S[(o + b + i) * ld + o + j] = -((a0 + a1) + (a2 + a3));
        }
        __syncthreads();
    }
}

// Fixed-order sum of `parts` arrays of `count` doubles, entry e:
// out(e) = sum_w x[w * count + e].  The loads of 8 partials are issued
// together so the sum is not bound by one memory latency per partial.
__device__ inline double sum_partials(const double* __restrict__ x, int parts, int64_t count, int64_t e) {
    double acc = 0.0;
    int w = 0;
    for (; w + 8 <= parts; w += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x[(w + u) * count + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; w < parts; ++w) acc += x[w * count + e];
    return acc;
}

__device__ inline int pow2_at_least8(int w) {
    int p = 8;
    while (p < w) p *= 2;
    return p;
}

}  // namespace bcur
