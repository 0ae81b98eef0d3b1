// One-workgroup FP64 building blocks shared by the small-factorization
// kernels: a register-resident Cholesky with the inverse of its factor, and a
// fixed-order sum of partial results.  Control flow is uniform across the
// workgroup (every loop bound depends only on the matrix size).
#pragma once

#include <hip/hip_runtime.h>

namespace bcur {

// Full-precision 1/sqrt(x) for x > 0 from the hardware estimate and two
// Newton steps (about 1 ulp; the factorizations need scalings accurate to
// working precision, not correctly rounded ones).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

// Register-resident Cholesky with the inverse of its factor, one workgroup of
// TG x TG threads, for a w x w symmetric matrix, w <= TG * NR.
//
// Storage: one lower triangle M, entry (i, c) held by thread (i mod TG,
// c mod TG) in slot tri_slot(i / TG, c / TG).  Step j reads the vector P (row j
// of M left of the diagonal, column j below it; d = P_j) from LDS, then every
// row i > j takes the rank-1 update
//     M[i][c] -= P_i P_c / d      (c != j),      M[i][j] = -P_i / d,
// and row j becomes final: M[j][c] = P_c / sqrt(d), M[j][j] = 1 / sqrt(d).
// Columns right of j still hold the Schur complement, columns up to j the
// rows of the inverse being formed (column-oriented forward substitution of
// L X = I fused into the right-looking factorization), so after w steps M
// holds X = L^-1 with G = L L^T.
// A pivot d not above `thr` drops index j: 1/sqrt(d) is taken as 0, which
// makes column j of L zero below a unit diagonal and zeroes row and column j
// of X, so X^T X is the inverse on the kept indices (zero elsewhere).
//
// The steps run in chunks of TG (j = TG A + jj) with the chunk A unrolled, so
// the slot row and column that hold index j, and the rows already final, are
// known at compile time; what remains at run time is per-lane predication.
// One barrier per step: P is double-buffered in `P` (2 * TG * NR doubles,
// plus one more that takes the stores a lane does not make).  The pivots go to `piv` (w doubles of LDS);
// pmin / pmax receive the smallest and largest pivot, ndrop the dropped count.
__host__ __device__ constexpr int tri_slot(int a, int b) { return a * (a + 1) / 2 + b; }

template <int TG, int NR, int A>
struct CholChunk {
    static __device__ __forceinline__ void run(double (&m)[NR * (NR + 1) / 2], int w, double thr, double* P,
                                               double* piv, int tr, int tc) {
        constexpr int WB = TG * NR;
        double* trash = P + 2 * WB;  // target of the stores a lane does not make
        if (TG * A < w) {
            const int jend = (TG * A + TG < w ? TG * A + TG : w) - TG * A;
            for (int jj = 0; jj < jend; ++jj) {
                const int j = TG * A + jj;
                const double* Pc = P + (j & 1) * WB;
                double* Pn = P + ((j + 1) & 1) * WB;
                const double d = Pc[j];
                double pc[NR], pr[NR];
#pragma unroll
                for (int b = 0; b < NR; ++b) pc[b] = Pc[tc + TG * b];
#pragma unroll
                for (int a = A; a < NR; ++a) pr[a] = Pc[tr + TG * a];
                if (threadIdx.x == 0) piv[j] = d;
                const double r = d > thr ? rsqrt_nr(d) : 0.0;
                const double rd = r * r;
                const bool colj = tc == jj;  // slot column A of this lane holds index j
#pragma unroll
                for (int a = A; a < NR; ++a) {
                    const double ai = (a > A || tr > jj) ? pr[a] * rd : 0.0;
#pragma unroll
                    for (int b = 0; b <= a; ++b) {
                        double& x = m[tri_slot(a, b)];
                        const double y = fma(-ai, pc[b], x);
                        x = (b == A && colj) ? -ai : y;
                    }
                }
                if (tr == jj) {  // row j becomes final
#pragma unroll
                    for (int b = 0; b <= A; ++b) {
                        const double v = pc[b] * r;
                        m[tri_slot(A, b)] = (b == A && colj) ? r : v;
                    }
                }
                // publish row j+1 (c <= j+1) and column j+1 (rows below it)
                const int jn = j + 1;
                if (jn < w) {
                    if (jj + 1 < TG) {
                        if (tr == jj + 1) {
#pragma unroll
                            for (int b = 0; b <= A; ++b) {
                                const bool ok = b < A || tc <= jj + 1;
                                *(ok ? Pn + tc + TG * b : trash) = m[tri_slot(A, b)];
                            }
                        }
                        if (tc == jj + 1) {
#pragma unroll
                            for (int a = A; a < NR; ++a) {
                                const int i = tr + TG * a;
                                const bool ok = (a > A || tr > jj + 1) && i < w;
                                *(ok ? Pn + i : trash) = m[tri_slot(a, A)];
                            }
                        }
                    } else if constexpr (A + 1 < NR) {
                        if (tr == 0) {
#pragma unroll
                            for (int b = 0; b <= A + 1; ++b) {
                                const bool ok = b <= A || tc == 0;
                                *(ok ? Pn + tc + TG * b : trash) = m[tri_slot(A + 1, b)];
                            }
                        }
                        if (tc == 0) {
#pragma unroll
                            for (int a = A + 1; a < NR; ++a) {
                                const int i = tr + TG * a;
                                const bool ok = (a > A + 1 || tr > 0) && i < w;
                                *(ok ? Pn + i : trash) = m[tri_slot(a, A + 1)];
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        if constexpr (A + 1 < NR) CholChunk<TG, NR, A + 1>::run(m, w, thr, P, piv, tr, tc);
    }
};

template <int TG, int NR>
__device__ inline void reg_chol_inv(double (&m)[NR * (NR + 1) / 2], int w, double thr, double* P, double* piv,
                                    double& pmin, double& pmax, int& ndrop) {
    const int tid = threadIdx.x, tr = tid / TG, tc = tid % TG;
    // publish row 0 / column 0
    if (tc == 0) {
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            const int i = tr + TG * a;
            if (i < w) P[i] = m[tri_slot(a, 0)];
        }
    }
    __syncthreads();
    CholChunk<TG, NR, 0>::run(m, w, thr, P, piv, tr, tc);
    // pivot range and count of dropped pivots, in every thread
    pmin = INFINITY;
    pmax = 0.0;
    ndrop = 0;
    for (int j = 0; j < w; ++j) {
        const double d = piv[j];
        pmin = fmin(pmin, d);
        pmax = fmax(pmax, d);
        ndrop += d > thr ? 0 : 1;
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


}  // namespace bcur
