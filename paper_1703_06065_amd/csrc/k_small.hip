// Small dense FP64 kernels of the range finder: Gram matrices of tall-skinny
// FP32 panels with FP64 accumulation, a one-workgroup shifted Cholesky with
// the inverse of its factor (for Cholesky QR), tall x small products, and a
// one-workgroup cyclic Jacobi eigensolver for the Rayleigh-Ritz step.
#include <math.h>

#include "bcur_internal.h"

namespace bcur {
namespace {

constexpr int kMaxL = 128;     // sketch width limit of the Gram / Cholesky / apply kernels
constexpr int kMaxLJ = 112;    // sketch width limit of the Jacobi kernel (LDS)
constexpr int kRC = 32;        // rows per LDS chunk

// partial[w] = X[rows of w]^T X[rows of w]; thread (ti, tj) owns the 4x4 block
// of entries (4 ti .. 4 ti + 3, 4 tj .. 4 tj + 3).  Products of two floats are
// exact in FP64 and every entry sums its rows in order, so T is symmetric bitwise.
__global__ __launch_bounds__(1024) void k_gram64(const float* __restrict__ X, int64_t rows, int l, int64_t ldx,
                                                 int64_t rows_per_wg, double* __restrict__ partial) {
    __shared__ __attribute__((aligned(16))) float xs[kRC * kMaxL];
    const int lp = (l + 3) & ~3, TT = lp / 4;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ti = tid / TT, tj = tid % TT;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = rows < r0 + rows_per_wg ? rows : r0 + rows_per_wg;
    for (int64_t rb = r0; rb < r1; rb += kRC) {
        const int nr = (int)(r1 - rb < kRC ? r1 - rb : kRC);
        __syncthreads();
        for (int e = tid; e < kRC * lp; e += nt) {
            const int rr = e / lp, cc = e % lp;
            xs[e] = (rr < nr && cc < l) ? X[(rb + rr) * ldx + cc] : 0.0f;
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            const float4 xi = *reinterpret_cast<const float4*>(&xs[rr * lp + 4 * ti]);
            const float4 xj = *reinterpret_cast<const float4*>(&xs[rr * lp + 4 * tj]);
            const double vi[4] = {xi.x, xi.y, xi.z, xi.w};
            const double vj[4] = {xj.x, xj.y, xj.z, xj.w};
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(vi[a], vj[b], acc[a][b]);
        }
    }
    double* out = partial + (int64_t)blockIdx.x * l * l;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = 4 * ti + a, j = 4 * tj + b;
            if (i < l && j < l) out[i * l + j] = acc[a][b];
        }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial, int wgs, int64_t ll,
                                                     double* __restrict__ T) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ll) return;
    double s = 0.0;
    for (int w = 0; w < wgs; ++w) s += partial[(int64_t)w * ll + e];
    T[e] = s;
}

// T + shift I = R^T R (R = L^T upper), Rinv = R^-1 upper.  One workgroup.
__global__ __launch_bounds__(256) void k_chol_rinv_small(const double* __restrict__ T, int l,
                                                         double* __restrict__ Rinv, int* __restrict__ info) {
    __shared__ double S[kMaxL * kMaxL];
    __shared__ double dinv[kMaxL];
    __shared__ double sshift;
    const int tid = threadIdx.x;
    for (int e = tid; e < l * l; e += 256) S[e] = T[e];
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < l; ++i) tr += S[i * l + i];
        double sh = (double)l * ldexp(1.0, -52) * tr;
        if (!(sh > 0.0)) sh = 1e-300;
        sshift = sh;
    }
    __syncthreads();
    const double shift = sshift;
    if (tid < l) S[tid * l + tid] += shift;
    double minpiv = INFINITY;
    for (int j = 0; j < l; ++j) {
        __syncthreads();
        double d = S[j * l + j];
        minpiv = fmin(minpiv, d);
        if (!(d > shift * 0.5)) d = shift;
        const int w = l - 1 - j;
        for (int e = tid; e < w * w; e += 256) {
            const int i = j + 1 + e / w, p = j + 1 + e % w;
            S[i * l + p] -= S[i * l + j] * S[p * l + j] / d;
        }
    }
    __syncthreads();
    // L[i][j] = S[i][j] / sqrt(d_j) (lower), L[j][j] = sqrt(d_j)
    for (int e = tid; e < l * l; e += 256) {
        const int i = e / l, j = e % l;
        if (i < j) continue;
        double d = S[j * l + j];
        if (!(d > shift * 0.5)) d = shift;
        const double sd = sqrt(d);
        if (i == j) continue;
        S[e] = S[e] / sd;
    }
    __syncthreads();
    if (tid < l) {
        double d = S[tid * l + tid];
        if (!(d > shift * 0.5)) d = shift;
        S[tid * l + tid] = sqrt(d);
    }
    __syncthreads();
    // X = L^-1 by forward substitution, one column per thread; X[p][c] (p > c)
    // is kept at S[c][p] (the unused upper triangle), X[c][c] in dinv[c].
    if (tid < l) {
        const int c = tid;
        dinv[c] = 1.0 / S[c * l + c];
        for (int i = c + 1; i < l; ++i) {
            double acc = S[i * l + c] * dinv[c];
            for (int p = c + 1; p < i; ++p) acc = fma(S[i * l + p], S[c * l + p], acc);
            S[c * l + i] = -acc / S[i * l + i];
        }
    }
    __syncthreads();
    // Rinv = X^T: Rinv[c][i] = X[i][c]
    for (int e = tid; e < l * l; e += 256) {
        const int c = e / l, i = e % l;
        Rinv[e] = i < c ? 0.0 : (i == c ? dinv[c] : S[c * l + i]);
    }
    if (tid == 0 && info) {
        if (minpiv < 1e3 * shift) atomicOr(info, 1);
    }
}

// out (rows x lo) = X (rows x li, FP32) * M (li x lo, FP64), FP64 accumulation.
__global__ __launch_bounds__(256) void k_apply_small(const float* __restrict__ X, int64_t rows, int li, int64_t ldx,
                                                     const double* __restrict__ M, int lo, int64_t ldm,
                                                     float* __restrict__ out, int64_t ldo) {
    __shared__ double Ms[kMaxL * kMaxL];
    __shared__ float Xs[kRC * (kMaxL + 1)];
    const int lop = (lo + 3) & ~3;
    const int lis = li + 1;
    const int tid = threadIdx.x;
    for (int e = tid; e < li * lop; e += 256) {
        const int i = e / lop, o = e % lop;
        Ms[e] = o < lo ? M[(int64_t)i * ldm + o] : 0.0;
    }
    const int tr = tid / 32, tc = tid % 32;   // 8 x 32 threads -> 32 rows x 128 columns
    for (int64_t rb = (int64_t)blockIdx.x * kRC; rb < rows; rb += (int64_t)gridDim.x * kRC) {
        const int nr = (int)(rows - rb < kRC ? rows - rb : kRC);
        __syncthreads();
        for (int e = tid; e < kRC * li; e += 256) {
            const int rr = e / li, cc = e % li;
            Xs[rr * lis + cc] = rr < nr ? X[(rb + rr) * ldx + cc] : 0.0f;
        }
        __syncthreads();
        if (4 * tc < lop) {
            double acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
            for (int i = 0; i < li; ++i) {
                double xv[4], mv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) xv[a] = Xs[(4 * tr + a) * lis + i];
#pragma unroll
                for (int b = 0; b < 4; ++b) mv[b] = Ms[i * lop + 4 * tc + b];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = fma(xv[a], mv[b], acc[a][b]);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int rr = 4 * tr + a;
                if (rr >= nr) continue;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int o = 4 * tc + b;
                    if (o < lo) out[(rb + rr) * ldo + o] = (float)acc[a][b];
                }
            }
        }
    }
}

__device__ __forceinline__ int pk(int i, int j, int L) {
    if (i > j) {
        const int t = i;
        i = j;
        j = t;
    }
    return i * L - (i * (i - 1)) / 2 + (j - i);
}

// Cyclic Jacobi on the symmetric l x l matrix T (FP64), one workgroup.
// Each round rotates L/2 disjoint index pairs (round-robin schedule), which
// lets every 2x2 block of T and every row of W be updated independently.
__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ T, int l, int k,
                                                 double* __restrict__ lam_out, double* __restrict__ Wk,
                                                 double* __restrict__ Wks, int* __restrict__ info) {
    __shared__ double P[kMaxLJ * (kMaxLJ + 1) / 2];
    __shared__ double W[kMaxLJ * kMaxLJ];
    __shared__ double cc[kMaxLJ / 2], ss[kMaxLJ / 2];
    __shared__ int cp[kMaxLJ / 2], cq[kMaxLJ / 2];
    __shared__ int rotflag;
    const int tid = threadIdx.x;
    const int L = l + (l & 1), H = L / 2;
    for (int e = tid; e < L * L; e += 1024) {
        const int i = e / L, j = e % L;
        if (i <= j) P[pk(i, j, L)] = (i < l && j < l) ? T[i * l + j] : 0.0;
        W[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    int sweeps = 0, converged = 0;
    for (int sw = 0; sw < 40; ++sw) {
        if (tid == 0) rotflag = 0;
        __syncthreads();
        for (int rd = 0; rd < L - 1; ++rd) {
            if (tid < H) {
                const int a = tid == 0 ? 0 : 1 + (tid - 1 + rd) % (L - 1);
                const int b = 1 + (L - 2 - tid + rd) % (L - 1);
                const int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < l) {
                    const double apq = P[pk(p, q, L)];
                    if (apq != 0.0) {
                        const double app = P[pk(p, p, L)], aqq = P[pk(q, q, L)];
                        if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
                            const double tau = (aqq - app) / (2.0 * apq);
                            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                            c = 1.0 / sqrt(1.0 + t * t);
                            s = t * c;
                            atomicOr(&rotflag, 1);
                        }
                    }
                }
                cp[tid] = p;
                cq[tid] = q;
                cc[tid] = c;
                ss[tid] = s;
            }
            __syncthreads();
            // T <- J^T T J, one 2x2 block per (pair a, pair b), a <= b
            for (int e = tid; e < H * H; e += 1024) {
                const int a = e / H, b = e % H;
                if (a > b) continue;
                const double s1 = ss[a], s2 = ss[b];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const double c1 = cc[a], c2 = cc[b];
                const int p1 = cp[a], q1 = cq[a], p2 = cp[b], q2 = cq[b];
                if (a == b) {
                    const double x00 = P[pk(p1, p1, L)], x01 = P[pk(p1, q1, L)], x11 = P[pk(q1, q1, L)];
                    const double y00 = c1 * x00 - s1 * x01, y01 = c1 * x01 - s1 * x11;
                    const double y10 = s1 * x00 + c1 * x01, y11 = s1 * x01 + c1 * x11;
                    P[pk(p1, p1, L)] = y00 * c1 - y01 * s1;
                    P[pk(q1, q1, L)] = y10 * s1 + y11 * c1;
                    P[pk(p1, q1, L)] = 0.0;
                } else {
                    const int i00 = pk(p1, p2, L), i01 = pk(p1, q2, L), i10 = pk(q1, p2, L), i11 = pk(q1, q2, L);
                    const double x00 = P[i00], x01 = P[i01], x10 = P[i10], x11 = P[i11];
                    const double y00 = c1 * x00 - s1 * x10, y01 = c1 * x01 - s1 * x11;
                    const double y10 = s1 * x00 + c1 * x10, y11 = s1 * x01 + c1 * x11;
                    P[i00] = y00 * c2 - y01 * s2;
                    P[i01] = y00 * s2 + y01 * c2;
                    P[i10] = y10 * c2 - y11 * s2;
                    P[i11] = y10 * s2 + y11 * c2;
                }
            }
            // W <- W J
            for (int e = tid; e < L * H; e += 1024) {
                const int i = e / H, a = e % H;
                const double s = ss[a];
                if (s == 0.0) continue;
                const double c = cc[a];
                const int p = cp[a], q = cq[a];
                const double wp = W[i * L + p], wq = W[i * L + q];
                W[i * L + p] = c * wp - s * wq;
                W[i * L + q] = s * wp + c * wq;
            }
            __syncthreads();
        }
        const int rf = rotflag;
        __syncthreads();
        ++sweeps;
        if (!rf) {
            converged = 1;
            break;
        }
    }
    // eigenvalues descending (ties by index) and the first k eigenvectors
    if (tid < l) {
        const double li = P[pk(tid, tid, L)];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double lj = P[pk(j, j, L)];
            rank += (lj > li) || (lj == li && j < tid);
        }
        lam_out[rank] = li;
        if (rank < k) {
            const double inv = li > 0.0 ? 1.0 / sqrt(li) : 0.0;
            for (int row = 0; row < l; ++row) {
                const double w = W[row * L + tid];
                Wk[row * k + rank] = w;
                if (Wks) Wks[row * k + rank] = w * inv;
            }
        }
    }
    if (tid == 0 && info) {
        info[0] = sweeps;
        info[1] = converged;
    }
}

}  // namespace

int gram_wgs(int64_t rows) {
    int64_t w = rows / 64;
    if (w > 240) w = 240;
    if (w < 1) w = 1;
    return (int)w;
}

hipError_t launch_gram64(const float* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs, double* T,
                         hipStream_t st) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    const int lp = ((int)l + 3) & ~3;
    const int nt = (lp / 4) * (lp / 4);
    const int64_t rpw = (rows + wgs - 1) / wgs;
    hipLaunchKernelGGL(k_gram64, dim3(wgs), dim3(nt < 64 ? 64 : nt), 0, st, X, rows, (int)l, ldx, rpw, partial);
    const int64_t ll = l * l;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ll + 255) / 256)), dim3(256), 0, st, (const double*)partial,
                       wgs, ll, T);
    return hipGetLastError();
}

hipError_t launch_chol_rinv_small(const double* T, int64_t l, double* Rinv, int* info, hipStream_t st) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_rinv_small, dim3(1), dim3(256), 0, st, T, (int)l, Rinv, info);
    return hipGetLastError();
}

hipError_t launch_apply_small(const float* X, int64_t rows, int64_t li, int64_t ldx, const double* M, int64_t lo,
                              int64_t ldm, float* out, int64_t ldo, hipStream_t st) {
    if (li < 1 || li > kMaxL || lo < 1 || lo > kMaxL) return hipErrorInvalidValue;
    int64_t blocks = (rows + kRC - 1) / kRC;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_apply_small, dim3((unsigned)blocks), dim3(256), 0, st, X, rows, (int)li, ldx, M, (int)lo,
                       ldm, out, ldo);
    return hipGetLastError();
}

hipError_t launch_jacobi_eigh(const double* T, int64_t l, int64_t k, double* lam, double* Wk, double* Wks, int* info,
                              hipStream_t st) {
    if (l < 1 || l > kMaxLJ || k < 1 || k > l) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, st, T, (int)l, (int)k, lam, Wk, Wks, info);
    return hipGetLastError();
}

}  // namespace bcur
