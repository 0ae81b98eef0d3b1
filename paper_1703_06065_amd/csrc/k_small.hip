// Small dense FP64 kernels of the range finder: Gram matrices of tall-skinny
// FP32 panels with FP64 accumulation, a one-workgroup shifted Cholesky with
// the inverse of its factor (for Cholesky QR), tall x small products, and a
// one-workgroup cyclic Jacobi eigensolver for the Rayleigh-Ritz step.
#include <math.h>

#include "bcur_internal.h"
#include "lds_linalg.h"

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

// T[e] = sum over the partial Gram matrices, fixed order: the `parts`
// partials are split into 4 groups (g = w mod 4), each thread sums one group
// for one entry with up to 16 loads in flight, and the 4 group sums are added
// in group order.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial, int parts, int64_t ll,
                                                     double* __restrict__ T) {
    __shared__ double sg[4][64];
    const int tid = threadIdx.x, g = tid >> 6, el = tid & 63;
    const int64_t e = (int64_t)blockIdx.x * 64 + el;
    double acc = 0.0;
    if (e < ll) {
        int w = g;
        for (; w + 12 < parts; w += 16) {
            const double v0 = partial[(int64_t)w * ll + e], v1 = partial[(int64_t)(w + 4) * ll + e];
            const double v2 = partial[(int64_t)(w + 8) * ll + e], v3 = partial[(int64_t)(w + 12) * ll + e];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; w < parts; w += 4) acc += partial[(int64_t)w * ll + e];
    }
    sg[g][el] = acc;
    __syncthreads();
    if (g == 0 && e < ll) T[e] = ((sg[0][el] + sg[1][el]) + sg[2][el]) + sg[3][el];
}

// T = sum of the `parts` l x l partial Gram matrices (fixed order); then
// T + shift I = R^T R with shift = l 2^-52 trace(T), and Rinv = R^-1 (upper,
// l x l).  One workgroup; LDS holds the padded matrix (row stride wp + 1).
__global__ __launch_bounds__(256) void k_chol_rinv_small(const double* __restrict__ partial, int parts, int l,
                                                         double* __restrict__ Rinv, int* __restrict__ info) {
    constexpr int LD = kMaxL + 1;
    __shared__ double S[kMaxL * LD];
    __shared__ double base[kMaxL * 8];
    __shared__ double dinv[kMaxL];
    __shared__ int drop[kMaxL];
    __shared__ double sshift;
    const int tid = threadIdx.x;
    const int wp = pow2_at_least8(l);
    const int ld = wp + 1;
    const int64_t ll = (int64_t)l * l;
    for (int i = tid / 16; i < l; i += 16)
        for (int j = tid & 15; j < l; j += 16) S[i * ld + j] = sum_partials(partial, parts, ll, i * l + j);
    (void)ll;
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < l; ++i) tr += S[i * ld + i];
        double sh = (double)l * ldexp(1.0, -52) * tr;
        if (!(sh > 0.0)) sh = 1e-300;
        sshift = sh;
    }
    __syncthreads();
    const double shift = sshift;
    if (tid < l) S[tid * ld + tid] += shift;
    double pmin, pmax;
    lds_cholesky(S, ld, l, wp, 0.0, drop, dinv, pmin, pmax);
    lds_tri_inverse(S, ld, wp, drop, base);
    // Rinv = X^T: Rinv[c][i] = X[i][c] for i >= c
    for (int e = tid; e < l * l; e += 256) {
        const int c = e / l, i = e % l;
        Rinv[e] = i < c ? 0.0 : S[i * ld + c];
    }
    if (tid == 0 && info && (pmin < 10.0 * shift)) atomicOr(info, 1);
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

// Full-precision 1/sqrt(x) and 1/x for x > 0 from the hardware estimates and
// two Newton steps (the rotations need c^2 + s^2 = 1 to working precision,
// not correctly rounded operations).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * fma(-x, y, 2.0);
    y = y * fma(-x, y, 2.0);
    return y;
}

// Cyclic Jacobi on the symmetric l x l matrix T (FP64), one workgroup.
// T is the sum of `parts` partial Gram matrices.  Each round rotates L/2
// disjoint index pairs (round-robin schedule), so every 2x2 block of T and
// every row of W is updated independently; a sweep is L-1 rounds and the
// iteration stops after a sweep without rotations.  A pair (p, q) is rotated
// while |a_pq| > max(2^-51 ||T||_F, 1e-15 sqrt|a_pp a_qq|).
// The tangent t of each rotation is computed in FP32 (hardware reciprocal and
// square root); c = 1/sqrt(1 + t^2) and s = t c are then formed in FP64 with
// Newton-refined estimates, so every rotation is orthogonal to FP64 precision
// while its angle is accurate to about 2^-23.  The (p, q) entry left by the
// slightly inexact angle is kept (not forced to zero), so no backward error is
// introduced; later rounds remove it.
__device__ __forceinline__ void jacobi_angle(double app, double aqq, double apq, double& c, double& s) {
    const double d = aqq - app;
    double t;
    if (fabs(apq) < 1e-30 * fabs(d)) {
        t = apq * rcp_nr(d);                       // |tau| > 1e30: t = 1 / (2 tau)
    } else {
        // scale both by one power of two so the FP32 conversion cannot overflow
        int e;
        frexp(fmax(fabs(d), fabs(apq)), &e);
        const float df = (float)ldexp(d, -e), af = (float)ldexp(apq, -e);
        const float tau = df * __builtin_amdgcn_rcpf(2.0f * af);
        const float at = fabsf(tau);
        float tf = __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.0f)));
        if (tau < 0.0f) tf = -tf;
        t = (double)tf;
    }
    c = rsqrt_nr(fma(t, t, 1.0));
    s = t * c;
}

__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ partial, int parts, int l, int k,
                                                 double* __restrict__ lam_out, double* __restrict__ Wk,
                                                 double* __restrict__ Wks, int* __restrict__ info) {
    __shared__ double P[kMaxLJ * (kMaxLJ + 1) / 2];
    __shared__ double W[kMaxLJ * kMaxLJ];
    __shared__ double cc[kMaxLJ / 2], ss[kMaxLJ / 2];
    __shared__ int cp[kMaxLJ / 2], cq[kMaxLJ / 2];
    __shared__ int blk[(kMaxLJ / 2) * (kMaxLJ / 2 + 1) / 2];
    __shared__ int rotflag;
    __shared__ double snorm, sred[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = l + (l & 1), H = L / 2;
    const int nblk = H * (H + 1) / 2;
    const int64_t ll = (int64_t)l * l;
    const int TX = 32, TY = nt / 32, tx = tid % 32, ty = tid / 32;
    for (int i = ty; i < L; i += TY)
        for (int j = tx; j < L; j += TX) {
            if (i <= j) P[pk(i, j, L)] = (i < l && j < l) ? sum_partials(partial, parts, ll, i * l + j) : 0.0;
            W[i * L + j] = i == j ? 1.0 : 0.0;
        }
    // block table: (a, b) with a <= b, packed as a | b << 16; row a starts at a H - a (a - 1) / 2
    if (tid < H) {
        const int a = tid, o = a * H - (a * (a - 1)) / 2;
        for (int b = a; b < H; ++b) blk[o + b - a] = a | (b << 16);
    }
    __syncthreads();
    {
        double f = 0.0;
        for (int i = ty; i < l; i += TY)
            for (int j = i + tx; j < l; j += TX) {
                const double v = P[pk(i, j, L)];
                f += (i == j ? 1.0 : 2.0) * v * v;
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, 64);
        if ((tid & 63) == 0) sred[tid >> 6] = f;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < nt / 64; ++w) t += sred[w];
            snorm = sqrt(t);
        }
        __syncthreads();
    }
    // rounding in the rotations leaves off-diagonal noise of about 2^-53 ||T||_F,
    // so the relative test alone cannot terminate when eigenvalues span decades
    const double abs_floor = ldexp(1.0, -51) * snorm;
    int sweeps = 0, converged = 0;
    for (int sw = 0; sw < 40; ++sw) {
        if (tid == 0) rotflag = 0;
        __syncthreads();
        for (int rd = 0; rd < L - 1; ++rd) {
            if (tid < H) {
                // round-robin: players 1..L-1 rotate by rd, player 0 stays
                int xa = tid - 1 + rd, xb = L - 2 - tid + rd;
                if (xa >= L - 1) xa -= L - 1;
                if (xb >= L - 1) xb -= L - 1;
                const int a = tid == 0 ? 0 : 1 + xa;
                const int b = 1 + xb;
                const int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < l) {
                    const double apq = P[pk(p, q, L)];
                    const double app = P[pk(p, p, L)], aqq = P[pk(q, q, L)];
                    if (fabs(apq) > abs_floor && apq * apq > 1e-30 * fabs(app * aqq)) {
                        jacobi_angle(app, aqq, apq, c, s);
                        rotflag = 1;
                    }
                }
                cp[tid] = p;
                cq[tid] = q;
                cc[tid] = c;
                ss[tid] = s;
            }
            __syncthreads();
            // T <- J^T T J, one 2x2 block per (pair a, pair b), a <= b
            for (int e = tid; e < nblk; e += nt) {
                const int ab = blk[e], a = ab & 0xffff, b = ab >> 16;
                const double s1 = ss[a], s2 = ss[b];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const double c1 = cc[a], c2 = cc[b];
                const int p1 = cp[a], q1 = cq[a], p2 = cp[b], q2 = cq[b];
                if (a == b) {
                    const int i00 = pk(p1, p1, L), i01 = pk(p1, q1, L), i11 = pk(q1, q1, L);
                    const double x00 = P[i00], x01 = P[i01], x11 = P[i11];
                    const double y00 = c1 * x00 - s1 * x01, y01 = c1 * x01 - s1 * x11;
                    const double y10 = s1 * x00 + c1 * x01, y11 = s1 * x01 + c1 * x11;
                    P[i00] = y00 * c1 - y01 * s1;
                    P[i01] = y00 * s1 + y01 * c1;
                    P[i11] = y10 * s1 + y11 * c1;
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
            // W <- W J: each thread loads all of its entries before updating them
            {
                constexpr int MI = (kMaxLJ + 31) / 32, MA = (kMaxLJ / 2 + 31) / 32;
                double wpv[MI][MA], wqv[MI][MA];
#pragma unroll
                for (int u = 0; u < MI; ++u)
#pragma unroll
                    for (int v = 0; v < MA; ++v) {
                        const int i = ty + u * TY, a = tx + v * TX;
                        if (i < L && a < H && ss[a] != 0.0) {
                            wpv[u][v] = W[i * L + cp[a]];
                            wqv[u][v] = W[i * L + cq[a]];
                        }
                    }
#pragma unroll
                for (int u = 0; u < MI; ++u)
#pragma unroll
                    for (int v = 0; v < MA; ++v) {
                        const int i = ty + u * TY, a = tx + v * TX;
                        if (i < L && a < H) {
                            const double s = ss[a];
                            if (s != 0.0) {
                                const double c = cc[a];
                                W[i * L + cp[a]] = c * wpv[u][v] - s * wqv[u][v];
                                W[i * L + cq[a]] = s * wpv[u][v] + c * wqv[u][v];
                            }
                        }
                    }
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
    if (w > 128) w = 128;
    if (w < 1) w = 1;
    return (int)w;
}

hipError_t launch_gram64(const float* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                         hipStream_t st) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    const int lp = ((int)l + 3) & ~3;
    const int nt = (lp / 4) * (lp / 4);
    const int64_t rpw = (rows + wgs - 1) / wgs;
    hipLaunchKernelGGL(k_gram64, dim3(wgs), dim3(nt < 64 ? 64 : nt), 0, st, X, rows, (int)l, ldx, rpw, partial);
    return hipGetLastError();
}

hipError_t launch_gram_reduce(const double* partial, int parts, int64_t l, double* T, hipStream_t st) {
    const int64_t ll = l * l;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ll + 63) / 64)), dim3(256), 0, st, partial, parts, ll, T);
    return hipGetLastError();
}

hipError_t launch_chol_rinv_small(const double* partial, int parts, int64_t l, double* Rinv, int* info,
                                  hipStream_t st) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_rinv_small, dim3(1), dim3(256), 0, st, partial, parts, (int)l, Rinv, info);
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

hipError_t launch_jacobi_eigh(const double* partial, int parts, int64_t l, int64_t k, double* lam, double* Wk,
                              double* Wks, int* info, hipStream_t st) {
    if (l < 1 || l > kMaxLJ || k < 1 || k > l) return hipErrorInvalidValue;
    const int L = (int)l + ((int)l & 1);
    const int nt = L <= 32 ? 256 : 1024;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(nt), 0, st, partial, parts, (int)l, (int)k, lam, Wk, Wks, info);
    return hipGetLastError();
}

}  // namespace bcur
