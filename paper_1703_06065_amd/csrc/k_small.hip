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

// T + shift I = R^T R for the l x l Gram matrix T (FP64, row-major), with
// shift = l 2^-52 trace(T), and Rinv = R^-1 (upper, l x l, R = L^T).  One
// workgroup of TG x TG threads; the matrix lives in registers (reg_chol_inv),
// l <= TG * NR.  Every entry is loaded and stored by its owning thread.
template <int TG, int NR>
__global__ __launch_bounds__(TG* TG) void k_chol_rinv_small(const double* __restrict__ T, int l,
                                                            double* __restrict__ Rinv, int* __restrict__ info) {
    __shared__ double P[2 * TG * NR + 1];
    __shared__ double pv[TG * NR];
    const int tid = threadIdx.x, tr = tid / TG, tc = tid % TG;
    double m[NR * (NR + 1) / 2];
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tr + TG * a, c = tc + TG * b;
            m[tri_slot(a, b)] = (i < l && c <= i) ? T[(int64_t)i * l + c] : 0.0;
        }
    // trace, summed in index order by every thread
#pragma unroll
    for (int a = 0; a < NR; ++a)
        if (tr == tc && tr + TG * a < l) pv[tr + TG * a] = m[tri_slot(a, a)];
    __syncthreads();
    double tr4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < l; ++i) tr4[i & 3] += pv[i];
    double shift = (double)l * ldexp(1.0, -52) * ((tr4[0] + tr4[1]) + (tr4[2] + tr4[3]));
    if (!(shift > 0.0)) shift = 1e-300;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NR; ++a)
        if (tr == tc && tr + TG * a < l) m[tri_slot(a, a)] += shift;
    double pmin, pmax;
    int ndrop;
    reg_chol_inv<TG, NR>(m, l, 0.0, P, pv, pmin, pmax, ndrop);
    // Rinv = X^T: Rinv[c][i] = X[i][c] for i >= c; the owner of (i, c) also
    // writes the zero at (i, c) below the diagonal
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tr + TG * a, c = tc + TG * b;
            if (i < l && c <= i) {
                Rinv[(int64_t)c * l + i] = m[tri_slot(a, b)];
                if (c < i) Rinv[(int64_t)i * l + c] = 0.0;
            }
        }
    if (tid == 0 && info && (pmin < 10.0 * shift || ndrop > 0)) atomicOr(info, 1);
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

// Full-precision 1/x for x != 0 from the hardware estimate and two Newton
// steps (the rotations need c^2 + s^2 = 1 to working precision, not correctly
// rounded operations; rsqrt_nr is its square-root counterpart).
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
// The tangent t of each rotation is estimated in FP32 (hardware reciprocal and
// square root) and refined by one Newton step to about 2^-46; c = 1/sqrt(1 +
// t^2) and s = t c are then formed in FP64 with Newton-refined estimates, so
// every rotation is orthogonal to FP64 precision.  The (p, q) entry left by
// the slightly inexact angle is kept (not forced to zero), so no backward
// error is introduced; later rounds remove it.
__device__ __forceinline__ void jacobi_angle(double app, double aqq, double apq, double& c, double& s) {
    const double d = aqq - app;
    double t;
    if (fabs(apq) < 1e-30 * fabs(d)) {
        t = apq * rcp_nr(d);                       // |tau| > 1e30: t = 1 / (2 tau)
    } else {
        // scale both by one power of two so the FP32 conversion cannot overflow
        int e;
        frexp(fmax(fabs(d), fabs(apq)), &e);
        const double ds = ldexp(d, -e), as = ldexp(apq, -e);
        const float df = (float)ds, af = (float)as;
        const float tau = df * __builtin_amdgcn_rcpf(2.0f * af);
        const float at = fabsf(tau);
        float tf = __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.0f)));
        if (tau < 0.0f) tf = -tf;
        // t is the root of smaller magnitude of  as t^2 + ds t - as = 0; one
        // Newton step from the FP32 estimate (residual in FP64, the small
        // correction's quotient in FP32) brings it to about 2^-46
        const double t0 = (double)tf;
        const double fv = fma(as * t0, t0, fma(ds, t0, -as));
        const double fd = fma(2.0 * as, t0, ds);
        t = t0 - (double)((float)fv * __builtin_amdgcn_rcpf((float)fd));
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


// Round-robin schedule: in round rd (0 <= rd < L - 1) pair slot t rotates the
// index pair (p, q), p < q; the L/2 pairs of a round are disjoint and every
// pair of indices meets exactly once per sweep.  Index 0 stays put, 1 .. L-1
// circulate.
__device__ __forceinline__ void rr_pair(int t, int rd, int L, int& p, int& q) {
    int xa = t - 1 + rd, xb = L - 2 - t + rd;
    if (xa >= L - 1) xa -= L - 1;
    if (xb >= L - 1) xb -= L - 1;
    const int x = t == 0 ? 0 : 1 + xa, y = 1 + xb;
    p = x < y ? x : y;
    q = x < y ? y : x;
}


// The same cyclic Jacobi for L <= 64, split in two kernels.
//
// k_jacobi64 (one workgroup) diagonalizes T kept in slot order: pair slot t
// of the round-robin schedule always occupies positions (2t, 2t+1), holding
// its top and bottom index (x_t, y_t).  From one round to the next every
// index moves to a fixed new position (slot_next), the same in every round,
// so each 2 x 2 block (u, v) of J^T T J is read from fixed positions and
// written to fixed permuted ones in the other copy of T (only the upper
// triangle is stored).  Wave 0 computes the rotations, lane t for slot t, and
// records them; after one barrier every thread applies them to its blocks.
// k_jacobi_vectors then forms rows of W = J_1 J_2 ... J_R from the record,
// two rows per wave across many workgroups, and writes the first k columns in
// eigenvalue order.
//
// The rotation of slot (x, y) is taken from T scaled by 1 / ||T||_F: it is
// made when |a_xy| > 2^-40 ||T||_F and |a_xy| > 1e-15 sqrt|a_xx a_yy|.  The
// tangent t is estimated in FP32 and refined by one Newton step to about
// 2^-46; c = 1/sqrt(1 + t^2) and s = t c are formed in FP64 with
// Newton-refined estimates, so every rotation is orthogonal to FP64 precision.
constexpr int kJ64 = 64, kJ64LD = 65, kJSweeps = 40;

// Indices (x, y) of pair slot t in round rd: index 0 stays in slot 0, the
// others circulate (x_t = 1 + (t - 1 + rd) mod (L - 1), y_t = 1 + (L - 2 - t +
// rd) mod (L - 1)); advanced by one per round (period L - 1).
struct RRSlot {
    int xa, xb;
    __device__ void init(int t, int L) {
        xa = t - 1;
        xb = L - 2 - t;
        if (xa < 0) xa += L - 1;
    }
    __device__ void pair(int t, int& x, int& y) const {
        x = t == 0 ? 0 : 1 + xa;
        y = 1 + xb;
    }
    __device__ void next(int L) {
        xa = xa + 1 == L - 1 ? 0 : xa + 1;
        xb = xb + 1 == L - 1 ? 0 : xb + 1;
    }
};

// Position, in the next round, of what sits at position `pos` now.
__device__ __forceinline__ int slot_next(int pos, int H) {
    if (H == 1 || pos == 0) return pos;
    if (pos == 2) return 1;
    if ((pos & 1) == 0) return pos - 2;
    return pos == 2 * H - 1 ? 2 * H - 2 : pos + 2;
}
// Position of index i in the first round of a sweep.
__device__ __forceinline__ int slot_pos0(int i, int L) { return i < L / 2 ? 2 * i : 2 * (L - 1 - i) + 1; }
__device__ __forceinline__ int up_idx(int i, int j) { return i <= j ? i * kJ64LD + j : j * kJ64LD + i; }

// Rotation from the scaled entries (|ds|, |as| <= 2, |as| > 2^-40).
__device__ __forceinline__ void jacobi_rotation_scaled(double ds, double as, double& c, double& s) {
    const float df = (float)ds, af = (float)as;
    const float tau = df * __builtin_amdgcn_rcpf(2.0f * af);
    const float at = fabsf(tau);
    float tf = __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.0f)));
    if (tau < 0.0f) tf = -tf;
    // t is the root of smaller magnitude of  as t^2 + ds t - as = 0
    const double t0 = (double)tf;
    const double fv = fma(as * t0, t0, fma(ds, t0, -as));
    const double fd = fma(2.0 * as, t0, ds);
    const double t = t0 - (double)((float)fv * __builtin_amdgcn_rcpf((float)fd));
    c = rsqrt_nr(fma(t, t, 1.0));
    s = t * c;
}

__global__ __launch_bounds__(512) void k_jacobi64(const double* __restrict__ Tin, int l, double* __restrict__ lam_out,
                                                  double2* __restrict__ rot, int* __restrict__ meta,
                                                  int* __restrict__ info) {
    __shared__ double Tb[2][kJ64 * kJ64LD];
    __shared__ double2 cs[kJ64 / 2];
    __shared__ double sred[8];
    __shared__ int flag[2];
    constexpr int NT = 512, NB = 2;  // blocks per thread: e = tid + NT r
    const int tid = threadIdx.x;
    const int L = l + (l & 1), H = L / 2, nblk = H * (H + 1) / 2;
    // slot-ordered upper triangle: entry (i, j) of T at positions (pos0(i), pos0(j))
    const int jc = tid & 63;
    double tv[kJ64 / 8];
#pragma unroll
    for (int u = 0; u < kJ64 / 8; ++u) {
        const int i = (tid >> 6) + 8 * u;
        tv[u] = (i <= jc && jc < l) ? Tin[(int64_t)i * l + jc] : 0.0;
    }
    double f = 0.0;
#pragma unroll
    for (int u = 0; u < kJ64 / 8; ++u) {
        const int i = (tid >> 6) + 8 * u;
        if (i <= jc && jc < L) Tb[0][up_idx(slot_pos0(i, L), slot_pos0(jc, L))] = tv[u];
        if (i <= jc) f += (i == jc ? 1.0 : 2.0) * tv[u] * tv[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, 64);
    if ((tid & 63) == 0) sred[tid >> 6] = f;
    if (tid < 2) flag[tid] = 0;
    // this thread's blocks (u <= v) of the packed list, row u starting at u H - u (u - 1) / 2,
    // with their fixed read and write positions
    int buv[NB], rdx[NB][4], wrx[NB][4];
    bool bok[NB], bdiag[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int e = tid + NT * r;
        bok[r] = e < nblk;
        int u = 0;
        while (bok[r] && (u + 1) * H - ((u + 1) * u) / 2 <= e) ++u;
        const int v = bok[r] ? u + (e - (u * H - (u * (u - 1)) / 2)) : 0;
        bdiag[r] = u == v;
        buv[r] = u | (v << 8);
        // entries (a0 b0, a0 b1, a1 b0, a1 b1); on the diagonal a1 b0 is a0 b1
        const int a0 = 2 * u, a1 = 2 * u + 1, b0 = 2 * v, b1 = 2 * v + 1;
        rdx[r][0] = up_idx(a0, b0);
        rdx[r][1] = up_idx(a0, b1);
        rdx[r][2] = up_idx(a1, b0);
        rdx[r][3] = up_idx(a1, b1);
        const int na0 = slot_next(a0, H), na1 = slot_next(a1, H), nb0 = slot_next(b0, H), nb1 = slot_next(b1, H);
        wrx[r][0] = up_idx(na0, nb0);
        wrx[r][1] = up_idx(na0, nb1);
        wrx[r][2] = up_idx(na1, nb0);
        wrx[r][3] = up_idx(na1, nb1);
    }
    __syncthreads();
    const double snorm = sqrt(((sred[0] + sred[1]) + (sred[2] + sred[3])) + ((sred[4] + sred[5]) + (sred[6] + sred[7])));
    const double inv = snorm > 0.0 ? 1.0 / snorm : 0.0;
    const double floor_s = ldexp(1.0, -40);
    const int t = tid;  // wave 0: lane t computes slot t
    int cur = 0, R = 0, sweeps = 0, converged = 0;
    for (int sw = 0; sw < kJSweeps; ++sw) {
        if (tid == 0) flag[sw & 1] = 0;
        for (int rd = 0; rd < L - 1; ++rd, ++R) {
            const double* T = Tb[cur];
            double* Tn = Tb[cur ^ 1];
            double x[NB][4];
#pragma unroll
            for (int r = 0; r < NB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) x[r][e] = T[rdx[r][e]];
            if (tid < 64) {
                double c = 1.0, s = 0.0;
                if (t < H) {
                    const double axx = T[(2 * t) * kJ64LD + 2 * t], ayy = T[(2 * t + 1) * kJ64LD + 2 * t + 1];
                    const double axy = T[(2 * t) * kJ64LD + 2 * t + 1];
                    const double as = axy * inv;
                    if (fabs(as) > floor_s && axy * axy > 1e-30 * fabs(axx * ayy))
                        jacobi_rotation_scaled((ayy - axx) * inv, as, c, s);
                    cs[t] = make_double2(c, s);
                    rot[(int64_t)R * H + t] = make_double2(c, s);
                }
                if (__ballot(s != 0.0) != 0 && tid == 0) flag[sw & 1] = 1;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                if (!bok[r]) continue;
                const double2 ru = cs[buv[r] & 0xff], rv = cs[buv[r] >> 8];
                const double c1 = ru.x, s1 = ru.y, c2 = rv.x, s2 = rv.y;
                if (bdiag[r]) {
                    // x = (a_xx, a_xy, a_xy, a_yy) of one slot
                    const double y00 = c1 * x[r][0] - s1 * x[r][1], y01 = c1 * x[r][1] - s1 * x[r][3];
                    const double y10 = s1 * x[r][0] + c1 * x[r][1], y11 = s1 * x[r][1] + c1 * x[r][3];
                    Tn[wrx[r][0]] = y00 * c1 - y01 * s1;
                    Tn[wrx[r][1]] = y00 * s1 + y01 * c1;
                    Tn[wrx[r][3]] = y10 * s1 + y11 * c1;
                } else {
                    const double y00 = c1 * x[r][0] - s1 * x[r][2], y01 = c1 * x[r][1] - s1 * x[r][3];
                    const double y10 = s1 * x[r][0] + c1 * x[r][2], y11 = s1 * x[r][1] + c1 * x[r][3];
                    Tn[wrx[r][0]] = y00 * c2 - y01 * s2;
                    Tn[wrx[r][1]] = y00 * s2 + y01 * c2;
                    Tn[wrx[r][2]] = y10 * c2 - y11 * s2;
                    Tn[wrx[r][3]] = y10 * s2 + y11 * c2;
                }
            }
            cur ^= 1;
            __syncthreads();
        }
        ++sweeps;
        if (!flag[sw & 1]) {
            converged = 1;
            break;
        }
    }
    // eigenvalues descending (ties by index); after whole sweeps index i is at slot_pos0(i)
    const double* T = Tb[cur];
    if (tid < l) {
        const int pi = slot_pos0(tid, L);
        const double li = T[pi * kJ64LD + pi];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const int pj = slot_pos0(j, L);
            const double lj = T[pj * kJ64LD + pj];
            rank += (lj > li) || (lj == li && j < tid);
        }
        lam_out[rank] = li;
        meta[1 + tid] = rank;
    }
    if (tid == 0) {
        meta[0] = converged ? R - (L - 1) : R;  // a converged last sweep rotated nothing
        if (info) {
            info[0] = sweeps;
            info[1] = converged;
        }
    }
}

// Rows 2 blockIdx.x + half of W from the recorded rotations (one wave; lane
// t of each half applies pair t), then Wk[i][rank] = W[i][col] for the k
// leading eigenvalues and Wks = Wk diag(1/sqrt(lam)).  Rotations are staged
// 16 rounds at a time in registers.
__global__ __launch_bounds__(64) void k_jacobi_vectors(const double2* __restrict__ rot, const int* __restrict__ meta,
                                                       const double* __restrict__ lam, int l, int k,
                                                       double* __restrict__ Wk, double* __restrict__ Wks) {
    __shared__ double row[2][kJ64];
    constexpr int CH = 16;
    const int lane = threadIdx.x, t = lane & 31, half = lane >> 5;
    const int i = 2 * blockIdx.x + half;
    const int L = l + (l & 1), H = L / 2;
    const int R = meta[0];
    row[half][t] = (t == i) ? 1.0 : 0.0;
    row[half][t + 32] = (t + 32 == i) ? 1.0 : 0.0;
    __syncthreads();
    const int tt = t < H ? t : 0;
    RRSlot st;
    st.init(tt, L);
    double* w = row[half];
    for (int r0 = 0; r0 < R; r0 += CH) {
        double2 cs[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            cs[u] = (r0 + u < R && t < H) ? rot[(int64_t)(r0 + u) * H + t] : make_double2(1.0, 0.0);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (r0 + u < R) {
                int x, y;
                st.pair(tt, x, y);
                if (cs[u].y != 0.0) {
                    const double wx = w[x], wy = w[y];
                    w[x] = cs[u].x * wx - cs[u].y * wy;
                    w[y] = cs[u].y * wx + cs[u].x * wy;
                }
                st.next(L);
            }
            // the next round's pairs read what this round wrote (in-order LDS within the wave)
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    if (i < l) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int col = t + 32 * e;
            if (col < l) {
                const int rank = meta[1 + col];
                if (rank < k) {
                    const double lv = lam[rank];
                    const double v = w[col];
                    Wk[(int64_t)i * k + rank] = v;
                    if (Wks) Wks[(int64_t)i * k + rank] = v * (lv > 0.0 ? 1.0 / sqrt(lv) : 0.0);
                }
            }
        }
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

hipError_t launch_chol_rinv_small(const double* T, int64_t l, double* Rinv, int* info, hipStream_t st) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    // one wave up to l = 64 (a step is latency-bound: fewer waves, cheaper barrier), four above
    if (l <= 64)
        hipLaunchKernelGGL((k_chol_rinv_small<8, 8>), dim3(1), dim3(64), 0, st, T, (int)l, Rinv, info);
    else
        hipLaunchKernelGGL((k_chol_rinv_small<16, 8>), dim3(1), dim3(256), 0, st, T, (int)l, Rinv, info);
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

size_t jacobi_ws_bytes(int64_t l) {
    const int64_t L = l + (l & 1), H = L / 2;
    return (size_t)kJSweeps * (size_t)(L - 1) * (size_t)H * sizeof(double2) + (size_t)(l + 1) * sizeof(int) + 256;
}

hipError_t launch_jacobi_eigh(const double* T, int64_t l, int64_t k, double* lam, double* Wk, double* Wks, void* ws,
                              int* info, hipStream_t st) {
    if (l < 1 || l > kMaxLJ || k < 1 || k > l) return hipErrorInvalidValue;
    const int L = (int)l + ((int)l & 1);
    if (L <= kJ64) {
        double2* rot = reinterpret_cast<double2*>(ws);
        const int64_t H = L / 2;
        int* meta = reinterpret_cast<int*>(rot + (int64_t)kJSweeps * (L - 1) * H);
        hipLaunchKernelGGL(k_jacobi64, dim3(1), dim3(512), 0, st, T, (int)l, lam, rot, meta, info);
        hipLaunchKernelGGL(k_jacobi_vectors, dim3((unsigned)((l + 1) / 2)), dim3(64), 0, st, (const double2*)rot,
                           (const int*)meta, (const double*)lam, (int)l, (int)k, Wk, Wks);
    } else {
        hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, st, T, 1, (int)l, (int)k, lam, Wk, Wks, info);
    }
    return hipGetLastError();
}

}  // namespace bcur
