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
constexpr int kRC = 32;        // rows per LDS chunk

// partial[w] = X[rows of w]^T X[rows of w]; thread (ti, tj) owns the 4x4 block
// of entries (4 ti .. 4 ti + 3, 4 tj .. 4 tj + 3).  Products of two floats are
// exact in FP64 and every entry sums its rows in order, so T is symmetric bitwise.
template <typename T>
__global__ __launch_bounds__(1024) void k_gram64(const T* __restrict__ X, int64_t rows, int l, int64_t ldx,
                                                 int64_t rows_per_wg, double* __restrict__ partial,
                                                 const int* __restrict__ gate) {
    __shared__ __attribute__((aligned(16))) T xs[kRC * kMaxL];
    if (gate && *gate == 0) return;
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
            xs[e] = (rr < nr && cc < l) ? X[(rb + rr) * ldx + cc] : (T)0;
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            double vi[4], vj[4];
            if constexpr (sizeof(T) == 4) {
                const float4 xi = *reinterpret_cast<const float4*>(&xs[rr * lp + 4 * ti]);
                const float4 xj = *reinterpret_cast<const float4*>(&xs[rr * lp + 4 * tj]);
                vi[0] = xi.x; vi[1] = xi.y; vi[2] = xi.z; vi[3] = xi.w;
                vj[0] = xj.x; vj[1] = xj.y; vj[2] = xj.z; vj[3] = xj.w;
            } else {
                const double2* pi = reinterpret_cast<const double2*>(&xs[rr * lp + 4 * ti]);
                const double2* pj = reinterpret_cast<const double2*>(&xs[rr * lp + 4 * tj]);
                const double2 i0 = pi[0], i1 = pi[1], j0 = pj[0], j1 = pj[1];
                vi[0] = i0.x; vi[1] = i0.y; vi[2] = i1.x; vi[3] = i1.y;
                vj[0] = j0.x; vj[1] = j0.y; vj[2] = j1.x; vj[3] = j1.y;
            }
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
// partials are split into 8 groups (g = w mod 8), each thread sums one group
// for one entry with 4 loads in flight, and the 8 group sums are added in a
// fixed tree.  The order depends on w only, so T keeps the bitwise symmetry of
// the partials.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial, int parts, int64_t ll,
                                                     double* __restrict__ T, const int* __restrict__ gate) {
    __shared__ double sg[8][32];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, g = tid >> 5, el = tid & 31;
    const int64_t e = (int64_t)blockIdx.x * 32 + el;
    double acc = 0.0;
    if (e < ll) {
        int w = g;
        for (; w + 24 < parts; w += 32) {
            const double v0 = partial[(int64_t)w * ll + e], v1 = partial[(int64_t)(w + 8) * ll + e];
            const double v2 = partial[(int64_t)(w + 16) * ll + e], v3 = partial[(int64_t)(w + 24) * ll + e];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; w < parts; w += 8) acc += partial[(int64_t)w * ll + e];
    }
    sg[g][el] = acc;
    __syncthreads();
    if (g == 0 && e < ll)
        T[e] = ((sg[0][el] + sg[1][el]) + (sg[2][el] + sg[3][el])) + ((sg[4][el] + sg[5][el]) + (sg[6][el] + sg[7][el]));
}

// T + shift I = R^T R for the l x l Gram matrix T (FP64, row-major), with
// shift = l 2^-52 trace(T), and Rinv = R^-1 (upper, l x l, R = L^T).  One
// workgroup of TG x TG threads; the matrix lives in registers (reg_chol_inv),
// l <= TG * NR.  Every entry is loaded and stored by its owning thread.
//
// With `gate` non-null the kernel returns at once when *gate == 0.  With
// `need2` non-null it writes 0 there when one Cholesky QR pass with this
// factor already leaves a basis orthonormal far below FP32 rounding: the
// orthogonality error of a pass is about u64 cond(T), and cond(T) <=
// ||T||_F ||Rinv||_F^2 (lambda_max <= ||T||_F, 1/lambda_min <= ||R^-1||_2^2), so
// a bound below 2^26 (error below 2^-26) suffices; otherwise it writes 1.
template <int TG, int NR>
__global__ __launch_bounds__(TG* TG) void k_chol_rinv_small(const double* __restrict__ T, int l,
                                                            double* __restrict__ Rinv, int* __restrict__ info,
                                                            const int* __restrict__ gate, int* __restrict__ need2) {
    constexpr int NW = TG * TG / 64;
    __shared__ double P[2 * TG * NR + 1];
    __shared__ double pv[TG * NR];
    __shared__ double sred[2][NW];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x, tr = tid / TG, tc = tid % TG;
    double m[NR * (NR + 1) / 2];
    double gf = 0.0;   // this thread's share of ||T||_F^2
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tr + TG * a, c = tc + TG * b;
            const double v = (i < l && c <= i) ? T[(int64_t)i * l + c] : 0.0;
            m[tri_slot(a, b)] = v;
            gf = fma(i == c ? v : 2.0 * v, v, gf);
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
    const bool small_pivot = pmin < 10.0 * shift || ndrop > 0;
    if (tid == 0 && info && small_pivot) atomicOr(info, 1);
    if (need2) {
        double xf = 0.0;
#pragma unroll
        for (int a = 0; a < NR; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                const int i = tr + TG * a, c = tc + TG * b;
                const double v = (i < l && c <= i) ? m[tri_slot(a, b)] : 0.0;
                xf = fma(v, v, xf);
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            gf += __shfl_xor(gf, o, 64);
            xf += __shfl_xor(xf, o, 64);
        }
        if ((tid & 63) == 0) {
            sred[0][tid >> 6] = gf;
            sred[1][tid >> 6] = xf;
        }
        __syncthreads();
        if (tid == 0) {
            double g2 = 0.0, x2 = 0.0;
            for (int w = 0; w < NW; ++w) {
                g2 += sred[0][w];
                x2 += sred[1][w];
            }
            const double bound = sqrt(g2) * x2;
            need2[0] = (small_pivot || !(bound < ldexp(1.0, 26))) ? 1 : 0;
        }
    }
}

// out (rows x lo) = X (rows x li, FP32) * M (li x lo, FP64), FP64 accumulation.
// Thread t owns row t / cg of a chunk of rg = 256 / cg rows and the four
// columns 4 (t % cg) .. + 3, cg = lop / 4 (lop = lo rounded up to 4), so every
// thread has work at any lo; M (li x lop) and the chunk of X sit in LDS sized
// to li (dynamic), which leaves room for several workgroups per compute unit.
// Each output sums its li products in order with FMAs.
__global__ __launch_bounds__(256) void k_apply_small(const float* __restrict__ X, int64_t rows, int li, int64_t ldx,
                                                     const double* __restrict__ M, int lo, int64_t ldm,
                                                     float* __restrict__ out, int64_t ldo,
                                                     const int* __restrict__ gate) {
    extern __shared__ __attribute__((aligned(16))) double apply_lds[];
    if (gate && *gate == 0) return;
    const int lop = (lo + 3) & ~3, cg = lop / 4, rg = 256 / cg;
    double* Ms = apply_lds;
    float* Xs = reinterpret_cast<float*>(apply_lds + li * lop);
    const int tid = threadIdx.x;
    for (int e = tid; e < li * lop; e += 256) {
        const int i = e / lop, o = e - i * lop;
        Ms[e] = o < lo ? M[(int64_t)i * ldm + o] : 0.0;
    }
    const int tr = tid / cg, tc = tid - tr * cg;
    const bool act = tr < rg;
    for (int64_t rb = (int64_t)blockIdx.x * rg; rb < rows; rb += (int64_t)gridDim.x * rg) {
        const int nr = (int)(rows - rb < rg ? rows - rb : rg);
        __syncthreads();
        for (int e = tid; e < rg * li; e += 256) {
            const int rr = e / li, cc = e - rr * li;
            Xs[e] = rr < nr ? X[(rb + rr) * ldx + cc] : 0.0f;
        }
        __syncthreads();
        if (act && tr < nr) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const float* xr = Xs + tr * li;
            const double* mc = Ms + 4 * tc;
            int i = 0;
            for (; i + 4 <= li; i += 4) {
                double xv[4];
                double2 m01[4], m23[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xv[u] = xr[i + u];
                    m01[u] = *reinterpret_cast<const double2*>(mc + (i + u) * lop);
                    m23[u] = *reinterpret_cast<const double2*>(mc + (i + u) * lop + 2);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[0] = fma(xv[u], m01[u].x, acc[0]);
                    acc[1] = fma(xv[u], m01[u].y, acc[1]);
                    acc[2] = fma(xv[u], m23[u].x, acc[2]);
                    acc[3] = fma(xv[u], m23[u].y, acc[3]);
                }
            }
            for (; i < li; ++i) {
                const double xv = xr[i];
                const double2 m01 = *reinterpret_cast<const double2*>(mc + i * lop);
                const double2 m23 = *reinterpret_cast<const double2*>(mc + i * lop + 2);
                acc[0] = fma(xv, m01.x, acc[0]);
                acc[1] = fma(xv, m01.y, acc[1]);
                acc[2] = fma(xv, m23.x, acc[2]);
                acc[3] = fma(xv, m23.y, acc[3]);
            }
            float* orow = out + (rb + tr) * ldo;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (4 * tc + b < lo) orow[4 * tc + b] = (float)acc[b];
        }
    }
}

// The same product for lo > 64: 32-row chunks, each thread a 4 x 4 block of
// outputs (8 x 32 threads: 32 rows x 128 columns), M in a fixed LDS array.
__global__ __launch_bounds__(256) void k_apply_wide(const float* __restrict__ X, int64_t rows, int li, int64_t ldx,
                                                     const double* __restrict__ M, int lo, int64_t ldm,
                                                     float* __restrict__ out, int64_t ldo,
                                                     const int* __restrict__ gate) {
    __shared__ double Ms[kMaxL * kMaxL];
    __shared__ float Xs[kRC * (kMaxL + 1)];
    if (gate && *gate == 0) return;
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

// Cyclic Jacobi eigensolver of the small symmetric Rayleigh-Ritz matrix T,
// in two kernels.
//
// Round-robin schedule: in round rd (0 <= rd < L - 1, L = l rounded up to even)
// pair slot t rotates the index pair (x_t, y_t); the L/2 pairs of a round are
// disjoint and every pair of indices meets exactly once in any L - 1
// consecutive rounds (index 0 stays in slot 0, the others circulate).
//
// k_jacobi_rr (one workgroup) keeps T in slot order: slot t always occupies
// positions (2t, 2t+1).  From one round to the next every index moves to a
// fixed new position (slot_next), so each 2 x 2 block (u, v) of J^T T J is
// read from fixed positions and written to fixed permuted ones in the other
// copy of T (upper triangle only).  Wave 0 owns the diagonal blocks (t, t) and
// one off-diagonal block per slot, which together hold every entry that the
// next round's rotations are computed from: after updating its blocks it
// forms the next round's rotations (lane t for slot t, neighbours' entries by
// lane shuffles) and publishes them while the other waves still update the
// remaining blocks, so a round costs one barrier.  The rotations are recorded
// for k_jacobi_vectors, which forms rows of W = J_1 J_2 ... J_R from the record
// across many workgroups and writes the first k columns in eigenvalue order.
//
// A pair (x, y) is rotated when |a_xy| > 2^-40 ||T||_F and |a_xy| > 1e-15
// sqrt|a_xx a_yy|, from T scaled by 1 / ||T||_F.  The iteration stops once L - 1
// consecutive rounds rotate nothing: then T did not change during them and
// every pair was found below the threshold.  It also stops as soon as every
// off-diagonal entry is at most 2^-40 ||T||_F, which every wave checks on the
// blocks it writes every kJCheck rounds: then no pair can rotate again, so the
// rounds that would follow are identities and the result is the same.  The tangent t is estimated in FP32
// and refined by one Newton step to about 2^-46; c = 1/sqrt(1 + t^2) and s = t c
// are formed in FP64 with a Newton-refined estimate, so every rotation is
// orthogonal to FP64 precision.  The entry left by the slightly inexact angle
// is kept, not forced to zero, so no backward error is introduced.
constexpr int kJSweeps = 40;  // at most kJSweeps (L - 1) rounds
constexpr int kJCheck = 8;    // rounds between the all-entries convergence checks

// Indices (x, y) of pair slot t in round rd: x_0 = 0, x_t = 1 + (t - 1 + rd)
// mod (L - 1), y_t = 1 + (L - 2 - t + rd) mod (L - 1); advanced by one round
// at a time (period L - 1).
struct RRSlot {
    int xa, xb;
    __device__ void init(int t, int L, int rd) {
        xa = (t - 1 + rd) % (L - 1);
        xb = (L - 2 - t + rd) % (L - 1);
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
// Position of index i in the first round.
__device__ __forceinline__ int slot_pos0(int i, int L) { return i < L / 2 ? 2 * i : 2 * (L - 1 - i) + 1; }

// Slot-ordered symmetric L x L matrix (L <= KL) stored as its upper 2 x 2
// blocks (u <= v), four doubles each (x00, x01, x10, x11), packed row by row,
// so a block is read with two 16-byte loads; a diagonal block leaves x10 unused.
// Four more doubles (kTrash) take the stores of lanes without a block.
template <int KL>
struct JStore {
    static constexpr int HB = KL / 2, kTrash = 4 * (HB * (HB + 1) / 2), kSize = kTrash + 4;
    __device__ static int blk(int u, int v) { return u * HB - (u * (u - 1)) / 2 + (v - u); }  // u <= v
    __device__ static int idx(int i, int j) {
        if ((i >> 1) > (j >> 1) || ((i >> 1) == (j >> 1) && i > j)) {
            const int x = i;
            i = j;
            j = x;
        }
        return 4 * blk(i >> 1, j >> 1) + 2 * (i & 1) + (j & 1);
    }
};

// Rotation (c, s) of a slot from its entries; (1, 0) below the threshold.
// Branch-free: below the threshold it runs on stand-in values and is discarded.
__device__ __forceinline__ double2 jacobi_rotation(double xx, double yy, double xy, double inv, double floor_s) {
    const double as0 = xy * inv;
    const bool rotate = fabs(as0) > floor_s && xy * xy > 1e-30 * fabs(xx * yy);
    // scaled entries: |ds|, |as| <= 2 and |as| > 2^-40, so the FP32 estimate cannot overflow
    const double as = rotate ? as0 : 1.0, ds = rotate ? (yy - xx) * inv : 0.0;
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
    const double c = rsqrt_nr(fma(t, t, 1.0));
    return rotate ? make_double2(c, t * c) : make_double2(1.0, 0.0);
}

// J_u^T X J_v of an off-diagonal block x = (x00, x01, x10, x11).
__device__ __forceinline__ void rot_block(const double (&x)[4], double c1, double s1, double c2, double s2,
                                          double (&o)[4]) {
    const double y00 = c1 * x[0] - s1 * x[2], y01 = c1 * x[1] - s1 * x[3];
    const double y10 = s1 * x[0] + c1 * x[2], y11 = s1 * x[1] + c1 * x[3];
    o[0] = y00 * c2 - y01 * s2;
    o[1] = y00 * s2 + y01 * c2;
    o[2] = y10 * c2 - y11 * s2;
    o[3] = y10 * s2 + y11 * c2;
}

// The e-th block (u < v) of those not owned by wave 0: (u, u+1) for 1 <= u <=
// H-3, then (u, v) with v - u >= 3, row by row.  Returns false past the end.
__device__ __forceinline__ bool other_block(int e, int H, int& u, int& v) {
    const int nA = H > 3 ? H - 3 : 0;
    if (e < nA) {
        u = e + 1;
        v = e + 2;
        return true;
    }
    e -= nA;
    if (e >= nA * (nA + 1) / 2) return false;
    // row u holds H - 3 - u blocks and starts at u (H - 3) - u (u - 1) / 2
    u = 0;
    while ((u + 1) * nA - ((u + 1) * u) / 2 <= e) ++u;
    v = u + 3 + (e - (u * nA - (u * (u - 1)) / 2));
    return true;
}

template <int KL, int NT, int NB>
__global__ __launch_bounds__(NT) void k_jacobi_rr(const double* __restrict__ Tin, int l,
                                                  double* __restrict__ lam_out, double2* __restrict__ rot,
                                                  int* __restrict__ meta, int* __restrict__ info,
                                                  const int* __restrict__ gate) {
    using St = JStore<KL>;
    static_assert((KL / 2) * (KL / 2 - 3) / 2 <= (NT - 64) * NB, "too few block slots");
    __shared__ __attribute__((aligned(16))) double Tb[2][St::kSize];
    __shared__ double2 cs[2][64];  // one entry per lane of wave 0; slots >= H are never read
    __shared__ double sred[NT / 64];
    __shared__ int stop[2];
    __shared__ int cflag[2][NT / 64];  // per wave: an entry it wrote is above the floor
    __shared__ int posof[KL];
    if (gate && *gate == 0) return;
    const int tid = threadIdx.x;
    const int L = l + (l & 1), H = L / 2;
    const int Rmax = kJSweeps * (L - 1);
    // slot-ordered upper triangle: entry (i, j) of T at positions (pos0(i), pos0(j))
    {
        constexpr int RS = NT / KL, NU = KL / RS;
        const int jc = tid % KL;
        double tv[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int i = tid / KL + RS * u;
            tv[u] = (i <= jc && jc < l) ? Tin[(int64_t)i * l + jc] : 0.0;
        }
        double f = 0.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int i = tid / KL + RS * u;
            if (i <= jc && jc < L) Tb[0][St::idx(slot_pos0(i, L), slot_pos0(jc, L))] = tv[u];
            if (i <= jc) f += (i == jc ? 1.0 : 2.0) * tv[u] * tv[u];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, 64);
        if ((tid & 63) == 0) sred[tid >> 6] = f;
    }
    __syncthreads();
    double nrm2 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) nrm2 += sred[w];
    const double snorm = sqrt(nrm2);
    const double inv = snorm > 0.0 ? 1.0 / snorm : 0.0;
    const double floor_s = ldexp(1.0, -40);
    int cur = 0, r = 0;
    if (tid < 64) {
        // ---- wave 0: diagonal block t and one off-diagonal block per slot ----
        // Lane t also recomputes, from LDS, the entries of its neighbours'
        // diagonal blocks that slot t's next rotation needs (bitwise the same
        // as the owner's values: same operations, explicit FMAs), so no lane
        // exchange sits on the round's critical path.
        const int t = tid, tt = t < H ? t : 0;
        const bool act_t = t < H;
        const bool has_up = act_t && t + 1 < H, has_dn = act_t && t >= 1;
        // off block feeding slot t's next a_xy: (0, 1) for slot 0, (t-1, t+1)
        // inside, (H-2, H-1) for the last slot; written by its owner only
        // (for H = 2 lane 1 reads the block lane 0 writes)
        const bool has_src = act_t && H >= 2;
        const bool has_off = has_src && (H >= 3 || t == 0);
        const int ou = !has_src || t == 0 ? 0 : (t == H - 1 ? H - 2 : t - 1);
        const int ov = !has_src ? 0 : (t == 0 ? 1 : (t == H - 1 ? H - 1 : t + 1));
        const int a0 = 2 * tt, a1 = 2 * tt + 1;
        const int na0 = slot_next(a0, H), na1 = slot_next(a1, H);
        // lanes without a block store to the spare entries
        const int dw0 = act_t ? St::idx(na0, na0) : St::kTrash, dw1 = act_t ? St::idx(na0, na1) : St::kTrash + 1,
                  dw3 = act_t ? St::idx(na1, na1) : St::kTrash + 2;
        const int tu = has_up ? t + 1 : tt, td = has_dn ? t - 1 : tt;
        // blocks read: own diagonal, the diagonal above and below, the off block
        const int dbk = St::blk(tt, tt), ubk = St::blk(tu, tu), xbk = St::blk(td, td), obk = St::blk(ou, ov);
        int owx[4];
        {
            const int u0 = 2 * ou, u1 = u0 + 1, v0 = 2 * ov, v1 = v0 + 1;
            const int nu0 = slot_next(u0, H), nu1 = slot_next(u1, H), nv0 = slot_next(v0, H),
                      nv1 = slot_next(v1, H);
            owx[0] = has_off ? St::idx(nu0, nv0) : St::kTrash;
            owx[1] = has_off ? St::idx(nu0, nv1) : St::kTrash + 1;
            owx[2] = has_off ? St::idx(nu1, nv0) : St::kTrash + 2;
            owx[3] = has_off ? St::idx(nu1, nv1) : St::kTrash + 3;
        }
        // rotations of round 0
        const double* T = Tb[0];
        double2 cst = act_t ? jacobi_rotation(T[4 * dbk], T[4 * dbk + 3], T[4 * dbk + 1], inv, floor_s)
                            : make_double2(1.0, 0.0);
        cs[0][t] = cst;
        if (act_t) rot[t] = cst;
        bool any = __ballot(cst.y != 0.0) != 0;
        int quiet = any ? 0 : 1, last_active = any ? 1 : 0;
        if (t == 0) stop[0] = quiet >= L - 1;
        bool conv = false;
        __syncthreads();
        for (; r < Rmax && quiet < L - 1 && !conv; ++r) {
            const int p = r & 1, q = p ^ 1;
            // the flags of the round before, when it was a check round
            const bool chk = r > 0 && r % kJCheck == 0;
            int cf = 0;
            if (chk) {
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) cf |= cflag[q][w];
            }
            T = Tb[cur];
            const double2* T2 = reinterpret_cast<const double2*>(T);
            double* Tn = Tb[cur ^ 1];
            const double2 d01 = T2[2 * dbk], u01 = T2[2 * ubk], w01 = T2[2 * xbk];
            const double x3 = T[4 * dbk + 3], u3 = T[4 * ubk + 3], w3 = T[4 * xbk + 3];
            const double2 olo = T2[2 * obk], ohi = T2[2 * obk + 1];
            const double2 csu = cs[p][tu], csd = cs[p][td];
            const double x0 = d01.x, x1 = d01.y, u0 = u01.x, u1 = u01.y, w0 = w01.x, w1 = w01.y;
            const double xo[4] = {olo.x, olo.y, ohi.x, ohi.y};
            // own diagonal block J^T X J, X = (a_xx, a_xy; a_xy, a_yy)
            const double c = cst.x, s = cst.y;
            const double y00 = fma(c, x0, -s * x1), y01 = fma(c, x1, -s * x3);
            const double y10 = fma(s, x0, c * x1), y11 = fma(s, x1, c * x3);
            const double r00 = fma(y00, c, -y01 * s), r01 = fma(y00, s, y01 * c), r11 = fma(y10, s, y11 * c);
            // r00 of the block above, r11 of the block below (the owners' operations)
            const double uy00 = fma(csu.x, u0, -csu.y * u1), uy01 = fma(csu.x, u1, -csu.y * u3);
            const double up00 = fma(uy00, csu.x, -uy01 * csu.y);
            const double wy10 = fma(csd.y, w0, csd.x * w1), wy11 = fma(csd.y, w1, csd.x * w3);
            const double dn11 = fma(wy10, csd.y, wy11 * csd.x);
            double o[4];
            {
                const double2 cu = t == 0 ? cst : csd, cv = t == H - 1 ? cst : csu;
                rot_block(xo, cu.x, cu.y, cv.x, cv.y, o);
            }
            Tn[dw0] = r00;
            Tn[dw1] = r01;
            Tn[dw3] = r11;
#pragma unroll
            for (int e = 0; e < 4; ++e) Tn[owx[e]] = o[e];
            if (r % kJCheck == kJCheck - 1) {
                bool big = act_t && fabs(r01) * inv > floor_s;
#pragma unroll
                for (int e = 0; e < 4; ++e) big = big || (has_off && fabs(o[e]) * inv > floor_s);
                const int f = __ballot(big) != 0;
                if (t == 0) cflag[p][0] = f;
            }
            // entries of slot t in the next round
            double xx, yy, xy;
            if (H == 1) {
                xx = r00;
                yy = r11;
                xy = r01;
            } else if (t == 0) {
                xx = r00;
                yy = up00;
                xy = o[0];
            } else if (t == H - 1) {
                xx = r11;
                yy = dn11;
                xy = o[3];
            } else {
                xx = up00;
                yy = dn11;
                xy = o[2];
            }
            cst = act_t ? jacobi_rotation(xx, yy, xy, inv, floor_s) : make_double2(1.0, 0.0);
            cs[q][t] = cst;
            any = __ballot(cst.y != 0.0) != 0;
            quiet = any ? 0 : quiet + 1;
            if (r + 1 < Rmax) {
                if (act_t) rot[(int64_t)(r + 1) * H + t] = cst;
                if (any) last_active = r + 2;
            }
            conv = chk && cf == 0;
            if (t == 0) stop[q] = quiet >= L - 1 || conv;
            cur ^= 1;
            __syncthreads();
        }
        if (t == 0) {
            meta[0] = last_active;
            if (info) {
                info[0] = (r + L - 2) / (L - 1);
                info[1] = r < Rmax;
            }
        }
        // positions of the indices in round r
        if (act_t) {
            RRSlot sl;
            sl.init(t, L, r % (L - 1));
            int x, y;
            sl.pair(t, x, y);
            posof[x] = 2 * t;
            posof[y] = 2 * t + 1;
        }
    } else {
        // ---- waves 1..: the remaining off-diagonal blocks ----
        int buv[NB], rbk[NB], wrx[NB][4];
        bool bok[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int u = 0, v = 1;
            bok[b] = other_block(tid - 64 + (NT - 64) * b, H, u, v);
            buv[b] = u | (v << 8);
            const int a0 = 2 * u, a1 = 2 * u + 1, b0 = 2 * v, b1 = 2 * v + 1;
            rbk[b] = St::blk(u, v);
            const int na0 = slot_next(a0, H), na1 = slot_next(a1, H), nb0 = slot_next(b0, H),
                      nb1 = slot_next(b1, H);
            wrx[b][0] = St::idx(na0, nb0);
            wrx[b][1] = St::idx(na0, nb1);
            wrx[b][2] = St::idx(na1, nb0);
            wrx[b][3] = St::idx(na1, nb1);
        }
        __syncthreads();
        for (; r < Rmax; ++r) {
            const int p = r & 1;
            const double2* T2 = reinterpret_cast<const double2*>(Tb[cur]);
            double* Tn = Tb[cur ^ 1];
            // the loads are issued before the stop test (all indices are in range)
            const int halt = stop[p];
            double x[NB][4];
            double2 ru[NB], rv[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (!bok[b]) continue;
                const double2 lo = T2[2 * rbk[b]], hi = T2[2 * rbk[b] + 1];
                x[b][0] = lo.x;
                x[b][1] = lo.y;
                x[b][2] = hi.x;
                x[b][3] = hi.y;
                ru[b] = cs[p][buv[b] & 0xff];
                rv[b] = cs[p][buv[b] >> 8];
            }
            if (halt) break;
            bool big = false;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (!bok[b]) continue;
                double o[4];
                rot_block(x[b], ru[b].x, ru[b].y, rv[b].x, rv[b].y, o);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Tn[wrx[b][e]] = o[e];
                    big = big || fabs(o[e]) * inv > floor_s;
                }
            }
            if (r % kJCheck == kJCheck - 1) {
                const int f = __ballot(big) != 0;
                if ((tid & 63) == 0) cflag[p][tid >> 6] = f;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
    __syncthreads();
    // eigenvalues descending (ties by index)
    const double* T = Tb[cur];
    if (tid < l) {
        const int pi = posof[tid];
        const double li = T[St::idx(pi, pi)];
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const int pj = posof[j];
            const double lj = T[St::idx(pj, pj)];
            rank += (lj > li) || (lj == li && j < tid);
        }
        lam_out[rank] = li;
        meta[1 + tid] = rank;
    }
}

// Rows of W from the recorded rotations: one wave applies them to RPW rows at
// once (lane t of each row applies slot t), then Wk[i][rank] = W[i][col] for
// the k leading eigenvalues and Wks = Wk diag(1/sqrt(lam)).  Rotations are
// staged 16 rounds at a time in registers.
template <int KL>
__global__ __launch_bounds__(64) void k_jacobi_vectors(const double2* __restrict__ rot, const int* __restrict__ meta,
                                                       const double* __restrict__ lam, int l, int k,
                                                       double* __restrict__ Wk, double* __restrict__ Wks,
                                                       const int* __restrict__ gate) {
    constexpr int HW = KL / 2, RPW = 64 / HW, CH = 16;
    __shared__ double row[RPW][KL];
    if (gate && *gate == 0) return;
    const int lane = threadIdx.x, t = lane % HW, half = lane / HW;
    const int i = RPW * blockIdx.x + half;
    const int L = l + (l & 1), H = L / 2;
    const int R = meta[0];
    row[half][t] = (t == i) ? 1.0 : 0.0;
    row[half][t + HW] = (t + HW == i) ? 1.0 : 0.0;
    __syncthreads();
    const int tt = t < H ? t : 0;
    RRSlot st;
    st.init(tt, L, 0);
    double* w = row[half];
    for (int r0 = 0; r0 < R; r0 += CH) {
        double2 c[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            c[u] = (r0 + u < R && t < H) ? rot[(int64_t)(r0 + u) * H + t] : make_double2(1.0, 0.0);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (r0 + u < R) {
                int x, y;
                st.pair(tt, x, y);
                if (c[u].y != 0.0) {
                    const double wx = w[x], wy = w[y];
                    w[x] = c[u].x * wx - c[u].y * wy;
                    w[y] = c[u].y * wx + c[u].x * wy;
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
            const int col = t + HW * e;
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
    // one 32-row chunk per workgroup up to 128 workgroups (latency-bound: a
    // longer chunk loop costs more than the larger partial sum)
    int64_t w = rows / 32;
    if (w > 128) w = 128;
    if (w < 1) w = 1;
    return (int)w;
}

template <typename T>
static hipError_t gram64_impl(const T* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                              hipStream_t st, const int* gate) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    const int lp = ((int)l + 3) & ~3;
    const int nt = (lp / 4) * (lp / 4);
    const int64_t rpw = (rows + wgs - 1) / wgs;
    hipLaunchKernelGGL(k_gram64<T>, dim3(wgs), dim3(nt < 64 ? 64 : nt), 0, st, X, rows, (int)l, ldx, rpw, partial,
                       gate);
    return hipGetLastError();
}

hipError_t launch_gram64(const float* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                         hipStream_t st, const int* gate) {
    return gram64_impl(X, rows, l, ldx, partial, wgs, st, gate);
}

hipError_t launch_gram64(const double* X, int64_t rows, int64_t l, int64_t ldx, double* partial, int wgs,
                         hipStream_t st) {
    return gram64_impl(X, rows, l, ldx, partial, wgs, st, nullptr);
}

hipError_t launch_gram_reduce(const double* partial, int parts, int64_t l, double* T, hipStream_t st,
                              const int* gate) {
    const int64_t ll = l * l;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ll + 31) / 32)), dim3(256), 0, st, partial, parts, ll, T,
                       gate);
    return hipGetLastError();
}

hipError_t launch_chol_rinv_small(const double* T, int64_t l, double* Rinv, int* info, hipStream_t st,
                                  const int* gate, int* need2) {
    if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
    // a step is latency-bound: up to l = 64 a 16 x 16 grid with 4 x 4 slots per
    // thread measured fastest (vs one wave with 8 x 8 slots); above, 16 x 16 with
    // 8 x 8 (74 us at l = 128, against 93 us for 32 x 32 with 4 x 4)
    if (l <= 64)
        hipLaunchKernelGGL((k_chol_rinv_small<16, 4>), dim3(1), dim3(256), 0, st, T, (int)l, Rinv, info, gate,
                           need2);
    else
        hipLaunchKernelGGL((k_chol_rinv_small<16, 8>), dim3(1), dim3(256), 0, st, T, (int)l, Rinv, info, gate,
                           need2);
    return hipGetLastError();
}

hipError_t launch_apply_small(const float* X, int64_t rows, int64_t li, int64_t ldx, const double* M, int64_t lo,
                              int64_t ldm, float* out, int64_t ldo, hipStream_t st, const int* gate) {
    if (li < 1 || li > kMaxL || lo < 1 || lo > kMaxL) return hipErrorInvalidValue;
    if (lo > 64) {
        int64_t wblocks = (rows + kRC - 1) / kRC;
        if (wblocks > 1024) wblocks = 1024;
        if (wblocks < 1) wblocks = 1;
        hipLaunchKernelGGL(k_apply_wide, dim3((unsigned)wblocks), dim3(256), 0, st, X, rows, (int)li, ldx, M,
                           (int)lo, ldm, out, ldo, gate);
        return hipGetLastError();
    }
    const int64_t lop = (lo + 3) & ~3, rg = 256 / (lop / 4);
    int64_t blocks = (rows + rg - 1) / rg;
    // every workgroup loads all of M: at most 16 MB of such loads in all (at least
    // 128 workgroups), so a large M is shared by several chunks of rows
    const int64_t cap = std::max<int64_t>(128, ((int64_t)16 << 20) / (li * lop * (int64_t)sizeof(double)));
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    // M (li x lop doubles), then the X chunk (rg x li floats)
    const size_t lds = (size_t)li * lop * sizeof(double) + (size_t)rg * li * sizeof(float);
    hipLaunchKernelGGL(k_apply_small, dim3((unsigned)blocks), dim3(256), lds, st, X, rows, (int)li, ldx, M, (int)lo,
                       ldm, out, ldo, gate);
    return hipGetLastError();
}

size_t jacobi_ws_bytes(int64_t l) {
    const int64_t L = l + (l & 1), H = L / 2;
    return (size_t)kJSweeps * (size_t)(L - 1) * (size_t)H * sizeof(double2) + (size_t)(l + 1) * sizeof(int) + 256;
}

hipError_t launch_jacobi_eigh(const double* T, int64_t l, int64_t k, double* lam, double* Wk, double* Wks, void* ws,
                              int* info, hipStream_t st, const int* gate) {
    if (l < 1 || l > kMaxL || k < 1 || k > l) return hipErrorInvalidValue;
    const int L = (int)l + ((int)l & 1);
    const int64_t H = L / 2;
    double2* rot = reinterpret_cast<double2*>(ws);
    int* meta = reinterpret_cast<int*>(rot + (int64_t)kJSweeps * (L - 1) * H);
    if (L <= 64) {
        hipLaunchKernelGGL((k_jacobi_rr<64, 512, 2>), dim3(1), dim3(512), 0, st, T, (int)l, lam, rot, meta, info,
                           gate);
        hipLaunchKernelGGL(k_jacobi_vectors<64>, dim3((unsigned)((l + 1) / 2)), dim3(64), 0, st,
                           (const double2*)rot, (const int*)meta, (const double*)lam, (int)l, (int)k, Wk, Wks, gate);
    } else {
        hipLaunchKernelGGL((k_jacobi_rr<128, 1024, 3>), dim3(1), dim3(1024), 0, st, T, (int)l, lam, rot, meta, info,
                           gate);
        hipLaunchKernelGGL(k_jacobi_vectors<128>, dim3((unsigned)l), dim3(64), 0, st, (const double2*)rot,
                           (const int*)meta, (const double*)lam, (int)l, (int)k, Wk, Wks, gate);
    }
    return hipGetLastError();
}

}  // namespace bcur
