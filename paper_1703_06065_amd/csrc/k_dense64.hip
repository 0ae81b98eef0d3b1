// FP64 dense kernels for the c x c normal-equation matrix G = C^T C of the
// fit: a tiled FP64 GEMM on the FP64 matrix cores, and G^-1 by a blocked right-looking Cholesky
// (64-wide panels factored in LDS), a blocked triangular inverse computed
// recursively (both halves, then the coupling block, one level of the
// recursion per pair of launches), and Ginv = L^-T L^-1.
#include <math.h>

#include "bcur_internal.h"
#include "lds_linalg.h"

namespace bcur {
namespace {

constexpr int NB = 64;   // panel width and GEMM tile
constexpr int KB = 16;   // GEMM k step
constexpr int kFullChol = 256;   // largest c factored by one workgroup

typedef double d4v __attribute__((ext_vector_type(4)));

// One 64 x 64 FP64 tile product per workgroup of 256 threads: acc += op(A)[0:M,
// 0:K] op(B)[0:K, 0:N] (A, B point at the tile's origin), staged through LDS
// 16 k at a time.  On the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; register v of the result
// is D[4 v + l / 16][l % 16]), each wave a 32 x 32 quarter as 2 x 2 MFMA tiles.
// Element e = 4 (2 i + j) + v of a thread's 16 is at tile_row(e), tile_col(e).
struct FTile {
    d4v t[2][2];
};
__device__ __forceinline__ int tile_row(int e) {
    const int lane = threadIdx.x & 63, wy = (threadIdx.x >> 6) >> 1;
    return 32 * wy + 16 * (e >> 3) + 4 * (e & 3) + (lane >> 4);
}
__device__ __forceinline__ int tile_col(int e) {
    const int lane = threadIdx.x & 63, wx = (threadIdx.x >> 6) & 1;
    return 32 * wx + 16 * ((e >> 2) & 1) + (lane & 15);
}
__device__ __forceinline__ double tile_get(const FTile& a, int e) { return a.t[e >> 3][(e >> 2) & 1][e & 3]; }

template <bool TA, bool TB, typename TAe = double, typename TBe = double>
__device__ __forceinline__ void tile_mm(FTile& acc, const TAe* __restrict__ A, int64_t lda,
                                        const TBe* __restrict__ B, int64_t ldb, int64_t M, int64_t N, int64_t K,
                                        double* As, double* Bs) {
    const int tid = threadIdx.x, lane = tid & 63, wy = (tid >> 6) >> 1, wx = (tid >> 6) & 1;
    constexpr int EPT = NB * KB / 256;  // elements of each operand a thread stages per step
    for (int64_t k0 = 0; k0 < K; k0 += KB) {
        // all of a step's global reads first (issued together), then the LDS stores
        double va[EPT], vb[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u;
            int row, kk;
            if (!TA) {
                row = e / KB;
                kk = e % KB;
            } else {
                kk = e / NB;
                row = e % NB;
            }
            const int64_t gk = k0 + kk;
            va[u] = (row < M && gk < K) ? (double)(TA ? A[gk * lda + row] : A[row * lda + gk]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u;
            int col, kk;
            if (!TB) {
                kk = e / NB;
                col = e % NB;
            } else {
                col = e / KB;
                kk = e % KB;
            }
            const int64_t gk = k0 + kk;
            vb[u] = (col < N && gk < K) ? (double)(TB ? B[col * ldb + gk] : B[gk * ldb + col]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u;
            const int row = !TA ? e / KB : e % NB, kk = !TA ? e % KB : e / NB;
            As[kk * (NB + 1) + row] = va[u];
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + 256 * u;
            const int col = !TB ? e % NB : e / KB, kk = !TB ? e / NB : e % KB;
            Bs[kk * (NB + 1) + col] = vb[u];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            const int kr = (kk + (lane >> 4)) * (NB + 1);
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr + 32 * wy + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kr + 32 * wx + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc.t[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.t[i][j], 0, 0, 0);
        }
    }
}

// D = alpha op(A) op(B) + beta D in FP64; A and B may be FP32 (products of
// two FP32 values are exact in FP64) or FP64.
template <bool TA, bool TB, typename TAe, typename TBe>
__global__ __launch_bounds__(256) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                               const TAe* __restrict__ A, int64_t lda,
                                               const TBe* __restrict__ B, int64_t ldb, double beta,
                                               double* D, int64_t ldd) {
    __shared__ double As[KB * (NB + 1)], Bs[KB * (NB + 1)];
    const int64_t m0 = (int64_t)blockIdx.x * NB, n0 = (int64_t)blockIdx.y * NB;
    FTile acc = {};
    const TAe* Ab = TA ? A + m0 : A + m0 * lda;
    const TBe* Bb = TB ? B + n0 * ldb : B + n0;
    tile_mm<TA, TB, TAe, TBe>(acc, Ab, lda, Bb, ldb, M - m0, N - n0, K, As, Bs);
    // a tile wholly inside D: the old values read together, then the stores,
    // with no per-element test (each would make the compiler issue and wait
    // for one read at a time)
    if (m0 + NB <= M && n0 + NB <= N) {
        double dv[16];
        if (beta != 0.0) {
#pragma unroll
            for (int e = 0; e < 16; ++e) dv[e] = D[(m0 + tile_row(e)) * ldd + n0 + tile_col(e)];
#pragma unroll
            for (int e = 0; e < 16; ++e) dv[e] = alpha * tile_get(acc, e) + beta * dv[e];
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) dv[e] = alpha * tile_get(acc, e);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) D[(m0 + tile_row(e)) * ldd + n0 + tile_col(e)] = dv[e];
        return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t row = m0 + tile_row(e), col = n0 + tile_col(e);
        if (row < M && col < N) {
            const double v = alpha * tile_get(acc, e);
            D[row * ldd + col] = beta == 0.0 ? v : v + beta * D[row * ldd + col];
        }
    }
}

__global__ __launch_bounds__(256) void k_maxdiag(const double* __restrict__ G, int64_t c, double* __restrict__ out) {
    __shared__ double sh[256];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < c; i += 256) mx = fmax(mx, G[i * c + i]);
    sh[threadIdx.x] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256; ++i) mx = fmax(mx, sh[i]);
        out[0] = mx;
    }
}

// Cholesky of the w x w diagonal block at (j0, j0) of G (w <= 64), with the
// inverse of its factor, in registers (reg_chol_inv).  A column whose
// Schur-complement pivot is not above tau = c rel_tau max diag(G) is
// numerically in the span of the columns before it: it is dropped (flagged),
// its column of L is zero so it updates nothing, and its row of L^-1 is zero so
// the inverse built from L^-1 is that of the kept columns, with zero rows and
// columns for the dropped ones.  Writes L^-1 (NB x NB, lower, zero padded) into
// Linv; G is only read (the diagonal block of L is not needed later).
// piv[0..1] receive the smallest and largest pivot.  Four waves (16 x 16
// threads, ten entries each): a pivot step's work is spread four times wider
// than on one wave of 8 x 8 threads (36 entries each), whose instruction
// stream bounded every step.
__global__ __launch_bounds__(256) void k_potrf_diag(const double* __restrict__ G, int64_t c, int64_t j0, int w,
                                                      const double* __restrict__ maxdiag, double rel_tau,
                                                      double* __restrict__ Linv, double* __restrict__ piv,
                                                      int* __restrict__ info) {
    constexpr int TG = 16, NR = 4;
    __shared__ double P[2 * TG * NR + 1];
    __shared__ double pv[TG * NR];
    const int tid = threadIdx.x, tr = tid / TG, tc = tid % TG;
    const double tau = (double)c * rel_tau * maxdiag[0];
    double m[NR * (NR + 1) / 2];
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tr + TG * a, cc = tc + TG * b;
            m[tri_slot(a, b)] = (i < w && cc <= i) ? G[(j0 + i) * c + (j0 + cc)] : 0.0;
        }
    double pmin, pmax;
    int ndrop;
    reg_chol_inv<TG, NR>(m, w, tau > 0.0 ? tau : 0.0, P, pv, pmin, pmax, ndrop);
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            const int i = tr + TG * a, cc = tc + TG * b;
            double v = 0.0;
            if (b <= a && i < w && cc <= i) v = m[tri_slot(a, b < a ? b : a)];
            Linv[i * NB + cc] = v;
        }
    if (tid == 0) {
        piv[0] = pmin;
        piv[1] = pmax;
        if (ndrop) atomicOr(info, 1);
    }
}

// The whole factorization for c <= 256 in one workgroup (tau from the largest
// diagonal entry; writes X = L^-1, zero above the diagonal, and the pivot
// range into every piv pair), blocked by 16-wide panels with the bulk on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; register v of the result is D[4 v + l / 16][l % 16]).
// The lower triangle is held as 16 x 16 tiles in the result layout, tile
// e = I (I + 1) / 2 + C (I >= C) in slot e / 8 of wave e mod 8 (eight waves: a
// lane's 256 registers hold the 17 tiles of its wave).  Panel J applies the 16
// rank-1 steps of reg_chol_inv as one block:
//   A  the diagonal tile S11 is factored in one wave by the rank-1 steps,
//      giving X11 = L11^-1 (pivots not above tau dropped, as there);
//   B  row J becomes final: X_J = X11 W_J for the tiles left of the diagonal;
//      column J gives L21 = S21 X11^T, and its tiles become -L21 X11;
//   C  every other tile below row J takes the rank-16 update
//      -= L21_I [X_J | L21^T]_C.
// Padding beyond c is the identity, so it never couples to the matrix.
constexpr int kMT = 16;      // tiles per side
constexpr int kMW = 8;       // waves
constexpr int kMSlots = 17;  // lower tiles per wave: ceil(136 / 8)
constexpr int kMLd = 17;     // padded row length of the LDS tiles

__global__ __launch_bounds__(kMW * 64) void k_chol_inv_mfma(const double* __restrict__ G, int64_t c, double rel_tau,
                                                        double* __restrict__ X, double* __restrict__ piv, int npiv,
                                                        int* __restrict__ info) {
    __shared__ double L21s[kMT * 16 * kMLd];       // L21, row i at i * kMLd
    __shared__ double Vs[16 * (kMT * 16 + 1)];     // X_J (columns < 16 J), row k at k * 257
    __shared__ double X11s[16 * kMLd];
    __shared__ double scr[kMW][16 * kMLd];         // one tile per wave
    __shared__ double pivs[kMT * 16];
    __shared__ double wmax[kMW];
    constexpr int LDV = kMT * 16 + 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: slot data in scalar registers
    const int g = lane >> 4, cc = lane & 15;
    const int w = (int)c, nt = (w + 15) / 16, ntiles = nt * (nt + 1) / 2;
    // zeros above the diagonal of X
    for (int64_t e = tid; e < c * c; e += kMW * 64) {
        const int64_t i = e / c, j = e - i * c;
        if (j > i) X[e] = 0.0;
    }
    // this wave's tiles: tm[s] = I | C << 8 (scalar), -1 past the last tile
    int tm[kMSlots];
#pragma unroll
    for (int s = 0; s < kMSlots; ++s) {
        const int e = wave + kMW * s;
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= e) ++I;
        tm[s] = e < ntiles ? (I | ((e - I * (I + 1) / 2) << 8)) : -1;
    }
    d4v acc[kMSlots];
#pragma unroll
    for (int s = 0; s < kMSlots; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * (tm[s] & 0xff) + 4 * v + g, j = 16 * (tm[s] >> 8) + cc;
            double x = 0.0;
            if (tm[s] >= 0 && j <= i) x = (i < w && j < w) ? G[(int64_t)i * c + j] : (i == j ? 1.0 : 0.0);
            acc[s][v] = x;
        }
    double dm = 0.0;
    for (int i = tid; i < w; i += kMW * 64) dm = fmax(dm, G[(int64_t)i * c + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
    if (lane == 0) wmax[wave] = dm;
    __syncthreads();
    dm = 0.0;
#pragma unroll
    for (int u = 0; u < kMW; ++u) dm = fmax(dm, wmax[u]);
    const double tau = fmax((double)c * rel_tau * dm, 0.0);
    double* S = scr[wave];

    for (int J = 0; J < nt; ++J) {
        // the tile coordinates are re-read every panel, so the LDS addresses
        // derived from them are not all kept live across the loop
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) asm volatile("" : "+s"(tm[s]));
        // ---- A: factor the diagonal tile (its owner wave) ----
        const int ed = J * (J + 1) / 2 + J;
        if (wave == ed % kMW) {
            const int sd = ed / kMW;
#pragma unroll
            for (int s = 0; s < kMSlots; ++s)
                if (s == sd)
#pragma unroll
                    for (int v = 0; v < 4; ++v) S[(4 * v + g) * kMLd + cc] = acc[s][v];
            d4v a;
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = S[(4 * v + g) * kMLd + cc];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double d = S[j * kMLd + j];
                double pr[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) pr[v] = S[(4 * v + g) * kMLd + j];
                const double pc = cc <= j ? S[j * kMLd + cc] : S[cc * kMLd + j];
                if (lane == 0) pivs[16 * J + j] = d;
                // branch-free (divergent branches cost more than the selects):
                // the root is taken of a positive stand-in and masked
                const double r = d > tau ? rsqrt_nr(d > tau ? d : 1.0) : 0.0, rd = r * r;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * v + g;
                    const double q = -pr[v] * rd;
                    const double below = cc == j ? q : (cc <= i ? fma(q, pc, a[v]) : a[v]);
                    const double onrow = cc < j ? pc * r : (cc == j ? r : a[v]);
                    a[v] = i > j ? below : (i == j ? onrow : a[v]);
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int v = 0; v < 4; ++v) S[(4 * v + g) * kMLd + cc] = a[v];
                __builtin_amdgcn_wave_barrier();
            }
            // X11 (zero above the diagonal): to LDS, to X, and kept as the final tile
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 4 * v + g;
                const double x = cc <= i ? a[v] : 0.0;
                a[v] = x;
                X11s[i * kMLd + cc] = x;
                const int gi = 16 * J + i, gj = 16 * J + cc;
                if (cc <= i && gi < w && gj < w) X[(int64_t)gi * c + gj] = x;
            }
#pragma unroll
            for (int s = 0; s < kMSlots; ++s)
                if (s == sd) acc[s] = a;
        }
        __syncthreads();
        // ---- B: row J final, column J to L21 ----
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            if (tm[s] < 0) continue;
            const int I = tm[s] & 0xff, C = tm[s] >> 8;
            if (I == J && C < J) {
                // X_J,C = X11 W (W: this tile; its register v is B's k-block v)
                d4v xt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    xt = __builtin_amdgcn_mfma_f64_16x16x4f64(X11s[cc * kMLd + 4 * kb + g], acc[s][kb], xt, 0, 0, 0);
                acc[s] = xt;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * v + g, gi = 16 * J + i, gj = 16 * C + cc;
                    Vs[i * LDV + gj] = xt[v];
                    if (gi < w) X[(int64_t)gi * c + gj] = xt[v];
                }
            } else if (I > J && C == J) {
                // L21 = S21 X11^T: S21 goes through this wave's scratch for the A layout
#pragma unroll
                for (int v = 0; v < 4; ++v) S[(4 * v + g) * kMLd + cc] = acc[s][v];
                __builtin_amdgcn_wave_barrier();
                d4v l21 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    l21 = __builtin_amdgcn_mfma_f64_16x16x4f64(S[cc * kMLd + 4 * kb + g], X11s[cc * kMLd + 4 * kb + g],
                                                               l21, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) L21s[(16 * I + 4 * v + g) * kMLd + cc] = l21[v];
                __builtin_amdgcn_wave_barrier();
                // this tile becomes -L21 X11
                d4v t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    t = __builtin_amdgcn_mfma_f64_16x16x4f64(-L21s[(16 * I + cc) * kMLd + 4 * kb + g],
                                                             X11s[(4 * kb + g) * kMLd + cc], t, 0, 0, 0);
                acc[s] = t;
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        // ---- C: rank-16 update of the tiles below row J ----
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            if (tm[s] < 0) continue;
            const int I = tm[s] & 0xff, C = tm[s] >> 8;
            if (I <= J || C == J) continue;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const double av = -L21s[(16 * I + cc) * kMLd + 4 * kb + g];
                const double bv = C < J ? Vs[(4 * kb + g) * LDV + 16 * C + cc] : L21s[(16 * C + cc) * kMLd + 4 * kb + g];
                acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[s], 0, 0, 0);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double pmin = INFINITY, pmax = 0.0;
        int ndrop = 0;
        for (int j = 0; j < w; ++j) {
            const double d = pivs[j];
            pmin = fmin(pmin, d);
            pmax = fmax(pmax, d);
            ndrop += d > tau ? 0 : 1;
        }
        for (int q = 0; q < npiv; ++q) {
            piv[2 * q] = pmin;
            piv[2 * q + 1] = pmax;
        }
        if (ndrop) atomicOr(info, 1);
    }
}

// One level of the recursive blocked inverse X = L^-1 (lower; NB-blocks, the
// diagonal blocks already in X).  Node z of the level covers the blocks
// b0 = 2 h z .. min(b0 + 2h, nblk) - 1; with mid = b0 + h its lower-left part
// is X21 = -X22 (L21 X11), X11 and X22 the inverses of its two halves (formed
// by the levels before).  PASS 0 forms T = L21 X11 (node z's T at
// T + z (h NB)^2, leading dimension h NB); PASS 1 writes X21 = -X22 T.  Both
// skip the zero parts of the triangular factors: T's columns from tn0 on need
// only rows k >= tn0 of X11, and X21's rows up to tm0 + NB only columns
// k < tm0 + NB of X22.  This equals the block forward substitution
// X_ij = -Linv_ii sum_{j <= p < i} L_ip X_pj (also with dropped pivots, whose
// rows of Linv are zero) up to the order of the sums.
template <int PASS>
__global__ __launch_bounds__(256) void k_trtri_level(const double* __restrict__ L, double* __restrict__ X, int64_t c,
                                                     int64_t h, int64_t nblk, double* __restrict__ T) {
    __shared__ double As[KB * (NB + 1)], Bs[KB * (NB + 1)];
    const int64_t z = blockIdx.z;
    const int64_t b0 = 2 * h * z, mid = b0 + h;
    if (mid >= nblk) return;
    const int64_t b1 = b0 + 2 * h < nblk ? b0 + 2 * h : nblk;
    const int64_t r0 = mid * NB, r1 = b1 * NB < c ? b1 * NB : c;
    const int64_t c0 = b0 * NB, c1 = mid * NB;
    const int64_t rows = r1 - r0, cols = c1 - c0;
    const int64_t tm0 = (int64_t)blockIdx.x * NB, tn0 = (int64_t)blockIdx.y * NB;
    if (tm0 >= rows || tn0 >= cols) return;
    const int64_t ldt = h * NB;
    double* Tz = T + z * ldt * ldt;
    FTile acc = {};
    if (PASS == 0)
        tile_mm<false, false>(acc, L + (r0 + tm0) * c + c0 + tn0, c, X + (c0 + tn0) * c + c0 + tn0, c, rows - tm0,
                              cols - tn0, cols - tn0, As, Bs);
    else
        tile_mm<false, false>(acc, X + (r0 + tm0) * c + r0, c, Tz + tn0, ldt, rows - tm0, cols - tn0,
                              rows < tm0 + NB ? rows : tm0 + NB, As, Bs);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t row = tm0 + tile_row(e), col = tn0 + tile_col(e);
        if (row < rows && col < cols) {
            if (PASS == 0) Tz[row * ldt + col] = tile_get(acc, e);
            else X[(r0 + row) * c + c0 + col] = -tile_get(acc, e);
        }
    }
}

// Doubles of the recursive inverse's T buffer: the largest level's nodes x (h NB)^2.
int64_t trtri_t_doubles(int64_t nblk) {
    int64_t best = 0;
    for (int64_t h = 1; h < nblk; h *= 2) {
        const int64_t nodes = (nblk + 2 * h - 1) / (2 * h);
        const int64_t v = nodes * (h * NB) * (h * NB);
        if (v > best) best = v;
    }
    return best;
}

// X = 0, then the diagonal blocks of X = L^-1 from Linv.
__global__ __launch_bounds__(256) void k_init_xinv(double* __restrict__ X, int64_t c, const double* __restrict__ Linv) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < c * c; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / c, j = e - i * c;
        const int64_t bi = i / NB, bj = j / NB;
        X[e] = bi == bj ? Linv[bi * NB * NB + (i - bi * NB) * NB + (j - bj * NB)] : 0.0;
    }
}

}  // namespace

size_t spd_inverse_ws_doubles(int64_t c) {
    const int64_t nblk = (c + NB - 1) / NB;
    return (size_t)(nblk * NB * NB) + (size_t)(c * c) + (size_t)(2 * nblk) + 8 +
           (c > kFullChol ? (size_t)trtri_t_doubles(nblk) : 0);
}

template <typename TAe, typename TBe>
hipError_t dgemm_any(int64_t M, int64_t N, int64_t K, double alpha, const TAe* A, int64_t lda, bool tA, const TBe* B,
                     int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((M + NB - 1) / NB), (unsigned)((N + NB - 1) / NB));
    if (!tA && !tB)
        hipLaunchKernelGGL((k_dgemm<false, false, TAe, TBe>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, D, ldd);
    else if (!tA && tB)
        hipLaunchKernelGGL((k_dgemm<false, true, TAe, TBe>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, D, ldd);
    else if (tA && !tB)
        hipLaunchKernelGGL((k_dgemm<true, false, TAe, TBe>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, D, ldd);
    else
        hipLaunchKernelGGL((k_dgemm<true, true, TAe, TBe>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, D, ldd);
    return hipGetLastError();
}

hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, bool tA,
                        const double* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st) {
    return dgemm_any(M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, D, ldd, st);
}
hipError_t launch_dgemm_ff(int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda, bool tA,
                           const float* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st) {
    return dgemm_any(M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, D, ldd, st);
}
hipError_t launch_dgemm_fd(int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda, bool tA,
                           const double* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st) {
    return dgemm_any(M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, D, ldd, st);
}
hipError_t launch_dgemm_df(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, bool tA,
                           const float* B, int64_t ldb, bool tB, double beta, double* D, int64_t ldd, hipStream_t st) {
    return dgemm_any(M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, D, ldd, st);
}

// ws: [Linv blocks nblk*NB*NB][X c*c][piv 2*nblk][maxdiag, 8][T of the
// recursive inverse].  Factor G (in place, lower L) and form X = L^-1 (lower)
// in the workspace; returns X.
static hipError_t chol_and_inverse_factor(double* G, int64_t c, double* ws, int* info, double* piv, double rel_tau,
                                          double** Xout, hipStream_t st) {
    const int64_t nblk = (c + NB - 1) / NB;
    double* Linv = ws;
    double* X = Linv + nblk * NB * NB;
    double* pivb = X + c * c;
    double* maxd = pivb + 2 * nblk;
    if (c <= kFullChol) {
        hipLaunchKernelGGL(k_chol_inv_mfma, dim3(1), dim3(kMW * 64), 0, st, (const double*)G, c, rel_tau, X,
                           piv ? piv : pivb, (int)nblk, info);
        *Xout = X;
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_maxdiag, dim3(1), dim3(256), 0, st, (const double*)G, c, maxd);
    for (int64_t jb = 0; jb < nblk; ++jb) {
        const int64_t j0 = jb * NB;
        const int w = (int)(c - j0 < NB ? c - j0 : NB);
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, (const double*)G, c, j0, w,
                           (const double*)maxd, rel_tau, Linv + jb * NB * NB, pivb + 2 * jb, info);
        const int64_t rows = c - j0 - w;
        if (rows > 0) {
            double* L21 = G + (j0 + w) * c + j0;
            hipError_t e = launch_dgemm(rows, w, w, 1.0, L21, c, false, Linv + jb * NB * NB, NB, true, 0.0, L21, c, st);
            if (e != hipSuccess) return e;
            e = launch_dgemm(rows, rows, w, -1.0, L21, c, false, L21, c, true, 1.0, G + (j0 + w) * c + (j0 + w), c, st);
            if (e != hipSuccess) return e;
        }
    }
    int64_t blocks = (c * c + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_init_xinv, dim3((unsigned)blocks), dim3(256), 0, st, X, c, (const double*)Linv);
    double* T = maxd + 8;
    for (int64_t h = 1; h < nblk; h *= 2) {
        const dim3 grid((unsigned)h, (unsigned)h, (unsigned)((nblk + 2 * h - 1) / (2 * h)));
        hipLaunchKernelGGL(k_trtri_level<0>, grid, dim3(256), 0, st, (const double*)G, X, c, h, nblk, T);
        hipLaunchKernelGGL(k_trtri_level<1>, grid, dim3(256), 0, st, (const double*)G, X, c, h, nblk, T);
    }
    if (piv) {
        const hipError_t e2 = hipMemcpyAsync(piv, pivb, sizeof(double) * 2 * nblk, hipMemcpyDeviceToDevice, st);
        if (e2 != hipSuccess) return e2;
    }
    *Xout = X;
    return hipGetLastError();
}

hipError_t launch_spd_inverse(double* G, int64_t c, double* Ginv, double* ws, int* info, double* piv, double rel_tau,
                              hipStream_t st) {
    double* X = nullptr;
    hipError_t e = chol_and_inverse_factor(G, c, ws, info, piv, rel_tau, &X, st);
    if (e != hipSuccess) return e;
    return launch_dgemm(c, c, c, 1.0, X, c, true, X, c, false, 0.0, Ginv, c, st);
}

hipError_t launch_chol_linv(double* G, int64_t c, double* ws, int* info, double* piv, double rel_tau, double** Linv,
                            hipStream_t st) {
    return chol_and_inverse_factor(G, c, ws, info, piv, rel_tau, Linv, st);
}

}  // namespace bcur
