// FP32 GEMMs on the CDNA4 matrix cores (v_mfma_f32_32x32x2_f32, FP32
// accumulation) for every contraction of the Block CUR path:
//   Z = A Q, Y = A^T Z          (range finder passes, N = sketch width)
//   H = C^T A                   (fit: projection onto the chosen columns)
//   G^-1 = X^T X, U = G^-1 H, ||A - C U||  (fit: solve and residual norm)
//   F = H - G U                 (fit: the refinement's right-hand side)
// D = op(A) B with op(A) = A (M x K) or A^T (A stored K x M), B is K x N; all
// operands row-major.  Tiles are staged through LDS in k-major order so each
// MFMA operand read is 32 consecutive floats.  Split-K writes partial tiles
// that a second kernel sums in a fixed order, so results are deterministic.
#include "bcur_internal.h"

namespace bcur {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct GemmArgs {
    int64_t M, N, K;
    const float* A;
    int64_t lda;
    const float* B;
    int64_t ldb;
    float* D;
    int64_t ldd;
    int64_t kchunk;
    int64_t split_stride;
    const float* X;
    int64_t ldx;
    const float* Y;
    int64_t ldy;
    double* wsum;
    int swz;            // tile order (see tile_of); 0: blockIdx.x, blockIdx.y are the M and N tiles
    int64_t tm, tn;     // M and N tiles
    bool full;          // k_xgemm: every tile and k-step inside the matrices (no bounds checks)
    // k_xgemm's norm-only residual (A not transposed): when not null, output
    // column j (< N) is column ncol[j] of B and X (null: column j)
    const int* ncol;
};

// Tile order.  Workgroups are handed to the eight XCDs (each with its own L2)
// round-robin by their linear index L, XCD L % 8; the order below gives every
// XCD a compact set of tiles, so the operand panels its workgroups stream are
// shared in its L2 instead of being fetched by several XCDs.  The grid is then
// one-dimensional in x (split-K in z).
//   swz 1 (tm % 64 == 0, tn % 8 == 0): XCD x owns the M-tiles x tm/8 ..
//          (x+1) tm/8 - 1 and every N-tile, walked as 8 x 8 squares of tiles
//          (M fastest), so each panel of either operand serves 8 workgroups.
// (H = C^T A keeps the plain order: giving each XCD a band of N-tiles raised
// its HBM fetch from 36 to 52 GiB at 65536 x 16384 x 2048 without changing
// its time.)
__device__ __forceinline__ void tile_of(const GemmArgs& g, int64_t& mt, int64_t& nt) {
    if (g.swz == 0) {
        mt = blockIdx.x;
        nt = blockIdx.y;
        return;
    }
    const int64_t L = blockIdx.x, x = L & 7, t = L >> 3;
    const int64_t band = g.tm >> 3, nbn = g.tn >> 3;
    const int64_t b = t >> 6, q = t & 63;
    mt = x * band + (b / nbn) * 8 + (q & 7);
    nt = (b % nbn) * 8 + (q >> 3);
}

// Load 4 consecutive floats p[0..3] (p 16-byte aligned), zero outside [c, cend).
__device__ __forceinline__ float4 ld4(const float* p, bool rowok, int64_t c, int64_t cend) {
    if (rowok && c + 3 < cend) return *reinterpret_cast<const float4*>(p);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (rowok) {
        if (c < cend) v.x = p[0];
        if (c + 1 < cend) v.y = p[1];
        if (c + 2 < cend) v.z = p[2];
        if (c + 3 < cend) v.w = p[3];
    }
    return v;
}

// The norm-only residual epilogue has two forms.  EPI_RESID_NORM reads the
// residual input X for the thread's outputs before the main loop (its latency
// hides behind the MFMA work; best for a short K, the loads occupy 64 more
// registers: two waves per SIMD).  kResidLate reads X in the epilogue and
// asks the compiler for four waves per SIMD (no spills at these tiles): for a
// long K the occupancy hides the main loop's own latency better (65536 x
// 16384 x 2048: 38.3 -> 36.4 ms; 8192 x 4096 x 256: 0.178 -> 0.187 ms, so the
// early read stays for short K).
constexpr int kResidLate = 5;

template <int BM, int BN, int BK, int WM, int WN, bool TA, int EPI>
__global__ __launch_bounds__(WM* WN * 64, EPI == kResidLate ? 4 : 1) void k_sgemm(const GemmArgs g) {
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    constexpr int LDAS = BM + 4, LDBS = BN + 4;
    constexpr int A_F4 = BM * BK / 4 / NT;
    constexpr int B_F4 = BK * BN / 4 / NT;
    static_assert(TM >= 1 && TN >= 1 && A_F4 >= 1 && B_F4 >= 1, "tile shape");
    static_assert((BM * BK / 4) % NT == 0 && (BK * BN / 4) % NT == 0, "tile shape");

    __shared__ __attribute__((aligned(16))) float As[BK * LDAS];
    __shared__ __attribute__((aligned(16))) float Bs[BK * LDBS];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int wm = wave % WM, wn = wave / WM;
    int64_t mtile, ntile;
    tile_of(g, mtile, ntile);
    const int64_t m0 = mtile * BM, n0 = ntile * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    float4 ra[A_F4], rb[B_F4];

    // EPI_RESID: the residual input X of this thread's outputs is read before the
    // main loop (a wave-uniform base plus one lane offset per load), so its HBM
    // latency is hidden behind the MFMA work instead of following it.
    constexpr bool kResid = EPI == EPI_RESID || EPI == EPI_RESID_NORM || EPI == kResidLate;
    constexpr bool kPre = EPI == EPI_RESID || EPI == EPI_RESID_NORM;
    constexpr int XM = kPre ? TM : 1, XN = kPre ? TN : 1;
    float xv[XM][XN][16];
    if constexpr (kPre) {
        const int wmu = __builtin_amdgcn_readfirstlane(wm), wnu = __builtin_amdgcn_readfirstlane(wn);
        const int64_t rb0 = m0 + wmu * WTM, cb0 = n0 + wnu * WTN;
        const float* xbase = g.X + rb0 * g.ldx + cb0;
        const int64_t lane_off = 4 * h * g.ldx + r;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int rr = 32 * i + 8 * (v >> 2) + (v & 3);
                    const int64_t row = rb0 + rr + 4 * h, col = cb0 + 32 * j + r;
                    const float* px = xbase + (int64_t)rr * g.ldx + 32 * j;
                    xv[i][j][v] = (row < g.M && col < g.N) ? px[lane_off] : 0.f;
                }
    }

    auto load_tiles = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < A_F4; ++u) {
            const int f = tid + u * NT;
            if (!TA) {
                const int row = f / (BK / 4), kq = f % (BK / 4);
                const int64_t gm = m0 + row, gk = k0 + kq * 4;
                ra[u] = ld4(g.A + gm * g.lda + gk, gm < g.M, gk, kend);
            } else {
                const int kr = f / (BM / 4), mq = f % (BM / 4);
                const int64_t gk = k0 + kr, gm = m0 + mq * 4;
                ra[u] = ld4(g.A + gk * g.lda + gm, gk < kend, gm, g.M);
            }
        }
#pragma unroll
        for (int u = 0; u < B_F4; ++u) {
            const int f = tid + u * NT;
            const int kr = f / (BN / 4), nq = f % (BN / 4);
            const int64_t gk = k0 + kr, gn = n0 + nq * 4;
            rb[u] = ld4(g.B + gk * g.ldb + gn, gk < kend, gn, g.N);
        }
    };
    // EPI_STORE_SQA: the sum of squares of the A operand as it passes through
    // (each element of A is loaded by exactly one workgroup of the first column
    // of tiles; the others do not count)
    constexpr bool kSqa = EPI == EPI_STORE_SQA && !TA;
    const bool count_sq = kSqa && ntile == 0;
    double sqa = 0.0;
    auto store_tiles = [&]() {
#pragma unroll
        for (int u = 0; u < A_F4; ++u) {
            const int f = tid + u * NT;
            if (kSqa && count_sq) {
                const double x0 = ra[u].x, x1 = ra[u].y, x2 = ra[u].z, x3 = ra[u].w;
                sqa = fma(x0, x0, sqa);
                sqa = fma(x1, x1, sqa);
                sqa = fma(x2, x2, sqa);
                sqa = fma(x3, x3, sqa);
            }
            if (!TA) {
                const int row = f / (BK / 4), kq = f % (BK / 4);
                As[(kq * 4 + 0) * LDAS + row] = ra[u].x;
                As[(kq * 4 + 1) * LDAS + row] = ra[u].y;
                As[(kq * 4 + 2) * LDAS + row] = ra[u].z;
                As[(kq * 4 + 3) * LDAS + row] = ra[u].w;
            } else {
                const int kr = f / (BM / 4), mq = f % (BM / 4);
                *reinterpret_cast<float4*>(&As[kr * LDAS + mq * 4]) = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < B_F4; ++u) {
            const int f = tid + u * NT;
            const int kr = f / (BN / 4), nq = f % (BN / 4);
            *reinterpret_cast<float4*>(&Bs[kr * LDBS + nq * 4]) = rb[u];
        }
    };

    int64_t k0 = kbeg;
    if (k0 < kend) load_tiles(k0);
    for (; k0 < kend; k0 += BK) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (k0 + BK < kend) load_tiles(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            float a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[(kk + h) * LDAS + wm * WTM + 32 * i + r];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[(kk + h) * LDBS + wn * WTN + 32 * j + r];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }

    // Output layout of a 32x32 MFMA tile: lane (r, h), register v holds
    // row 8 (v / 4) + 4 h + (v % 4), column r.
    float* D = g.D + (int64_t)blockIdx.z * g.split_stride;
    double wacc = 0.0;
    // a tile wholly inside D takes the form without per-element tests, so the
    // compiler issues its reads of X together instead of one at a time (not
    // with the X + D and Y reads of EPI_ADD_DOT and the early X of EPI_RESID:
    // there it would raise the registers past two waves per SIMD)
    auto epilogue = [&](auto checked) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + wm * WTM + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                    const int64_t col = n0 + wn * WTN + 32 * j + r;
                    if (!decltype(checked)::value || (row < g.M && col < g.N)) {
                        const float x = acc[i][j][v];
                        if (EPI == EPI_STORE || EPI == EPI_STORE_SQA) {
                            D[row * g.ldd + col] = x;
                        } else if (kResid) {
                            float xe;
                            if constexpr (kPre) xe = xv[i][j][v];
                            else xe = g.X[row * g.ldx + col];
                            const float e = xe - x;
                            if (EPI == EPI_RESID) D[row * g.ldd + col] = e;
                            wacc += (double)e * (double)e;
                        } else {
                            D[row * g.ldd + col] = g.X[row * g.ldx + col] + x;
                            wacc += (double)x * (double)g.Y[row * g.ldy + col];
                        }
                    }
                }
    };
    constexpr bool kWhole = EPI == EPI_STORE || EPI == EPI_STORE_SQA || EPI == kResidLate;
    if (kWhole && m0 + BM <= g.M && n0 + BN <= g.N)
        epilogue(std::false_type{});
    else
        epilogue(std::true_type{});
    if constexpr (EPI == EPI_STORE_SQA) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sqa += __shfl_xor(sqa, o, 64);
        if (lane == 0) red[wave] = sqa;
        __syncthreads();
        if (tid == 0) {
            double s2 = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s2 += red[w];
            g.wsum[blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)] = s2;
        }
    } else if (EPI != EPI_STORE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wacc += __shfl_xor(wacc, o, 64);
        if (lane == 0) red[wave] = wacc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            g.wsum[blockIdx.x + (int64_t)gridDim.x * blockIdx.y] = s;
        }
    }
}

// The same products with each FP32 operand split exactly into three BF16
// terms, a = a0 + a1 + a2 (a0 = bf16(a), a1 = bf16(a - a0), a2 = the rest,
// each rounded to nearest: a has 24 significant bits, a0 and a1 take 8 each
// and the remainder has at most 8, so the split loses nothing), and the
// product a b formed by six BF16 MFMAs (v_mfma_f32_32x32x16_bf16, FP32
// accumulation) as a0 b0 + a0 b1 + a1 b0 + a0 b2 + a1 b1 + a2 b0.  The
// dropped terms a1 b2 + a2 b1 + a2 b2 are below 2^-23 |a b| (|a1| <= 2^-8 |a|,
// |a2| <= 2^-16 |a|), so each product is within two FP32 unit roundoffs of
// the exact one, below the rounding of the FP32 accumulation that follows.
// The BF16 matrix cores run sixteen times the FP32 MFMA rate, so the six
// products take 6/16 of the FP32 MFMA time.  (Valid for |a| < 3.38e38: larger
// finite FP32 values round to infinity in BF16; infinities and NaNs give NaN.)
//
// Tile 256 x 256 x 16 for eight waves (128 x 64 each), LDS double-buffered
// (one barrier per step).  Each operand tile sits in LDS as three BF16
// planes, one 48-byte row (16 k values and 16 bytes of padding) per output
// row or column, so each MFMA operand read (8 consecutive k per lane) is one
// 16-byte LDS read.  Each thread splits 8 consecutive k of one row or column
// into the planes (three 16-byte LDS writes per 8 values):
//   * A stored k-contiguous: four consecutive lanes read 64 contiguous bytes
//     of each of two rows (16 rows per wave load instruction) and swap one
//     16-byte half with the neighbouring lane, so each ends with one row's
//     octet;
//   * an operand stored with k as the row index (A when transposed, and B):
//     a thread takes a pair of adjacent columns and one octet of k, eight
//     8-byte loads contiguous across the wave (A on waves 0-3, B on waves
//     4-7); the transposition into k-contiguous LDS rows comes with the split.
// FULL (every tile and k-step inside the matrices): no bounds checks, and
// the loads address a wave-uniform base in scalar registers plus a 32-bit
// lane offset, so the step's vector ALU work is the split itself.
typedef __bf16 xbf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 xbf16x8 __attribute__((ext_vector_type(8)));
typedef float xf32x2 __attribute__((ext_vector_type(2)));
typedef float xf32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(const float* v, uint4& p0, uint4& p1, uint4& p2) {
    uint32_t w0[4], w1[4], w2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const xf32x2 x = {v[2 * i], v[2 * i + 1]};
        const xbf16x2 h0 = __builtin_convertvector(x, xbf16x2);
        const xf32x2 r1 = x - __builtin_convertvector(h0, xf32x2);
        const xbf16x2 h1 = __builtin_convertvector(r1, xbf16x2);
        const xf32x2 r2 = r1 - __builtin_convertvector(h1, xf32x2);
        const xbf16x2 h2 = __builtin_convertvector(r2, xbf16x2);
        w0[i] = __builtin_bit_cast(uint32_t, h0);
        w1[i] = __builtin_bit_cast(uint32_t, h1);
        w2[i] = __builtin_bit_cast(uint32_t, h2);
    }
    p0 = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    p1 = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    p2 = make_uint4(w2[0], w2[1], w2[2], w2[3]);
}

// A wave-uniform global address, moved to scalar registers (kept in the
// global address space, so its loads are global loads, not FLAT ones that
// the LDS wait counter would also have to wait for).
typedef const __attribute__((address_space(1))) char* gchar_ptr;
__device__ __forceinline__ gchar_ptr uniform_ptr(const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<gchar_ptr>(((uint64_t)hi << 32) | lo);
}

// The largest leading dimension (floats) the FULL kernels address with
// 32-bit lane offsets (8 rows of it, and 32 rows of A not transposed).
constexpr int64_t kXFullMaxLd = (int64_t)1 << 25;
constexpr bool kXBCol = true;

template <bool TA, int EPI, bool FULL, int BM, int BN>
__global__ __launch_bounds__(BM * 2) void k_xgemm(const GemmArgs g) {
    static_assert((BM == 256 && BN == 256) || (BM == 128 && (BN == 128 || BN == 64)), "tile shape");
    // eight waves for 256 rows (128 x 64 per wave), four for 128 (64 x 64 or 64 x 32)
    constexpr int NW = BM / 32, BK = 16, NT = 64 * NW;
    constexpr int WM = 2, WN = NW / WM;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    constexpr int ROW = 24;                         // bf16 per LDS row: 16 k + 8 padding (48 bytes)
    constexpr int PA = BM * ROW, PB = BN * ROW;     // one plane
    constexpr int STAGE = 3 * PA + 3 * PB;          // one buffer: three A planes, three B planes
    static_assert(EPI == EPI_STORE || EPI == EPI_STORE_SQA || EPI == kResidLate || EPI == EPI_RESID ||
                      EPI == EPI_ADD_DOT, "epilogue");
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int wm = wave % WM, wn = wave / WM;
    int64_t mtile, ntile;
    tile_of(g, mtile, ntile);
    const int64_t m0 = mtile * BM, n0 = ntile * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    // A not transposed: lanes 4j .. 4j+3 of wave w read rows w*32 + 2j and
    // w*32 + 2j + 1 at k-quad lane & 3; afterwards the lane holds row
    // w*32 + 2j + (lane & 1), octet (lane >> 1) & 1.
    const int xg = lane >> 2, xe = lane & 1, xo = (lane >> 1) & 1;
    // k-row-major operands, W columns wide: unit u = 64 (wave - first wave)
    // + lane is column pair u % (W/2), octet u / (W/2).  A when transposed on
    // the first BM/64 waves; B on the last BN/64
    constexpr int WB0 = NW - BN / 64;
    // With A not transposed every wave already stages A, so B is staged one
    // column per thread (column u % BN, octet u / BN for u = tid < 2 BN, eight
    // 4-byte loads contiguous across the wave) and spread over all the waves;
    // column pairs on the last waves only would give those waves three times
    // the staging work of the others, and the rest would wait at each barrier.
    // (A 64-wide B is always staged by columns: as column pairs it would not
    // fill a wave per octet.  With A transposed its columns go on the last
    // 2 BN / 64 waves, after A's units.)
    constexpr bool BCOL = (!TA && kXBCol) || BN == 64;
    constexpr int BC0 = TA ? NT - 2 * BN : 0;
    const bool bwave = !BCOL && wave >= WB0;
    // (on the 256 x 256 tile with A not transposed every thread stages a
    // column, known at compile time: its stores need no branch)
    const bool bcol = BCOL && ((BM == 256 && BC0 == 0 && 2 * BN == NT) || (tid >= BC0 && tid < BC0 + 2 * BN));
    const int bcc = (tid - BC0) % BN, bco = (tid - BC0) / BN;
    // the column of B this thread stages: through the residual's column list
    // when it has one (read once per tile)
    constexpr bool kCols = EPI == kResidLate && !TA;
    int64_t bsrc = 0;
    if constexpr (kCols) {
        bsrc = n0 + bcc;
        if (g.ncol && bcol && bsrc < g.N) bsrc = g.ncol[bsrc];
    }
    const int uu = 64 * (bwave ? wave - WB0 : wave) + lane;
    const int uw = bwave ? BN / 2 : BM / 2;
    const int cp = uu % uw, ko = uu / uw;
    const bool xwave = !TA;                   // A not transposed: every wave holds 32 of its rows
    const bool awave = TA && wave < BM / 64;  // A transposed: units on the first BM/64 waves
    float pa[8], ku[16], pb[8];

    // FULL with a 128-wide tile: B's columns past N (a sketch width that is
    // not a multiple of 128) are masked per lane; N is even, so a column
    // pair is wholly inside or outside
    auto load_units = [&](const float* base, int64_t ld, int64_t c0, int64_t ncols, int64_t k0) {
        const int64_t gk = k0 + 8 * ko;
        if constexpr (FULL) {
            const gchar_ptr sb = uniform_ptr(base + gk * ld + c0);
            const uint32_t voff = 8u * (uint32_t)cp, rstep = 4u * (uint32_t)ld;
            const bool colok = BN == 256 || c0 + 2 * cp < ncols;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                xf32x2 x = {0.f, 0.f};
                if (colok)
                    x = *reinterpret_cast<const __attribute__((address_space(1))) xf32x2*>(sb + (t * rstep + voff));
                ku[t] = x[0];
                ku[8 + t] = x[1];
            }
        } else {
            const int64_t gc = c0 + 2 * cp;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float* q = base + (gk + t) * ld + gc;
                const bool kin = gk + t < kend;
                if (kin && gc + 1 < ncols) {
                    const float2 x = *reinterpret_cast<const float2*>(q);
                    ku[t] = x.x;
                    ku[8 + t] = x.y;
                } else {
                    ku[t] = (kin && gc < ncols) ? q[0] : 0.f;
                    ku[8 + t] = (kin && gc + 1 < ncols) ? q[1] : 0.f;
                }
            }
        }
    };
    auto load = [&](int64_t k0) {
        if (xwave) {
            float4 l1, l2;
            if constexpr (FULL) {
                typedef const __attribute__((address_space(1))) xf32x4* gf4_ptr;
                const gchar_ptr sb = uniform_ptr(g.A + (m0 + wave * 32) * g.lda + k0);
                const uint32_t voff = (uint32_t)(2 * xg * g.lda + 4 * (lane & 3)) * 4u;
                const xf32x4 v1 = *reinterpret_cast<gf4_ptr>(sb + voff);
                const xf32x4 v2 = *reinterpret_cast<gf4_ptr>(sb + (voff + 4u * (uint32_t)g.lda));
                l1 = make_float4(v1[0], v1[1], v1[2], v1[3]);
                l2 = make_float4(v2[0], v2[1], v2[2], v2[3]);
            } else {
                const int64_t ra = m0 + wave * 32 + 2 * xg, gk = k0 + 4 * (lane & 3);
                l1 = ld4(g.A + ra * g.lda + gk, ra < g.M, gk, kend);
                l2 = ld4(g.A + (ra + 1) * g.lda + gk, ra + 1 < g.M, gk, kend);
            }
            // raw loads; the swap happens in store(), a step later
            pa[0] = l1.x; pa[1] = l1.y; pa[2] = l1.z; pa[3] = l1.w;
            pa[4] = l2.x; pa[5] = l2.y; pa[6] = l2.z; pa[7] = l2.w;
        } else if (awave) {
            load_units(g.A, g.lda, m0, g.M, k0);
        }
        if (bwave) load_units(g.B, g.ldb, n0, g.N, k0);
        if (bcol) {
            const int64_t gk = k0 + 8 * bco, gn = n0 + bcc;
            if constexpr (FULL) {
                // (with a column list the lane offset carries the whole column:
                // below N <= ldb <= kXFullMaxLd, so 4 (7 ldb + column) fits 32 bits)
                const gchar_ptr sb = uniform_ptr(g.B + gk * g.ldb + (kCols ? 0 : n0));
                const uint32_t voff = 4u * (uint32_t)(kCols ? bsrc : bcc), rstep = 4u * (uint32_t)g.ldb;
                const bool colok = BN == 256 || gn < g.N;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    float x = 0.f;
                    if (colok) x = *reinterpret_cast<const __attribute__((address_space(1))) float*>(sb + (t * rstep + voff));
                    pb[t] = x;
                }
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    pb[t] = (gn < g.N && gk + t < kend) ? g.B[(gk + t) * g.ldb + (kCols ? bsrc : gn)] : 0.f;
            }
        }
    };
    // EPI_STORE_SQA: the sum of squares of the A operand as it passes through
    // (the workgroups of the first column of tiles load each element once)
    constexpr bool kSqa = EPI == EPI_STORE_SQA && !TA;
    const bool count_sq = kSqa && ntile == 0;
    double sqa = 0.0;
    auto put = [&](uint16_t* q, int plane_stride, const float* v) {
        uint4 p0, p1, p2;
        split3(v, p0, p1, p2);
        *reinterpret_cast<uint4*>(q) = p0;
        *reinterpret_cast<uint4*>(q + plane_stride) = p1;
        *reinterpret_cast<uint4*>(q + 2 * plane_stride) = p2;
    };
    auto put_units = [&](uint16_t* q, int plane_stride) {
        float v0[8], v1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            v0[t] = ku[t];
            v1[t] = ku[8 + t];
        }
        put(q, plane_stride, v0);
        put(q + ROW, plane_stride, v1);
    };
    // counted: the step is a real one (the loop's last store repeats a step)
    auto store = [&](int buf, bool counted) {
        uint16_t* base = lds + buf * STAGE;
        if (xwave) {
            // even lanes keep their first row's quad and take the odd neighbour's,
            // odd lanes give their first and keep their second row's (DPP quad
            // permute 1 0 3 2: plain VALU, no LDS round trip)
            float v[8];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float snd = xe ? pa[t] : pa[4 + t];
                const float rcv = __int_as_float(
                    __builtin_amdgcn_mov_dpp(__float_as_int(snd), 0xB1, 0xF, 0xF, false));
                v[t] = xe ? rcv : pa[t];
                v[4 + t] = xe ? pa[4 + t] : rcv;
            }
            if (kSqa && count_sq && counted)
#pragma unroll
                for (int t = 0; t < 8; ++t) sqa = fma((double)v[t], (double)v[t], sqa);
            put(base + (wave * 32 + 2 * xg + xe) * ROW + 8 * xo, PA, v);
        } else if (awave) {
            put_units(base + 2 * cp * ROW + 8 * ko, PA);
        }
        if (bwave) put_units(base + 3 * PA + 2 * cp * ROW + 8 * ko, PB);
        if (bcol) put(base + 3 * PA + bcc * ROW + 8 * bco, PB, pb);
    };

    int64_t k0 = kbeg;
    int buf = 0;
    if (k0 < kend) {
        load(k0);
        store(0, true);
    }
    __syncthreads();
    for (; k0 < kend; k0 += BK) {
        // the next step's operands (the last step reloads its own, which the
        // idle buffer then receives unused: the loop body has no branch)
        const bool more = k0 + BK < kend;
        load(more ? k0 + BK : k0);
        // keep the loads here, a whole step ahead of their use (left alone, the
        // compiler sinks them next to the split and waits on them at once)
        __builtin_amdgcn_sched_barrier(0);
        const uint16_t* As = lds + buf * STAGE;
        const uint16_t* Bs = As + 3 * PA;
        auto fa = [&](int p, int i) {
            return *reinterpret_cast<const xbf16x8*>(&As[p * PA + (wm * WTM + 32 * i + r) * ROW + 8 * h]);
        };
        auto fb = [&](int p, int j) {
            return *reinterpret_cast<const xbf16x8*>(&Bs[p * PB + (wn * WTN + 32 * j + r) * ROW + 8 * h]);
        };
        // one plane pair over all TM x TN accumulators (consecutive MFMAs independent)
        auto mfma_all = [&](const xbf16x8 (&a)[TM], const xbf16x8 (&b)[TN]) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        };
        // the small terms first: a2 b0, a1 b1, a1 b0, then a0 (b2, b1, b0)
        xbf16x8 b0[TN], b1[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) b0[j] = fb(0, j);
        {
            xbf16x8 a2[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a2[i] = fa(2, i);
            mfma_all(a2, b0);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) b1[j] = fb(1, j);
        {
            xbf16x8 a1[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a1[i] = fa(1, i);
            mfma_all(a1, b1);
            mfma_all(a1, b0);
        }
        {
            xbf16x8 a0[TM], b2[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a0[i] = fa(0, i);
#pragma unroll
            for (int j = 0; j < TN; ++j) b2[j] = fb(2, j);
            mfma_all(a0, b2);
            mfma_all(a0, b1);
            mfma_all(a0, b0);
        }
        // the other buffer was last read in the previous step, before the barrier
        store(buf ^ 1, more);
        __syncthreads();
        buf ^= 1;
    }

    float* D = g.D + (int64_t)blockIdx.z * g.split_stride;
    double wacc = 0.0;
    // a tile wholly inside D (always, in the full 256 x 256 form: M and N are
    // multiples of 256) takes the form without per-element tests, so the
    // compiler issues its reads of X and Y together instead of one at a time
    // with a column list, the column of X each lane reads in block column j
    int64_t xcol[TN] = {};
    if constexpr (kCols)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            xcol[j] = n0 + wn * WTN + 32 * j + r;
            if (g.ncol && xcol[j] < g.N) xcol[j] = g.ncol[xcol[j]];
        }
    auto epilogue = [&](auto checked) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                // whole tiles: the sixteen reads of X (and Y) of a 32 x 32 block
                // before its stores, so they are issued together even where D
                // is X (U += dU in place: each element is read before it is
                // written, and blocks do not overlap)
                float xr[16], yr[16];
                if constexpr (!decltype(checked)::value && EPI != EPI_STORE && EPI != EPI_STORE_SQA) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int64_t row = m0 + wm * WTM + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                        const int64_t col = n0 + wn * WTN + 32 * j + r;
                        xr[v] = g.X[row * g.ldx + (kCols ? xcol[j] : col)];
                        if constexpr (EPI == EPI_ADD_DOT) yr[v] = g.Y[row * g.ldy + col];
                    }
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + wm * WTM + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                    const int64_t col = n0 + wn * WTN + 32 * j + r;
                    if (!decltype(checked)::value || (row < g.M && col < g.N)) {
                        const float x = acc[i][j][v];
                        if (EPI == EPI_STORE || EPI == EPI_STORE_SQA) {
                            D[row * g.ldd + col] = x;
                        } else if (EPI == kResidLate || EPI == EPI_RESID) {
                            const float xe =
                                decltype(checked)::value ? g.X[row * g.ldx + (kCols ? xcol[j] : col)] : xr[v];
                            const float e = xe - x;
                            if (EPI == EPI_RESID) D[row * g.ldd + col] = e;
                            wacc += (double)e * (double)e;
                        } else {
                            const float xe = decltype(checked)::value ? g.X[row * g.ldx + col] : xr[v];
                            const float ye = decltype(checked)::value ? g.Y[row * g.ldy + col] : yr[v];
                            D[row * g.ldd + col] = xe + x;
                            wacc += (double)x * (double)ye;
                        }
                    }
                }
            }
    };
    if ((FULL && BM == 256 && BN == 256) || (m0 + BM <= g.M && n0 + BN <= g.N))
        epilogue(std::false_type{});
    else
        epilogue(std::true_type{});
    if constexpr (EPI == EPI_STORE_SQA) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sqa += __shfl_xor(sqa, o, 64);
        if (lane == 0) red[wave] = sqa;
        __syncthreads();
        if (tid == 0) {
            double s2 = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s2 += red[w];
            g.wsum[blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)] = s2;
        }
    } else if constexpr (EPI != EPI_STORE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wacc += __shfl_xor(wacc, o, 64);
        if (lane == 0) red[wave] = wacc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            g.wsum[blockIdx.x + (int64_t)gridDim.x * blockIdx.y] = s;
        }
    }
}

// D[row][col] = sum_s P[s][row][col] in the order s = 0, 1, ...
__global__ __launch_bounds__(256) void k_splitk_reduce(const float* __restrict__ P, int splits, int64_t stride,
                                                       int64_t M, int64_t N, float* __restrict__ D, int64_t ldd) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        float s = P[e];
        for (int z = 1; z < splits; ++z) s += P[z * stride + e];
        const int64_t row = e / N, col = e - row * N;
        D[row * ldd + col] = s;
    }
}

// The same sum for a contiguous D (ldd = N), four elements per thread: P and D
// are 16-byte aligned and M N is a multiple of 4, so element e4 covers
// 4 e4 .. 4 e4 + 3 of every split with one vector load (same order of addition).
__global__ __launch_bounds__(256) void k_splitk_reduce_v4(const float4* __restrict__ P, int splits, int64_t stride4,
                                                          int64_t total4, float4* __restrict__ D) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total4; e += (int64_t)gridDim.x * 256) {
        float4 s = P[e];
        for (int z = 1; z < splits; ++z) {
            const float4 v = P[z * stride4 + e];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        D[e] = s;
    }
}

// The split-K sum with the EPI_RESID epilogue: D = X - sum_s P[s] in the order
// s = 0, 1, ...
__global__ __launch_bounds__(256) void k_splitk_reduce_sub(const float* __restrict__ P, int splits, int64_t stride,
                                                           int64_t M, int64_t N, float* __restrict__ D, int64_t ldd,
                                                           const float* __restrict__ X, int64_t ldx) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        float s = P[e];
        for (int z = 1; z < splits; ++z) s += P[z * stride + e];
        const int64_t row = e / N, col = e - row * N;
        D[row * ldd + col] = X[row * ldx + col] - s;
    }
}

// The split-K sum with the EPI_ADD_DOT epilogue: D = X + S, S = sum_s P[s] in
// the order s = 0, 1, ..., and wsum[block] = sum of S * Y over the block's
// elements (each thread's in order, then the threads in a fixed tree).
constexpr int kAddDotBlocks = 512;
__global__ __launch_bounds__(256) void k_splitk_reduce_add_dot(const float* __restrict__ P, int splits, int64_t stride,
                                                               int64_t M, int64_t N, float* D, int64_t ldd,
                                                               const float* X, int64_t ldx,
                                                               const float* __restrict__ Y, int64_t ldy,
                                                               double* __restrict__ wsum) {
    __shared__ double red[4];
    const int64_t total = M * N;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        float s = P[e];
        for (int z = 1; z < splits; ++z) s += P[z * stride + e];
        const int64_t row = e / N, col = e - row * N;
        D[row * ldd + col] = X[row * ldx + col] + s;
        acc += (double)s * (double)Y[row * ldy + col];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) wsum[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// k_splitk_reduce_sub and k_splitk_reduce_add_dot for contiguous D, X and Y
// (leading dimension N), four elements per thread with vector loads: sub
// writes D = X - S; add_dot writes D = X + S and wsum[block] = sum of S * Y
// (each thread's elements in order, then the threads in a fixed tree).
__global__ __launch_bounds__(256) void k_splitk_reduce_sub_v4(const float4* __restrict__ P, int splits,
                                                              int64_t stride4, int64_t total4,
                                                              float4* __restrict__ D, const float4* __restrict__ X) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total4; e += (int64_t)gridDim.x * 256) {
        float4 s = P[e];
        for (int z = 1; z < splits; ++z) {
            const float4 v = P[z * stride4 + e];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        const float4 x = X[e];
        D[e] = make_float4(x.x - s.x, x.y - s.y, x.z - s.z, x.w - s.w);
    }
}

__global__ __launch_bounds__(256) void k_splitk_reduce_add_dot_v4(const float4* __restrict__ P, int splits,
                                                                  int64_t stride4, int64_t total4, float4* D,
                                                                  const float4* X, const float4* __restrict__ Y,
                                                                  double* __restrict__ wsum) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total4; e += (int64_t)gridDim.x * 256) {
        float4 s = P[e];
        for (int z = 1; z < splits; ++z) {
            const float4 v = P[z * stride4 + e];
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        const float4 x = X[e], y = Y[e];
        D[e] = make_float4(x.x + s.x, x.y + s.y, x.z + s.z, x.w + s.w);
        acc += (double)s.x * (double)y.x;
        acc += (double)s.y * (double)y.y;
        acc += (double)s.z * (double)y.z;
        acc += (double)s.w * (double)y.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) wsum[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

bool contiguous_v4(int64_t M, int64_t N, const void* a, int64_t lda, const void* b, int64_t ldb, const void* c,
                   int64_t ldc, const void* d) {
    const auto al = [](const void* q) { return q == nullptr || ((uintptr_t)q & 15) == 0; };
    return (M * N) % 4 == 0 && lda == N && ldb == N && ldc == N && al(a) && al(b) && al(c) && al(d);
}

int64_t add_dot_blocks(int64_t M, int64_t N) {
    int64_t b = (M * N + 255) / 256;
    if (b > kAddDotBlocks) b = kAddDotBlocks;
    return b < 1 ? 1 : b;
}

struct Cfg {
    int BM, BN;
};
// Products large enough for the three-term BF16 split kernel (k_xgemm): the
// 256 x 256 tile for N >= 256 (at least 8e9 multiply-adds), the 128 x 128
// tile for the sketch widths 64 < N <= 128 and the 128 x 64 tile for
// 32 < N <= 64 (at least 1e9).
bool split_bf16_pays(int64_t M, int64_t N, int64_t K) {
    return M >= 256 && N >= 256 && K >= 256 && (double)M * (double)N * (double)K >= 8.0e9;
}
constexpr double kXNarrowMin = 1.0e9;   // multiply-adds of the smallest narrow product on the split tiles
bool split_bf16_narrow_pays(int64_t M, int64_t N, int64_t K) {
    return M >= 256 && N > 64 && N <= 128 && K >= 256 && (double)M * (double)N * (double)K >= kXNarrowMin;
}
bool split_bf16_narrow64_pays(int64_t M, int64_t N, int64_t K) {
    return M >= 256 && N > 32 && N <= 64 && K >= 256 && (double)M * (double)N * (double)K >= kXNarrowMin;
}
// tile configuration of a product with a fused epilogue (the norm-only
// residual, D = X - AB and D = X + AB; A not transposed)
int resid_cfg(int epi, int64_t M, int64_t N, int64_t K) {
    return (epi == EPI_RESID_NORM || epi == EPI_RESID || epi == EPI_ADD_DOT) && split_bf16_pays(M, N, K) ? 4 : 2;
}
// 0-3: FP32 MFMA tiles; 4, 6, 7: split-BF16 tiles (5, a 256 x 128 split tile of
// eight waves, measured slower than 6 for the sketch widths, is not used)
constexpr Cfg kCfg[8] = {{128, 64}, {128, 128}, {128, 128}, {256, 128}, {256, 256}, {256, 128}, {128, 128},
                         {128, 64}};
constexpr int kBK = 16;

template <int CFG, bool TA, int EPI>
hipError_t run(const GemmArgs& a, dim3 grid, hipStream_t st) {
    if constexpr (CFG == 0)
        hipLaunchKernelGGL((k_sgemm<128, 64, kBK, 4, 1, TA, EPI>), grid, dim3(256), 0, st, a);
    else if constexpr (CFG == 1)
        hipLaunchKernelGGL((k_sgemm<128, 128, kBK, 4, 1, TA, EPI>), grid, dim3(256), 0, st, a);
    else if constexpr (CFG == 2)
        hipLaunchKernelGGL((k_sgemm<128, 128, kBK, 2, 2, TA, EPI>), grid, dim3(256), 0, st, a);
    else if constexpr (CFG == 3)
        hipLaunchKernelGGL((k_sgemm<256, 128, kBK, 4, 2, TA, EPI>), grid, dim3(512), 0, st, a);
    else if constexpr (CFG == 4) {
        if (a.full)
            hipLaunchKernelGGL((k_xgemm<TA, EPI, true, 256, 256>), grid, dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((k_xgemm<TA, EPI, false, 256, 256>), grid, dim3(512), 0, st, a);
    } else if constexpr (CFG == 6) {
        if (a.full)
            hipLaunchKernelGGL((k_xgemm<TA, EPI, true, 128, 128>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_xgemm<TA, EPI, false, 128, 128>), grid, dim3(256), 0, st, a);
    } else {
        if (a.full)
            hipLaunchKernelGGL((k_xgemm<TA, EPI, true, 128, 64>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_xgemm<TA, EPI, false, 128, 64>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

GemmPlan plan_sgemm(int64_t M, int64_t N, int64_t K, bool transA, bool allow_split) {
    GemmPlan p;
    p.cfg = N <= 64 ? 0 : (N <= 128 ? 1 : 2);
    // wide products with A transposed, more than 128 rows and a long K
    // (H = C^T A): 256 x 128 tiles of eight waves, so the long operand is streamed
    // half as often; the split-K target counts workgroups of eight waves
    if (transA && M > 128 && N > 128 && K >= 2048) p.cfg = 3;
    if (split_bf16_pays(M, N, K)) p.cfg = 4;
    if (split_bf16_narrow_pays(M, N, K)) p.cfg = 6;
    if (split_bf16_narrow64_pays(M, N, K)) p.cfg = 7;
    const int64_t tiles = ((M + kCfg[p.cfg].BM - 1) / kCfg[p.cfg].BM) * ((N + kCfg[p.cfg].BN - 1) / kCfg[p.cfg].BN);
    const int64_t target = p.cfg >= 3 ? 256 : 512;
    int64_t splits = 1;
    if (p.cfg >= 3 && allow_split) {
        // a workgroup of eight waves fills a compute unit (two of the 128 x 128
        // split tile's four): pick the split count that minimises (rounds of
        // resident workgroups) x (K per workgroup + a fixed cost of about 64 K
        // steps), so no round runs mostly empty
        const int64_t round = p.cfg >= 6 ? 512 : 256;
        const int64_t maxs = std::max<int64_t>(1, K / (4 * kBK));
        int64_t best = -1;
        for (int64_t s = 1; s <= maxs; ++s) {
            const int64_t kc = ((K + s - 1) / s + kBK - 1) / kBK * kBK;
            const int64_t cost = ((tiles * s + round - 1) / round) * (kc + 64);
            if (best < 0 || cost < best) {
                best = cost;
                splits = s;
            }
        }
    } else if (allow_split && tiles < target - 32) {
        splits = (target + tiles - 1) / tiles;
        const int64_t maxs = K / (4 * kBK);
        if (splits > maxs) splits = maxs;
        if (splits < 1) splits = 1;
    }
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = ((kchunk + kBK - 1) / kBK) * kBK;
    if (kchunk < kBK) kchunk = kBK;
    splits = (K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    p.splits = (int)splits;
    p.kchunk = kchunk;
    p.wgs = tiles * splits;
    return p;
}

size_t sgemm_partial_floats(const GemmPlan& p, int64_t M, int64_t N) {
    return p.splits > 1 ? (size_t)p.splits * (size_t)M * (size_t)N : 0;
}

GemmPlan plan_sgemm_within(int64_t M, int64_t N, int64_t K, bool transA, size_t cap_floats) {
    GemmPlan p = plan_sgemm(M, N, K, transA, true);
    if (sgemm_partial_floats(p, M, N) <= cap_floats) return p;
    const int64_t most = std::max<int64_t>(1, (int64_t)(cap_floats / ((size_t)M * (size_t)N)));
    int64_t kchunk = (K + most - 1) / most;
    kchunk = std::max<int64_t>(kBK, (kchunk + kBK - 1) / kBK * kBK);
    const int64_t splits = std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
    p.splits = (int)splits;
    p.kchunk = kchunk;
    const Cfg c = kCfg[p.cfg];
    p.wgs = ((M + c.BM - 1) / c.BM) * ((N + c.BN - 1) / c.BN) * splits;
    return p;
}

hipError_t launch_sgemm_main(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A,
                             int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd, float* partial, int epi,
                             const float* X, int64_t ldx, const float* Y, int64_t ldy, double* wsum, hipStream_t st,
                             const int* ncol) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const bool store_like = epi == EPI_STORE || epi == EPI_STORE_SQA;
    if (ncol && (epi != EPI_RESID_NORM || transA || !resid_cols_ok(M, N, K))) return hipErrorInvalidValue;
    if (!store_like && p.splits != 1) return hipErrorInvalidValue;
    if (epi == EPI_STORE_SQA && transA) return hipErrorInvalidValue;
    GemmArgs a;
    a.M = M;
    a.N = N;
    a.K = K;
    a.A = A;
    a.lda = lda;
    a.B = B;
    a.ldb = ldb;
    a.kchunk = p.kchunk;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.wsum = wsum;
    a.swz = 0;
    a.full = false;
    a.ncol = ncol;
    if (p.splits > 1) {
        a.D = partial;
        a.ldd = N;
        a.split_stride = M * N;
    } else {
        a.D = D;
        a.ldd = ldd;
        a.split_stride = 0;
    }
    // the fused epilogues run on the square FP32 tile (a 256 x 128 residual tile
    // measured slower: 202 us against 192 us for the residual A - C U at 8192 x
    // 4096 x 256), the norm-only residual of a large product on the split-BF16 tile
    const int cfg = store_like ? p.cfg : resid_cfg(epi, M, N, K);
    const Cfg c = kCfg[cfg];
    a.tm = (M + c.BM - 1) / c.BM;
    a.tn = (N + c.BN - 1) / c.BN;
    dim3 grid((unsigned)a.tm, (unsigned)a.tn, (unsigned)p.splits);
    // XCD-compact tile order for the big square-tile products
    if ((cfg == 2 || cfg == 4) && a.tm % 64 == 0 && a.tn % 8 == 0) a.swz = 1;
    if (a.swz) grid = dim3((unsigned)(a.tm * a.tn), 1, (unsigned)p.splits);
    a.full = (cfg == 4 ? N % 256 == 0 : cfg >= 5 && N % 2 == 0) && M % kCfg[cfg].BM == 0 &&
             K % kBK == 0 &&
             p.kchunk % kBK == 0 &&
             lda <= kXFullMaxLd && ldb <= kXFullMaxLd && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0 &&
             lda % 4 == 0 && ldb % 4 == 0;
    hipError_t e;
    switch (cfg * 100 + (transA ? 10 : 0) + epi) {
        case 0: e = run<0, false, EPI_STORE>(a, grid, st); break;
        case 10: e = run<0, true, EPI_STORE>(a, grid, st); break;
        case 100: e = run<1, false, EPI_STORE>(a, grid, st); break;
        case 110: e = run<1, true, EPI_STORE>(a, grid, st); break;
        case 200: e = run<2, false, EPI_STORE>(a, grid, st); break;
        case 210: e = run<2, true, EPI_STORE>(a, grid, st); break;
        case 310: e = run<3, true, EPI_STORE>(a, grid, st); break;
        case 400: e = run<4, false, EPI_STORE>(a, grid, st); break;
        case 410: e = run<4, true, EPI_STORE>(a, grid, st); break;
        case 404: e = run<4, false, EPI_STORE_SQA>(a, grid, st); break;
        case 403: e = run<4, false, kResidLate>(a, grid, st); break;
        case 401: e = run<4, false, EPI_RESID>(a, grid, st); break;
        case 402: e = run<4, false, EPI_ADD_DOT>(a, grid, st); break;
        case 600: e = run<6, false, EPI_STORE>(a, grid, st); break;
        case 610: e = run<6, true, EPI_STORE>(a, grid, st); break;
        case 604: e = run<6, false, EPI_STORE_SQA>(a, grid, st); break;
        case 700: e = run<7, false, EPI_STORE>(a, grid, st); break;
        case 710: e = run<7, true, EPI_STORE>(a, grid, st); break;
        case 704: e = run<7, false, EPI_STORE_SQA>(a, grid, st); break;
        case 4: e = run<0, false, EPI_STORE_SQA>(a, grid, st); break;
        case 104: e = run<1, false, EPI_STORE_SQA>(a, grid, st); break;
        case 204: e = run<2, false, EPI_STORE_SQA>(a, grid, st); break;
        case 201: e = run<2, false, EPI_RESID>(a, grid, st); break;
        case 203:
            e = K >= 1024 ? run<2, false, kResidLate>(a, grid, st) : run<2, false, EPI_RESID_NORM>(a, grid, st);
            break;
        case 202: e = run<2, false, EPI_ADD_DOT>(a, grid, st); break;
        case 212: e = run<2, true, EPI_ADD_DOT>(a, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return e;
}

hipError_t launch_splitk_reduce(const GemmPlan& p, int64_t M, int64_t N, const float* partial, float* D, int64_t ldd,
                                hipStream_t st) {
    if (p.splits <= 1 || M <= 0 || N <= 0) return hipSuccess;
    if (ldd == N && (M * N) % 4 == 0 && ((uintptr_t)partial & 15) == 0 && ((uintptr_t)D & 15) == 0) {
        const int64_t total4 = M * N / 4;
        int64_t blocks = (total4 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_splitk_reduce_v4, dim3((unsigned)blocks), dim3(256), 0, st,
                           reinterpret_cast<const float4*>(partial), p.splits, total4, total4,
                           reinterpret_cast<float4*>(D));
        return hipGetLastError();
    }
    int64_t blocks = (M * N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, st, partial, p.splits, M * N, M, N, D,
                       ldd);
    return hipGetLastError();
}

bool resid_cols_ok(int64_t M, int64_t N, int64_t K) {
    return resid_cfg(EPI_RESID_NORM, M, N, K) == 4;
}

int64_t resid_rounds(int64_t M, int64_t N, int64_t K) {
    return (resid_parts(M, N, K) + 255) / 256;
}

int64_t resid_parts(int64_t M, int64_t N, int64_t K) {
    const Cfg c = kCfg[resid_cfg(EPI_RESID_NORM, M, N, K)];
    return ((M + c.BM - 1) / c.BM) * ((N + c.BN - 1) / c.BN);
}

int64_t resid_parts_max(int64_t M, int64_t N) {
    const Cfg c = kCfg[2];   // the smaller of the two residual tiles
    return ((M + c.BM - 1) / c.BM) * ((N + c.BN - 1) / c.BN);
}

int64_t resid_store_parts(int64_t M, int64_t N) {
    return ((M + kCfg[2].BM - 1) / kCfg[2].BM) * ((N + kCfg[2].BN - 1) / kCfg[2].BN);
}

int64_t add_dot_parts(const GemmPlan& p, int64_t M, int64_t N, int64_t K) {
    if (p.splits > 1) return add_dot_blocks(M, N);
    const Cfg c = kCfg[resid_cfg(EPI_ADD_DOT, M, N, K)];
    return ((M + c.BM - 1) / c.BM) * ((N + c.BN - 1) / c.BN);
}

int64_t add_dot_parts_max(int64_t M, int64_t N) {
    return std::max<int64_t>(kAddDotBlocks, ((M + kCfg[2].BM - 1) / kCfg[2].BM) * ((N + kCfg[2].BN - 1) / kCfg[2].BN));
}

hipError_t launch_sgemm_add_dot(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A,
                                int64_t lda, const float* B, int64_t ldb, float* D, int64_t ldd, float* partial,
                                const float* X, int64_t ldx, const float* Y, int64_t ldy, double* wsum, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (p.splits <= 1)
        return launch_sgemm_main(p, M, N, K, transA, A, lda, B, ldb, D, ldd, partial, EPI_ADD_DOT, X, ldx, Y, ldy,
                                 wsum, st);
    const hipError_t e = launch_sgemm_main(p, M, N, K, transA, A, lda, B, ldb, D, ldd, partial, EPI_STORE, nullptr, 0,
                                           nullptr, 0, nullptr, st);
    if (e != hipSuccess) return e;
    if (contiguous_v4(M, N, D, ldd, X, ldx, Y, ldy, partial)) {
        const int64_t total4 = M * N / 4;
        hipLaunchKernelGGL(k_splitk_reduce_add_dot_v4, dim3((unsigned)add_dot_blocks(M, N)), dim3(256), 0, st,
                           reinterpret_cast<const float4*>(partial), p.splits, total4, total4,
                           reinterpret_cast<float4*>(D), reinterpret_cast<const float4*>(X),
                           reinterpret_cast<const float4*>(Y), wsum);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_splitk_reduce_add_dot, dim3((unsigned)add_dot_blocks(M, N)), dim3(256), 0, st, partial,
                       p.splits, M * N, M, N, D, ldd, X, ldx, Y, ldy, wsum);
    return hipGetLastError();
}

hipError_t launch_sgemm(const GemmPlan& p, int64_t M, int64_t N, int64_t K, bool transA, const float* A, int64_t lda,
                        const float* B, int64_t ldb, float* D, int64_t ldd, float* partial, int epi, const float* X,
                        int64_t ldx, const float* Y, int64_t ldy, double* wsum, hipStream_t st) {
    if (epi == EPI_RESID && p.splits > 1) {
        // D = X - A B split over K: partial products, then the subtracting sum
        // (no sum of squares: wsum is not written on this path)
        if (M <= 0 || N <= 0) return hipSuccess;
        const hipError_t e = launch_sgemm_main(p, M, N, K, transA, A, lda, B, ldb, D, ldd, partial, EPI_STORE,
                                               nullptr, 0, nullptr, 0, nullptr, st);
        if (e != hipSuccess) return e;
        if (contiguous_v4(M, N, D, ldd, X, ldx, partial, N, nullptr)) {
            const int64_t total4 = M * N / 4;
            int64_t blocks = (total4 + 255) / 256;
            if (blocks > 8192) blocks = 8192;
            hipLaunchKernelGGL(k_splitk_reduce_sub_v4, dim3((unsigned)blocks), dim3(256), 0, st,
                               reinterpret_cast<const float4*>(partial), p.splits, total4, total4,
                               reinterpret_cast<float4*>(D), reinterpret_cast<const float4*>(X));
            return hipGetLastError();
        }
        int64_t blocks = (M * N + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_splitk_reduce_sub, dim3((unsigned)blocks), dim3(256), 0, st, partial, p.splits, M * N, M,
                           N, D, ldd, X, ldx);
        return hipGetLastError();
    }
    const hipError_t e = launch_sgemm_main(p, M, N, K, transA, A, lda, B, ldb, D, ldd, partial, epi, X, ldx, Y, ldy,
                                           wsum, st);
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(p, M, N, partial, D, ldd, st);
}

}  // namespace bcur
