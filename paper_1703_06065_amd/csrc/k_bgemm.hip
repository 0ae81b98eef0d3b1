// BF16 sketch passes on the CDNA4 matrix cores (v_mfma_f32_32x32x16_bf16,
// FP32 accumulation).  Both operands are stored with k contiguous ("NT"):
// D (M x N, FP32) = A (M x K, bf16) * B^T, B stored N x K (bf16).  A tile
// row of 64 k values is 128 bytes; each lane's MFMA operand is 8 consecutive
// k values, one 16-byte LDS read.  The passes are bound by HBM latency (a
// sketch product has few tiles), so each step stages 64 k: four 16-byte
// loads of A and four of B per thread in flight behind the step's MFMAs
// (542 -> 452 us a pass at 65536 x 16384, l = 110, against 32 k a step; 128 k
// measured no better).  Split-K partial tiles are summed in a
// fixed order by the FP32 GEMM's reduction kernel.
//
// Also here: the casts that produce the k-contiguous operands:
//   A (m x n, f32) -> A_bf (m x n) and A_bf^T (n x m), one tiled pass;
//   X (rows x l, f32) -> X_bf^T (l x rows) for the sketch panels.
#include "bcur_internal.h"

namespace bcur {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// out (m x n, ldo) = bf16(A); outT (n x m, ldt) = bf16(A)^T, through 64 x 64 LDS tiles; the
// grid covers the tiles from row rb and column cb on.
__global__ __launch_bounds__(256) void k_cast_bf16_both(const float* __restrict__ A, int64_t m, int64_t n,
                                                        int64_t lda, uint16_t* __restrict__ out, int64_t ldo,
                                                        uint16_t* __restrict__ outT, int64_t ldt, int64_t rb,
                                                        int64_t cb) {
    __shared__ uint16_t tile[64][66];
    const int64_t r0 = rb + (int64_t)blockIdx.y * 64, c0 = cb + (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        uint16_t v = 0;
        if (r < m && c < n) {
            v = bf16_rne(A[r * lda + c]);
            if (out) out[r * ldo + c] = v;
        }
        tile[i][tx] = v;
    }
    __syncthreads();
    if (!outT) return;
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (c < n && r < m) outT[c * ldt + r] = tile[tx][i];
    }
}

// The same casts for a whole 64 x 64 tile inside A with lda, ldo and ldt
// multiples of 4 and 16-byte aligned A (8-byte aligned outputs): each thread
// loads 4 consecutive floats of a row (one 16-byte load) and stores their 4
// BF16 values with one 8-byte store to out; the transposed tile goes out
// from LDS as 4 consecutive rows of one column per thread (one 8-byte store).
__global__ __launch_bounds__(256) void k_cast_bf16_both_v4(const float* __restrict__ A, int64_t lda,
                                                           uint16_t* __restrict__ out, int64_t ldo,
                                                           uint16_t* __restrict__ outT, int64_t ldt) {
    __shared__ uint16_t tile[64][68];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    // the four 16-byte reads first (issued together), then the casts and stores
    float4 va[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) va[i] = *reinterpret_cast<const float4*>(A + (r0 + ty + 16 * i) * lda + c0 + 4 * tx);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = ty + 16 * i;
        const float4 v = va[i];
        const uint16_t b0 = bf16_rne(v.x), b1 = bf16_rne(v.y), b2 = bf16_rne(v.z), b3 = bf16_rne(v.w);
        if (out) {
            uint2 pk;
            pk.x = b0 | ((uint32_t)b1 << 16);
            pk.y = b2 | ((uint32_t)b3 << 16);
            *reinterpret_cast<uint2*>(out + (r0 + row) * ldo + c0 + 4 * tx) = pk;
        }
        tile[row][4 * tx + 0] = b0;
        tile[row][4 * tx + 1] = b1;
        tile[row][4 * tx + 2] = b2;
        tile[row][4 * tx + 3] = b3;
    }
    if (!outT) return;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int col = ty + 16 * i;
        uint2 pk;
        pk.x = tile[4 * tx + 0][col] | ((uint32_t)tile[4 * tx + 1][col] << 16);
        pk.y = tile[4 * tx + 2][col] | ((uint32_t)tile[4 * tx + 3][col] << 16);
        *reinterpret_cast<uint2*>(outT + (c0 + col) * ldt + r0 + 4 * tx) = pk;
    }
}

struct BArgs {
    int64_t M, N, K;
    const uint16_t* A;
    int64_t lda;
    const uint16_t* B;
    int64_t ldb;
    float* D;
    int64_t ldd;
    int64_t kchunk;
    int64_t split_stride;
};

// 8 bf16 (16 bytes) at p[0..7] when 16-byte aligned and in range, else
// element-wise with zeros outside [c, cend).
__device__ __forceinline__ uint4 ld8(const uint16_t* p, bool rowok, int64_t c, int64_t cend) {
    if (rowok && c + 7 < cend) return *reinterpret_cast<const uint4*>(p);
    uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (rowok)
        for (int e = 0; e < 8; ++e)
            if (c + e < cend) v[e] = p[e];
    uint4 r;
    r.x = v[0] | ((uint32_t)v[1] << 16);
    r.y = v[2] | ((uint32_t)v[3] << 16);
    r.z = v[4] | ((uint32_t)v[5] << 16);
    r.w = v[6] | ((uint32_t)v[7] << 16);
    return r;
}

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void k_bgemm_nt(const BArgs g) {
    constexpr int BK = 64;                 // k per LDS stage
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    constexpr int LDS_ROW = BK + 8;        // bf16 per LDS row (144 bytes: spreads banks)
    constexpr int A_V = BM * BK / 8 / NT;  // 16-byte vectors per thread
    constexpr int B_V = BN * BK / 8 / NT;
    static_assert(TM >= 1 && TN >= 1 && A_V >= 1 && B_V >= 1, "tile shape");
    __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDS_ROW];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDS_ROW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    uint4 ra[A_V], rb[B_V];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < A_V; ++u) {
            const int f = tid + u * NT, row = f / (BK / 8), kq = f % (BK / 8);
            const int64_t gm = m0 + row, gk = k0 + kq * 8;
            ra[u] = ld8(g.A + gm * g.lda + gk, gm < g.M, gk, kend);
        }
#pragma unroll
        for (int u = 0; u < B_V; ++u) {
            const int f = tid + u * NT, row = f / (BK / 8), kq = f % (BK / 8);
            const int64_t gn = n0 + row, gk = k0 + kq * 8;
            rb[u] = ld8(g.B + gn * g.ldb + gk, gn < g.N, gk, kend);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < A_V; ++u) {
            const int f = tid + u * NT, row = f / (BK / 8), kq = f % (BK / 8);
            *reinterpret_cast<uint4*>(&As[row * LDS_ROW + kq * 8]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B_V; ++u) {
            const int f = tid + u * NT, row = f / (BK / 8), kq = f % (BK / 8);
            *reinterpret_cast<uint4*>(&Bs[row * LDS_ROW + kq * 8]) = rb[u];
        }
    };

    int64_t k0 = kbeg;
    if (k0 < kend) load(k0);
    for (; k0 < kend; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8 a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * WTM + 32 * i + r) * LDS_ROW + kk + 8 * h]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * WTN + 32 * j + r) * LDS_ROW + kk + 8 * h]);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    float* D = g.D + (int64_t)blockIdx.z * g.split_stride;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = m0 + wm * WTM + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                const int64_t col = n0 + wn * WTN + 32 * j + r;
                if (row < g.M && col < g.N) D[row * g.ldd + col] = acc[i][j][v];
            }
}

}  // namespace

hipError_t launch_cast_bf16_both(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out, int64_t ldo,
                                 uint16_t* outT, int64_t ldt, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const bool vec = ((uintptr_t)A & 15) == 0 && (lda & 3) == 0 && ((uintptr_t)out & 7) == 0 && (ldo & 3) == 0 &&
                     ((uintptr_t)outT & 7) == 0 && (ldt & 3) == 0;
    const int64_t m64 = vec ? m / 64 * 64 : 0, n64 = vec ? n / 64 * 64 : 0;
    if (m64 > 0 && n64 > 0) {
        hipLaunchKernelGGL(k_cast_bf16_both_v4, dim3((unsigned)(n64 / 64), (unsigned)(m64 / 64)), dim3(256), 0, st, A,
                           lda, out, ldo, outT, ldt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the rest: columns n64 .. n-1 of every row, then rows m64 .. m-1 of columns 0 .. n64-1
    const int64_t mm = (m64 > 0 && n64 > 0) ? m64 : 0, nn = (m64 > 0 && n64 > 0) ? n64 : 0;
    if (nn < n) {
        dim3 grid((unsigned)((n - nn + 63) / 64), (unsigned)((m + 63) / 64));
        hipLaunchKernelGGL(k_cast_bf16_both, grid, dim3(256), 0, st, A, m, n, lda, out, ldo, outT, ldt, (int64_t)0,
                           nn);
    }
    if (mm < m && nn > 0) {
        dim3 grid((unsigned)(nn / 64), (unsigned)((m - mm + 63) / 64));
        hipLaunchKernelGGL(k_cast_bf16_both, grid, dim3(256), 0, st, A, m, nn, lda, out, ldo, outT, ldt, mm,
                           (int64_t)0);
    }
    return hipGetLastError();
}

GemmPlan plan_bgemm(int64_t M, int64_t N, int64_t K) {
    GemmPlan p;
    p.cfg = N <= 64 ? 0 : 1;
    const int64_t BM = 128, BN = N <= 64 ? 64 : 128;
    const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    int64_t splits = 1;
    if (tiles < 480) {
        // the HBM-bound passes need many loads in flight: products that are
        // split anyway and have a long K (A^T Z: 65536 rows) aim at 2048
        // workgroups (3.69 against 4.02 ms at 65536 x 16384, l = 110); a grid
        // already near 512 tiles (A Q) gains nothing from splitting
        const int64_t target = K >= 8192 ? 2048 : 512;
        splits = (target + tiles - 1) / tiles;
        const int64_t maxs = K / 256;
        if (splits > maxs) splits = maxs;
        if (splits < 1) splits = 1;
    }
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = ((kchunk + 63) / 64) * 64;
    splits = (K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    p.splits = (int)splits;
    p.kchunk = kchunk;
    p.wgs = tiles * splits;
    return p;
}

hipError_t launch_bgemm_nt(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda,
                           const uint16_t* B, int64_t ldb, float* D, int64_t ldd, float* partial, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    BArgs a;
    a.M = M;
    a.N = N;
    a.K = K;
    a.A = A;
    a.lda = lda;
    a.B = B;
    a.ldb = ldb;
    a.kchunk = p.kchunk;
    if (p.splits > 1) {
        a.D = partial;
        a.ldd = N;
        a.split_stride = M * N;
    } else {
        a.D = D;
        a.ldd = ldd;
        a.split_stride = 0;
    }
    if (p.cfg == 0) {
        dim3 grid((unsigned)((M + 127) / 128), (unsigned)((N + 63) / 64), (unsigned)p.splits);
        hipLaunchKernelGGL((k_bgemm_nt<128, 64, 4, 1>), grid, dim3(256), 0, st, a);
    } else {
        dim3 grid((unsigned)((M + 127) / 128), (unsigned)((N + 127) / 128), (unsigned)p.splits);
        hipLaunchKernelGGL((k_bgemm_nt<128, 128, 4, 1>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace bcur
