// Bandwidth-bound kernels of the Block CUR path: the Frobenius norm, block
// leverage scores, block sampling, gathers and small utilities.
#include <math.h>

#include <algorithm>

#include "bcur_internal.h"

namespace bcur {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup in a fixed tree order; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) r += sh[i];
    }
    return r;
}

__device__ __forceinline__ double sq4(float4 v) {
    const double x = v.x, y = v.y, z = v.z, w = v.w;
    return (x * x + y * y) + (z * z + w * w);
}

// ||A||_F^2 partial sums: one double per workgroup, fixed order per thread.
__global__ __launch_bounds__(256) void k_frob2_partial(const float* __restrict__ A, int64_t m, int64_t n,
                                                       int64_t lda, double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    const int tid = threadIdx.x;
    if (lda == n && (n & 3) == 0) {
        // dense rows: the matrix is one contiguous run of m*n floats
        const float4* A4 = reinterpret_cast<const float4*>(A);
        const int64_t total4 = m * n / 4;
        const int64_t stride = (int64_t)gridDim.x * 256;
        int64_t i = (int64_t)blockIdx.x * 256 + tid;
        for (; i + 3 * stride < total4; i += 4 * stride) {
            const float4 v0 = A4[i], v1 = A4[i + stride], v2 = A4[i + 2 * stride], v3 = A4[i + 3 * stride];
            acc0 += sq4(v0);
            acc1 += sq4(v1);
            acc2 += sq4(v2);
            acc3 += sq4(v3);
        }
        for (; i < total4; i += stride) acc0 += sq4(A4[i]);
    } else {
        for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
            const float* a = A + row * lda;
            if ((lda & 3) == 0) {
                const int64_t n4 = n >> 2;
                const float4* a4 = reinterpret_cast<const float4*>(a);
                for (int64_t j = tid; j < n4; j += 256) acc0 += sq4(a4[j]);
                for (int64_t j = n4 * 4 + tid; j < n; j += 256) {
                    const double x = a[j];
                    acc1 += x * x;
                }
            } else {
                for (int64_t j = tid; j < n; j += 256) {
                    const double x = a[j];
                    acc1 += x * x;
                }
            }
        }
    }
    const double r = block_sum<256>((acc0 + acc1) + (acc2 + acc3), sh);
    if (tid == 0) partial[blockIdx.x] = r;
}

// out[0] = sum of x[0..count) in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_sum_f64(const double* __restrict__ x, int64_t count,
                                                 double* __restrict__ out) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) acc += x[i];
    const double r = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) out[0] = r;
}

// Def. 2: scores[g] = sum of squares of rows off[g]..off[g+1]-1 of V (n x k, ldv).
__global__ __launch_bounds__(256) void k_block_scores(const float* __restrict__ V, int64_t k, int64_t ldv,
                                                      const int64_t* __restrict__ off,
                                                      double* __restrict__ scores) {
    __shared__ double sh[4];
    const int64_t g = blockIdx.x;
    const int64_t r0 = off[g], r1 = off[g + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (ldv == k) {
        // the block's rows are one contiguous run: 16-byte loads from the first
        // 16-byte boundary on, the few elements before it and after the last
        // whole float4 one by one; four independent FP64 sums per thread
        const float* base = V + r0 * k;
        const int64_t cnt = (r1 - r0) * k;
        const int64_t head = min<int64_t>((int64_t)((16 - ((uintptr_t)base & 15)) & 15) / 4, cnt);
        if (threadIdx.x < head) {
            const double x = base[threadIdx.x];
            a0 += x * x;
        }
        const float4* b4 = reinterpret_cast<const float4*>(base + head);
        const int64_t n4 = (cnt - head) / 4;
        for (int64_t e = threadIdx.x; e < n4; e += 256) {
            const float4 v = b4[e];
            const double x = v.x, y = v.y, z = v.z, w = v.w;
            a0 += x * x;
            a1 += y * y;
            a2 += z * z;
            a3 += w * w;
        }
        const int64_t t = head + 4 * n4 + threadIdx.x;
        if (t < cnt) {
            const double x = base[t];
            a1 += x * x;
        }
    } else {
        const int64_t cnt = (r1 - r0) * k;
        for (int64_t e = threadIdx.x; e < cnt; e += 256) {
            const int64_t r = e / k, c = e - r * k;
            const double x = V[(r0 + r) * ldv + c];
            a0 += x * x;
        }
    }
    const double r = block_sum<256>((a0 + a1) + (a2 + a3), sh);
    if (threadIdx.x == 0) scores[g] = r;
}

__device__ __forceinline__ int ceil_log2_i64(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) ++r;
    return r;
}

constexpr int kSampleLds = 4096;   // blocks whose weights the sampler keeps in LDS

// Alg. 1 step 2 with exact integer weights (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_sample(const double* __restrict__ scores, int64_t G,
                                                 const uint64_t* __restrict__ draws, int64_t s, int replace,
                                                 uint64_t* __restrict__ qbuf, uint64_t* __restrict__ pref,
                                                 int64_t* __restrict__ idx, double* __restrict__ weights,
                                                 double* __restrict__ margins, int* __restrict__ status) {
    __shared__ uint64_t scan[1024];
    __shared__ double smax[16];
    __shared__ int sbad[16];
    __shared__ uint64_t lq[kSampleLds], lp[kSampleLds], lr[kSampleLds];
    __shared__ int ltaken[kSampleLds];
    const int tid = threadIdx.x;

    // 1. largest score and validity
    double mx = 0.0;
    int bad = 0;
    for (int64_t g = tid; g < G; g += 1024) {
        const double x = scores[g];
        if (!(x >= 0.0) || !isfinite(x)) bad = 1;
        else mx = fmax(mx, x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if ((tid & 63) == 0) {
        smax[tid >> 6] = mx;
        sbad[tid >> 6] = bad;
    }
    __syncthreads();
    mx = 0.0;
    bad = 0;
    for (int i = 0; i < 16; ++i) {
        mx = fmax(mx, smax[i]);
        bad |= sbad[i];
    }
    if (bad) {
        if (tid == 0) status[0] = 1;
        return;
    }
    int sh = 0;
    if (mx > 0.0) {
        int E;
        frexp(mx, &E);
        sh = 62 - ceil_log2_i64(G) - E;
    }

    // 2. q_g = floor(l_g 2^sh) and their inclusive prefix sums
    uint64_t carry = 0;
    for (int64_t base = 0; base < G; base += 1024) {
        const int64_t g = base + tid;
        uint64_t v = 0;
        if (g < G && mx > 0.0) v = (uint64_t)floor(ldexp(scores[g], sh));
        if (g < G) qbuf[g] = v;
        scan[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint64_t add = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        if (g < G) {
            pref[g] = carry + scan[tid];
            if (G <= kSampleLds) {
                lq[g] = v;
                lp[g] = carry + scan[tid];
            }
        }
        const uint64_t tot = scan[1023];
        __syncthreads();
        carry += tot;
    }
    __syncthreads();

    // 3. the draws, one after the other.  When the weights fit in LDS every
    // thread tests its blocks for the unique j with f(j-1) <= x < f(j), where
    // f(j) = pref[j] - (weight already removed at indices <= j) is kept as an
    // LDS prefix of removed weight; otherwise thread 0 walks global memory.
    const uint64_t total = pref[G - 1];
    if (G <= kSampleLds) {
        __shared__ uint64_t s_W, s_x, s_removed;
        __shared__ int64_t s_j;
        __shared__ int s_zero;
        for (int64_t g = tid; g < G; g += 1024) {
            lr[g] = 0;
            ltaken[g] = 0;
        }
        if (tid == 0) {
            s_removed = 0;
            s_zero = 0;
        }
        __syncthreads();
        for (int64_t t = 0; t < s; ++t) {
            if (tid == 0) {
                const uint64_t W = total - s_removed;
                s_W = W;
                s_x = W ? __umul64hi(draws[t], W) : 0;
                s_j = G;
            }
            __syncthreads();
            const uint64_t W = s_W, x = s_x;
            if (W == 0) {
                // every remaining weight is zero: the smallest remaining index
                for (int64_t g = tid; g < G; g += 1024)
                    if (!ltaken[g]) atomicMin((unsigned long long*)&s_j, (unsigned long long)g);
            } else {
                for (int64_t g = tid; g < G; g += 1024) {
                    const uint64_t f = lp[g] - lr[g];
                    const uint64_t fp = g ? lp[g - 1] - lr[g - 1] : 0;
                    if (f > x && fp <= x) s_j = g;
                }
            }
            __syncthreads();
            const int64_t j = s_j;
            if (tid == 0) {
                double margin = 0.0;
                if (W != 0) {
                    const uint64_t fj = lp[j] - lr[j];
                    const uint64_t lo_edge = fj - lq[j];
                    const uint64_t a = x - lo_edge, b = fj - 1 - x;
                    margin = ldexp((double)(a < b ? a : b), -sh);
                } else {
                    s_zero = 1;
                }
                idx[t] = j;
                if (margins) margins[t] = margin;
                if (weights) weights[t] = lq[j] == 0 ? INFINITY : sqrt((double)total / ((double)s * (double)lq[j]));
                if (!replace) {
                    s_removed += lq[j];
                    ltaken[j] = 1;
                }
            }
            if (!replace) {
                const uint64_t qj = lq[j];
                for (int64_t g = j + tid; g < G; g += 1024) lr[g] += qj;
            }
            __syncthreads();
        }
        if (tid == 0) {
            status[0] = 0;
            status[1] = s_zero;
        }
        return;
    }
    if (tid == 0) {
        int zero_drawn = 0;
        for (int64_t t = 0; t < s; ++t) {
            uint64_t removed = 0;
            if (!replace)
                for (int64_t u = 0; u < t; ++u) removed += qbuf[idx[u]];
            const uint64_t W = total - removed;
            int64_t j;
            double margin = 0.0;
            if (W == 0) {
                j = 0;
                for (;;) {
                    bool taken = false;
                    if (!replace)
                        for (int64_t u = 0; u < t; ++u) taken |= (idx[u] == j);
                    if (!taken) break;
                    ++j;
                }
                zero_drawn = 1;
            } else {
                const uint64_t x = __umul64hi(draws[t], W);
                int64_t lo = 0, hi = G - 1;
                while (lo < hi) {
                    const int64_t mid = lo + ((hi - lo) >> 1);
                    uint64_t f = pref[mid];
                    if (!replace)
                        for (int64_t u = 0; u < t; ++u)
                            if (idx[u] <= mid) f -= qbuf[idx[u]];
                    if (f > x) hi = mid;
                    else lo = mid + 1;
                }
                j = lo;
                uint64_t fj = pref[j];
                if (!replace)
                    for (int64_t u = 0; u < t; ++u)
                        if (idx[u] <= j) fj -= qbuf[idx[u]];
                const uint64_t lo_edge = fj - qbuf[j];
                const uint64_t a = x - lo_edge, b = fj - 1 - x;
                margin = ldexp((double)(a < b ? a : b), -sh);
            }
            idx[t] = j;
            if (margins) margins[t] = margin;
            if (weights) {
                const uint64_t qj = qbuf[j];
                weights[t] = qj == 0 ? INFINITY : sqrt((double)total / ((double)s * (double)qj));
            }
        }
        status[0] = 0;
        status[1] = zero_drawn;
    }
}

// The column (row) list of s chosen blocks of equal width b drawn without
// replacement: out[t b + i] = map[off[idx[t]] + i] (map null: the identity).
// A block index outside [0, G) (the sampler did not run on valid scores) is
// read as block 0, so every later access stays in bounds; the host rejects
// such a result after its synchronization.
// ---- the seeded test matrix ---------------------------------------------------
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011): four 64-bit counter
// words and two key words; each of the ten rounds takes the full 128-bit
// products of words 0 and 2 with the two round multipliers and bumps the key
// by the two Weyl constants.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Rademacher test matrix: row i is the Philox block of counter (i, 0, 0, 0)
// and key (seed, 0); bit j of its 256 bits (word j / 64, bit j % 64) gives
// +1 (bit 0) or -1 (bit 1) in column j < l; columns l .. wcols-1 get 0.  One
// workgroup makes kOmRows rows: one thread per row draws the block into LDS,
// then the workgroup writes the rows with consecutive threads on consecutive
// columns.
constexpr int kOmRows = 64;
__global__ __launch_bounds__(256) void k_test_matrix(uint64_t seed, int64_t n, int l, int wcols,
                                                     float* __restrict__ Q, int64_t ldq) {
    __shared__ uint64_t words[kOmRows][4];
    const int64_t r0 = (int64_t)blockIdx.x * kOmRows;
    const int t = threadIdx.x;
    if (t < kOmRows && r0 + t < n) {
        uint64_t c[4] = {(uint64_t)(r0 + t), 0, 0, 0};
        philox4x64_10(c, seed, 0);
#pragma unroll
        for (int w = 0; w < 4; ++w) words[t][w] = c[w];
    }
    __syncthreads();
    const int rows = (int)min<int64_t>(kOmRows, n - r0);
    const int total = rows * wcols;
    for (int e = t; e < total; e += 256) {
        const int i = e / wcols, j = e - i * wcols;
        float v = 0.0f;
        if (j < l) v = ((words[i][j >> 6] >> (j & 63)) & 1) ? -1.0f : 1.0f;
        Q[(r0 + i) * ldq + j] = v;
    }
}

__global__ __launch_bounds__(256) void k_expand_blocks(const int64_t* __restrict__ idx, int64_t s,
                                                      const int64_t* __restrict__ off, int64_t G,
                                                      const int64_t* __restrict__ map, int64_t b,
                                                      int64_t* __restrict__ out) {
    const int64_t total = s * b;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t t = e / b, i = e - t * b;
        int64_t j = idx[t];
        if (j < 0 || j >= G) j = 0;
        const int64_t pos = off[j] + i;
        out[e] = map ? map[pos] : pos;
    }
}

// C[i][t] = A[i][cols[t]]
__global__ __launch_bounds__(256) void k_gather_cols(const float* __restrict__ A, int64_t lda, int64_t m,
                                                     const int64_t* __restrict__ cols, int64_t c,
                                                     float* __restrict__ C, int64_t ldc) {
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const float* a = A + i * lda;
        float* o = C + i * ldc;
        for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < c; t += (int64_t)gridDim.x * 256)
            o[t] = a[cols[t]];
    }
}

// The same copy with 16-byte moves.  Output columns go in groups of four; a
// group whose four source columns are consecutive and start at a multiple of
// 4 (part of a contiguous block) moves as one float4, any other group element
// by element.  Workgroup (x, y) reads the source of groups y*kGatherGroups ..
// into LDS once and copies them for a band of `band` rows, consecutive threads
// on consecutive groups of a row.  Needs A, C 16-byte aligned and lda, ldc
// multiples of 4.
constexpr int kGatherGroups = 1024;
__global__ __launch_bounds__(256) void k_gather_cols_v4(const float* __restrict__ A, int64_t lda, int64_t m,
                                                        const int64_t* __restrict__ cols, int64_t c,
                                                        float* __restrict__ C, int64_t ldc, int64_t band) {
    __shared__ int64_t src[kGatherGroups];
    const int tid = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.y * kGatherGroups;
    const int ng = (int)min<int64_t>(kGatherGroups, (c + 3) / 4 - g0);
    int mine = 1;
    for (int q = tid; q < ng; q += 256) {
        const int64_t t = (g0 + q) * 4;
        const int64_t s0 = cols[t];
        bool ok = t + 3 < c && (s0 & 3) == 0;
        if (ok) ok = cols[t + 1] == s0 + 1 && cols[t + 2] == s0 + 2 && cols[t + 3] == s0 + 3;
        src[q] = ok ? s0 : -1;
        mine &= ok ? 1 : 0;
    }
    // every group of this workgroup a contiguous aligned run
    const bool all = __syncthreads_and(mine) != 0;
    const int64_t i0 = (int64_t)blockIdx.x * band;
    const int64_t rows = min<int64_t>(band, m - i0);
    const int64_t total = rows * ng;
    // every group a contiguous aligned run (the usual case: blocks of whole
    // float4s): eight moves per thread at a time, the eight reads issued
    // together and the stores with no test between them
    constexpr int U = 8;
    int64_t e0 = tid;
    if (all) {
        for (; e0 + (U - 1) * 256 < total; e0 += U * 256) {
            float4 v[U];
            float* o[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = e0 + u * 256, i = i0 + e / ng;
                const int q = (int)(e % ng);
                v[u] = *reinterpret_cast<const float4*>(A + i * lda + src[q]);
                o[u] = C + i * ldc + (g0 + q) * 4;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) *reinterpret_cast<float4*>(o[u]) = v[u];
        }
    }
    for (int64_t e = e0; e < total; e += 256) {
        const int64_t i = i0 + e / ng;
        const int q = (int)(e % ng);
        const int64_t t = (g0 + q) * 4;
        const int64_t s0 = src[q];
        const float* a = A + i * lda;
        float* o = C + i * ldc + t;
        if (s0 >= 0) {
            *reinterpret_cast<float4*>(o) = *reinterpret_cast<const float4*>(a + s0);
        } else {
            for (int u = 0; u < 4 && t + u < c; ++u) o[u] = a[cols[t + u]];
        }
    }
}

// R[t][j] = A[rows[t]][j]
__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ A, int64_t lda, int64_t n,
                                                     const int64_t* __restrict__ rows, int64_t r,
                                                     float* __restrict__ R, int64_t ldr) {
    for (int64_t t = blockIdx.y; t < r; t += gridDim.y) {
        const float* a = A + rows[t] * lda;
        float* o = R + t * ldr;
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
            o[j] = a[j];
    }
}

// G = C^T C read from H = C^T A at the chosen columns, symmetrized, FP64.
__global__ __launch_bounds__(256) void k_gram_from_cols(const float* __restrict__ H, int64_t ldh,
                                                        const int64_t* __restrict__ cols, int64_t c,
                                                        double* __restrict__ G, float* __restrict__ G32,
                                                        int64_t ldg32) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= c * c) return;
    const int64_t i = e / c, j = e - i * c;
    const double a = H[i * ldh + cols[j]], b = H[j * ldh + cols[i]];
    const double g = 0.5 * (a + b);
    G[e] = g;
    if (G32) G32[i * ldg32 + j] = (float)g;
}

__global__ __launch_bounds__(256) void k_f64_to_f32(const double* __restrict__ x, int64_t count,
                                                    float* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        y[e] = (float)x[e];
}

// wy: the columns of each row of y written (cols, or ldy to zero the padding)
__global__ __launch_bounds__(256) void k_f64_to_f32_2d(const double* __restrict__ x, int64_t rows, int64_t cols,
                                                       int64_t ldx, float* __restrict__ y, int64_t ldy, int64_t wy) {
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < wy; j += (int64_t)gridDim.x * 256)
            y[i * ldy + j] = j < cols ? (float)x[i * ldx + j] : 0.0f;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ A, int64_t m, int64_t n,
                                                   int64_t lda, uint16_t* __restrict__ out, int64_t ldo) {
    const int64_t n4 = n >> 2;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const float* a = A + i * lda;
        uint16_t* o = out + i * ldo;
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n4; j += (int64_t)gridDim.x * 256) {
            const float4 v = reinterpret_cast<const float4*>(a)[j];
            ushort4 w;
            w.x = f32_to_bf16_rne(v.x);
            w.y = f32_to_bf16_rne(v.y);
            w.z = f32_to_bf16_rne(v.z);
            w.w = f32_to_bf16_rne(v.w);
            reinterpret_cast<ushort4*>(o)[j] = w;
        }
        for (int64_t j = n4 * 4 + (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
            o[j] = f32_to_bf16_rne(a[j]);
    }
}

__global__ __launch_bounds__(256) void k_zero_f32(float* __restrict__ x, int64_t rows, int64_t cols,
                                                  int64_t ld) {
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256)
            x[i * ld + j] = 0.0f;
}

// out[0] = sum(a) - sum(b), out[1] = sum(a), out[2] = sum(b), fixed order.
__global__ __launch_bounds__(256) void k_fit_err(const double* __restrict__ a, int64_t na,
                                                 const double* __restrict__ b, int64_t nb,
                                                 double* __restrict__ out) {
    __shared__ double sh[4];
    double x = 0.0;
    for (int64_t i = threadIdx.x; i < na; i += 256) x += a[i];
    const double sa = block_sum<256>(x, sh);
    __syncthreads();
    double y = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) y += b[i];
    const double sb = block_sum<256>(y, sh);
    if (threadIdx.x == 0) {
        out[0] = sa - sb;
        out[1] = sa;
        out[2] = sb;
    }
}

// The columns not chosen, ascending, in one workgroup: the chosen columns as
// a bit set in LDS, each thread a run of its words, and a scan of the runs'
// counts giving each thread where it writes.
__global__ __launch_bounds__(1024) void k_complement_cols(const int64_t* __restrict__ cols, int64_t c, int64_t n,
                                                          int* __restrict__ ncol, int* __restrict__ bad) {
    __shared__ uint32_t bits[kComplementMaxN / 32];
    __shared__ int wtot[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t words = (n + 31) / 32;
    for (int64_t w = tid; w < words; w += 1024) bits[w] = 0u;
    __syncthreads();
    int outside = 0;
    for (int64_t k = tid; k < c; k += 1024) {
        const int64_t j = cols[k];
        if (j >= 0 && j < n)
            atomicOr(&bits[j >> 5], 1u << (j & 31));
        else
            outside = 1;
    }
    outside = __syncthreads_or(outside);
    const int64_t per = (words + 1023) / 1024;
    const int64_t w0 = min<int64_t>(words, (int64_t)tid * per), w1 = min<int64_t>(words, w0 + per);
    auto avail = [&](int64_t w) {
        uint32_t f = ~bits[w];
        if (w == words - 1 && (n & 31)) f &= (1u << (n & 31)) - 1u;
        return f;
    };
    int cnt = 0;
    for (int64_t w = w0; w < w1; ++w) cnt += __popc(avail(w));
    int inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        if (v < wave) base += wtot[v];
        total += wtot[v];
    }
    const int64_t lim = n - c;
    int64_t pos = base + inc - cnt;
    for (int64_t w = w0; w < w1; ++w) {
        uint32_t f = avail(w);
        while (f) {
            const int b = __ffs(f) - 1;
            f &= f - 1u;
            if (pos < lim) ncol[pos] = (int)(w * 32 + b);
            ++pos;
        }
    }
    if (tid == 0 && (outside || total != lim)) *bad = 1;
}

__global__ __launch_bounds__(256) void k_pin_selected(const int64_t* __restrict__ cols, int64_t c,
                                                      float* __restrict__ U, int64_t ldu, float* __restrict__ F,
                                                      int64_t ldf) {
    const int64_t total = c * c;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / c, k = e - i * c, j = cols[k];
        U[i * ldu + j] = i == k ? 1.0f : 0.0f;
        if (F) F[i * ldf + j] = 0.0f;
    }
}

inline dim3 grid2d(int64_t cols, int64_t rows) {
    int64_t gx = (cols + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    int64_t gy = rows < 65535 ? rows : 65535;
    if (gy < 1) gy = 1;
    return dim3((unsigned)gx, (unsigned)gy);
}

}  // namespace

int frob2_grid(int64_t m, int64_t n) {
    int64_t g = (m * n + 16383) / 16384;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_frob2(const float* A, int64_t m, int64_t n, int64_t lda, double* partial, int grid, double* out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_frob2_partial, dim3(grid), dim3(256), 0, st, A, m, n, lda, partial);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, (const double*)partial, (int64_t)grid, out);
    return hipGetLastError();
}

hipError_t launch_sum_f64(const double* x, int64_t count, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, x, count, out);
    return hipGetLastError();
}

hipError_t launch_block_scores(const float* V, int64_t k, int64_t ldv, const int64_t* d_off, int64_t G,
                               double* scores, hipStream_t st) {
    hipLaunchKernelGGL(k_block_scores, dim3((unsigned)G), dim3(256), 0, st, V, k, ldv, d_off, scores);
    return hipGetLastError();
}

hipError_t launch_sample(const double* scores, int64_t G, const uint64_t* draws, int64_t s, int replace,
                         uint64_t* qbuf, uint64_t* pref, int64_t* idx, double* weights, double* margins,
                         int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_sample, dim3(1), dim3(1024), 0, st, scores, G, draws, s, replace, qbuf, pref, idx,
                       weights, margins, status);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const float* A, int64_t lda, int64_t m, const int64_t* d_cols, int64_t c, float* C,
                              int64_t ldc, hipStream_t st) {
    if (m <= 0 || c <= 0) return hipSuccess;
    if (((uintptr_t)A & 15) == 0 && ((uintptr_t)C & 15) == 0 && (lda & 3) == 0 && (ldc & 3) == 0) {
        const int64_t groups = (c + 3) / 4;
        const int64_t gy = (groups + kGatherGroups - 1) / kGatherGroups;
        const int64_t per = std::min<int64_t>(groups, kGatherGroups);
        // about 16 float4 moves per thread for each band of rows
        const int64_t band = std::max<int64_t>(1, 4096 / per);
        const int64_t gx = (m + band - 1) / band;
        hipLaunchKernelGGL(k_gather_cols_v4, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, A, lda, m, d_cols,
                           c, C, ldc, band);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gather_cols, grid2d(c, m), dim3(256), 0, st, A, lda, m, d_cols, c, C, ldc);
    return hipGetLastError();
}

hipError_t launch_test_matrix(uint64_t seed, int64_t n, int64_t l, int64_t wcols, float* Q, int64_t ldq,
                              hipStream_t st) {
    if (n <= 0 || wcols <= 0) return hipSuccess;
    const int64_t grid = (n + kOmRows - 1) / kOmRows;
    k_test_matrix<<<(unsigned)grid, 256, 0, st>>>(seed, n, (int)l, (int)wcols, Q, ldq);
    return hipGetLastError();
}

hipError_t launch_expand_blocks(const int64_t* idx, int64_t s, const int64_t* off, int64_t G, const int64_t* map,
                                int64_t b, int64_t* out, hipStream_t st) {
    if (s < 1 || b < 1 || G < 1) return hipErrorInvalidValue;
    int64_t blocks = (s * b + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_expand_blocks, dim3((unsigned)blocks), dim3(256), 0, st, idx, s, off, G, map, b, out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* A, int64_t lda, int64_t n, const int64_t* d_rows, int64_t r, float* R,
                              int64_t ldr, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rows, grid2d(n, r), dim3(256), 0, st, A, lda, n, d_rows, r, R, ldr);
    return hipGetLastError();
}

hipError_t launch_gram_from_cols(const float* H, int64_t ldh, const int64_t* d_cols, int64_t c, double* G,
                                 hipStream_t st, float* G32, int64_t ldg32) {
    const int64_t blocks = (c * c + 255) / 256;
    hipLaunchKernelGGL(k_gram_from_cols, dim3((unsigned)blocks), dim3(256), 0, st, H, ldh, d_cols, c, G, G32,
                       ldg32);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* x, int64_t count, float* y, hipStream_t st) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)blocks), dim3(256), 0, st, x, count, y);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32_2d(const double* x, int64_t rows, int64_t cols, int64_t ldx, float* y, int64_t ldy,
                                bool zero_pad, hipStream_t st) {
    const int64_t wy = zero_pad ? ldy : cols;
    hipLaunchKernelGGL(k_f64_to_f32_2d, grid2d(wy, rows), dim3(256), 0, st, x, rows, cols, ldx, y, ldy, wy);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out, int64_t ldo,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_cast_bf16, grid2d((n + 3) / 4, m), dim3(256), 0, st, A, m, n, lda, out, ldo);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* x, int64_t rows, int64_t cols, int64_t ld, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f32, grid2d(cols, rows), dim3(256), 0, st, x, rows, cols, ld);
    return hipGetLastError();
}

hipError_t launch_complement_cols(const int64_t* cols, int64_t c, int64_t n, int* ncol, int* bad, hipStream_t st) {
    if (c < 1 || n <= c || n > kComplementMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_complement_cols, dim3(1), dim3(1024), 0, st, cols, c, n, ncol, bad);
    return hipGetLastError();
}

hipError_t launch_pin_selected(const int64_t* cols, int64_t c, float* U, int64_t ldu, float* F, int64_t ldf,
                               hipStream_t st) {
    if (c < 1) return hipSuccess;
    int64_t blocks = (c * c + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pin_selected, dim3((unsigned)blocks), dim3(256), 0, st, cols, c, U, ldu, F, ldf);
    return hipGetLastError();
}

hipError_t launch_fit_err(const double* parts, int64_t nparts_e, const double* dot_parts, int64_t nparts_d,
                          double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_fit_err, dim3(1), dim3(256), 0, st, parts, nparts_e, dot_parts, nparts_d, out);
    return hipGetLastError();
}

}  // namespace bcur
