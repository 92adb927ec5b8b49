// mlp.hip -- learned sampling proposal for the SGTP planner on gfx950 (project
// extension; not part of the paper's method).
//
// A 50 -> 256 -> 256 -> 200 MLP with tanh-form GELU predicts, for every horizon
// step, the mean and log-scale of the (acceleration, steering) perturbation
// distribution from the vehicle's features.  All matrix products run on BF16
// MFMA (v_mfma_f32_16x16x32_bf16) with float32 accumulation: forward, the two
// backward products per layer (input gradient and weight gradient) and the
// Gaussian negative log-likelihood of the planner's own selected controls.
// Master weights and Adam moments are float32; the GEMM operands are BF16 copies.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "sgtp.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int D_IN = SGTP_FEAT_DIM;  // 50 features
constexpr int D_INP = 64;            // padded input width
constexpr int D_H = 256;
constexpr int D_OUT = SGTP_MLP_OUT;  // 200 outputs
constexpr int D_OUTP = 256;          // padded output width
constexpr int N_H = SGTP_MLP_OUT / 4;
constexpr float A_SCALE = 4.0f, D_SCALE = 0.2f, LS_MIN = -4.0f, LS_MAX = 1.0f;
constexpr int FUSED_MAX_ROWS = 4096;  // forward batches up to this size use the fused kernel
// waves per workgroup of the fused forward: one 16-column tile per wave and layer (16 rows
// per workgroup leave one workgroup per CU at planning and training batch sizes, so the
// waves are what hides the latency)
constexpr int FWD_WAVES = 16;

// packed float32 parameter layout (the oracle's): W1[50][256] b1 W2[256][256] b2 W3[256][200] b3
constexpr size_t P_W1 = 0, P_B1 = P_W1 + (size_t)D_IN * D_H, P_W2 = P_B1 + D_H, P_B2 = P_W2 + (size_t)D_H * D_H,
                 P_W3 = P_B2 + D_H, P_B3 = P_W3 + (size_t)D_H * D_OUT, P_TOTAL = P_B3 + D_OUT;

// ------------------------------------------------------------------------------
// BF16 MFMA GEMM: C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]); optional GELU copy in BF16.
// A(m, k) = A[m a_m + k a_k], B(k, n) = B[k b_k + n b_n] (any strides, so transposed
// operands need no copies).  Workgroup tile 64 x 64; each of the 4 waves owns a 32 x 32
// quarter as 2 x 2 MFMA tiles of 16 x 16 x 32.  K runs in chunks of 64 through two LDS
// buffers: the global loads of the next chunk are issued before the MFMAs of the current
// one.  An operand whose unit stride runs along k is read as 16-byte vectors of 8 k; one
// whose unit stride runs along its rows (a transposed operand) as vectors of 8 rows,
// scattered into the [row][k] LDS layout.  The MFMAs take the 32-k blocks in increasing
// order with the same lane -> (row, k) map whatever the staging, so the sums do not
// depend on it (the fused forward below relies on this).
// ------------------------------------------------------------------------------
struct GemmArgs {
    const bf16 *A;
    long long a_m, a_k;
    const bf16 *B;
    long long b_k, b_n;
    int M, N, K;
    const float *bias;  // [N] or NULL
    float *C;           // [M][ldc] float32 result (pre-activation), or NULL
    long long ldc;
    long long c_split;  // split K: slice z writes its partial product to C + z c_split
    bf16 *H;            // [M][ldh] BF16 GELU(result) -- or, with gpre, BF16 result x GELU'(gpre) -- or NULL
    long long ldh;
    const float *gpre;  // [M][ldh] pre-activations for the activation-gradient output, or NULL
    int a_mode, b_mode; // operand staging: STAGE_ELEM, STAGE_VEC_K or STAGE_VEC_ROW
    int ones_row;       // row index of A that reads as 1 for every k (a bias gradient), or -1
};

// STAGE_BLK16: a row-blocked operand, Op(r, k) = P[r s_r + (k / 16) s_k + k % 16] (16
// consecutive k of a row contiguous), staged as 16-byte vectors of k like STAGE_VEC_K
constexpr int STAGE_ELEM = 0, STAGE_VEC_K = 1, STAGE_VEC_ROW = 2, STAGE_BLK16 = 3;
constexpr int GK = 64;          // K per LDS chunk
constexpr int LROW = GK + 8;    // LDS row in bf16 (144 bytes: 16-byte aligned, banks staggered)

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Registers of one operand chunk (64 rows x GK k): two 8-element vectors per thread.
// Vector q = tid + 256 i covers, for STAGE_ELEM / STAGE_VEC_K / STAGE_BLK16, row q / 8 and
// k 8 (q % 8) .. + 7; for STAGE_VEC_ROW, k q / 8 and rows 8 (q % 8) .. + 7.  Op(r, k) =
// P[r s_r + k s_k] (STAGE_BLK16: P[r s_r + (k / 16) s_k + k % 16]) for r < R and k < kend,
// zero beyond; row `ones` reads as 1 (for k < kend).
__device__ __forceinline__ void load_chunk(const bf16 *__restrict__ P, long long s_r, long long s_k, int mode, int r0,
                                           int R, int k0, int kend, int ones, int tid, u16x8 (&v)[2]) {
    const unsigned short ONE = 0x3F80;  // bf16 1.0
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int q = tid + 256 * i;
        u16x8 x;
        if (mode == STAGE_VEC_ROW) {
            const int k = k0 + (q >> 3), r = r0 + 8 * (q & 7);
            if (r + 8 <= R && (ones < r || ones >= r + 8) && k < kend) {
                x = *(const u16x8 *)&P[(long long)r * s_r + (long long)k * s_k];
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int rr = r + j;
                    x[j] = (k >= kend) ? (unsigned short)0
                           : (rr == ones) ? ONE
                           : (rr < R) ? __builtin_bit_cast(unsigned short, P[(long long)rr * s_r + (long long)k * s_k])
                                      : (unsigned short)0;
                }
            }
        } else {
            const int r = r0 + (q >> 3), k = k0 + 8 * (q & 7);
            const bool blk = mode == STAGE_BLK16;
            if ((mode == STAGE_VEC_K || blk) && r < R && r != ones && k + 8 <= kend) {
                x = *(const u16x8 *)&P[(long long)r * s_r + (blk ? (long long)(k >> 4) * s_k + (k & 15) : k)];
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int kk = k + j;
                    const long long o = (long long)r * s_r + (blk ? (long long)(kk >> 4) * s_k + (kk & 15)
                                                                  : (long long)kk * s_k);
                    x[j] = (kk >= kend) ? (unsigned short)0
                           : (r == ones) ? ONE
                           : (r < R) ? __builtin_bit_cast(unsigned short, P[o])
                                     : (unsigned short)0;
                }
            }
        }
        v[i] = x;
    }
}

__device__ __forceinline__ void store_chunk(bf16 (*S)[LROW], int mode, int tid, const u16x8 (&v)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int q = tid + 256 * i;
        if (mode == STAGE_VEC_ROW) {
            const int k = q >> 3, r = 8 * (q & 7);
#pragma unroll
            for (int j = 0; j < 8; ++j) *(unsigned short *)&S[r + j][k] = v[i][j];
        } else {
            *(u16x8 *)&S[q >> 3][8 * (q & 7)] = v[i];
        }
    }
}

__device__ __forceinline__ float gelu_f(float x) {
    const float c = 0.7978845608f;
    return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
    const float c = 0.7978845608f;
    const float u = c * (x + 0.044715f * x * x * x);
    const float t = tanhf(u);
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

// One 64 x 64 tile (column tile bx, row tile by) of K slice bz of nz.
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bx, int by, int bz, int nz) {
    __shared__ __align__(16) bf16 As[2][64][LROW];  // [buffer][m][k]
    __shared__ __align__(16) bf16 Bs[2][64][LROW];  // [buffer][n][k]
    const int m0 = by * 64, n0 = bx * 64;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    // split K: slice bz of nz covers [kbeg, kend) (a multiple of 32 long, but the
    // last) and writes its partial product to its own slice of C (summed afterwards in
    // slice order: the result does not depend on timing)
    const int kslice = ((g.K + 32 * nz - 1) / (32 * nz)) * 32;
    const int kbeg = bz * kslice, kend = min(g.K, kbeg + kslice);
    const int nk = kend > kbeg ? (kend - kbeg + GK - 1) / GK : 0;
    u16x8 va[2], vb[2];
    if (nk > 0) {
        load_chunk(g.A, g.a_m, g.a_k, g.a_mode, m0, g.M, kbeg, kend, g.ones_row, tid, va);
        load_chunk(g.B, g.b_n, g.b_k, g.b_mode, n0, g.N, kbeg, kend, -1, tid, vb);
    }
    const int kk = 8 * (l >> 4);
    for (int it = 0; it < nk; ++it) {
        const int buf = it & 1;
        store_chunk(As[buf], g.a_mode, tid, va);
        store_chunk(Bs[buf], g.b_mode, tid, vb);
        __syncthreads();
        const int k0 = kbeg + it * GK;
        if (it + 1 < nk) {  // next chunk's loads in flight during this chunk's MFMAs
            load_chunk(g.A, g.a_m, g.a_k, g.a_mode, m0, g.M, k0 + GK, kend, g.ones_row, tid, va);
            load_chunk(g.B, g.b_n, g.b_k, g.b_mode, n0, g.N, k0 + GK, kend, -1, tid, vb);
        }
#pragma unroll
        for (int ks = 0; ks < GK; ks += 32) {
            if (k0 + ks >= kend) break;  // no all-zero block beyond the slice (same blocks as K steps of 32)
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *(const bf16x8 *)&As[buf][wm + 16 * i + (l & 15)][ks + kk];
                b[i] = *(const bf16x8 *)&Bs[buf][wn + 16 * i + (l & 15)][ks + kk];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        // the buffer written at iteration it + 2 is read here: the barrier of iteration
        // it + 1 separates the two
    }
    // D(16 x 16) of one MFMA: lane l, element v -> row 4 (l / 16) + v, column l % 16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + 16 * i + 4 * (l >> 4) + v;
                const int n = n0 + wn + 16 * j + (l & 15);
                if (m < g.M && n < g.N) {
                    float x = acc[i][j][v];
                    if (nz > 1) {
                        g.C[bz * g.c_split + (long long)m * g.ldc + n] = x;
                        continue;
                    }
                    if (g.bias) x += g.bias[n];
                    if (g.C) g.C[(long long)m * g.ldc + n] = x;
                    if (g.H)
                        g.H[(long long)m * g.ldh + n] =
                            g.gpre ? (bf16)(x * gelu_grad_f(g.gpre[(long long)m * g.ldh + n])) : (bf16)gelu_f(x);
                }
            }
}

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    gemm_tile(g, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z);
}

// Up to three independent products in one launch: blocks [first[p], first[p + 1]) are
// product p's grid gx[p] x gy[p] x gz[p] (x fastest), each block as k_gemm_bf16's.
struct GemmGroup {
    GemmArgs g[3];
    int gx[3], gy[3], gz[3];
    int first[4];
};
__global__ void __launch_bounds__(256) k_gemm_bf16_group(GemmGroup gg) {
    const int bid = blockIdx.x;
    const int p = bid < gg.first[1] ? 0 : bid < gg.first[2] ? 1 : 2;
    const int q = bid - gg.first[p], gx = gg.gx[p], gy = gg.gy[p];
    gemm_tile(gg.g[p], q % gx, (q / gx) % gy, q / (gx * gy), gg.gz[p]);
}

// a row-blocked copy [B / 16][C][16] back to rows [B][C]
__global__ void k_unblock(const bf16 *src, int C, int B, bf16 *dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)B * C) return;
    const int b = (int)(e / C), c = (int)(e % C);
    dst[e] = src[((long long)(b >> 4) * C + c) * 16 + (b & 15)];
}

__global__ void k_to_bf16_rows(const float *X, int B, int din, int ldx, bf16 *Y, int ldy) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = e / ldy, c = e % ldy;
    if (b >= B) return;
    Y[(long long)b * ldy + c] = (c < din) ? (bf16)X[(long long)b * ldx + c] : (bf16)0.0f;
}

// Philox4x32-10 (Salmon et al., SC'11: two 32 x 32 -> 64-bit products per round, Weyl key
// schedule): the counter-based generator of the minibatch draw
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Minibatch row b: data row i = floor(r M / 2^32), r the first Philox word at counter
// (b, t, 0, 0), t the Adam steps taken (read on the device); its features as BF16 operands
// [b][64] (zero padding) and its targets [b][N][2].  One block of 128 threads per row.
__global__ void k_gather_sampled(const float *X_all, const float *U_all, long long M, int N, uint32_t k0,
                                 uint32_t k1, const int *t, bf16 *Xb, float *Ub, int *idx) {
    const int b = blockIdx.x;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)b, (uint32_t)*t, 0u, 0u), k0, k1);
    const long long i = (long long)(((unsigned long long)r.x * (unsigned long long)M) >> 32);
    if (threadIdx.x == 0) idx[b] = (int)i;
    if (threadIdx.x < D_INP)
        Xb[(long long)b * D_INP + threadIdx.x] =
            threadIdx.x < D_IN ? (bf16)X_all[i * D_IN + threadIdx.x] : (bf16)0.0f;
    for (int e = threadIdx.x; e < 2 * N; e += blockDim.x) Ub[(long long)b * 2 * N + e] = U_all[i * 2 * N + e];
}

// packed float32 weights -> BF16 GEMM operands (W3 padded to 256 columns)
__global__ void k_refresh_bf16(const float *P, bf16 *W1, bf16 *W2, bf16 *W3, float *b3p) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < D_IN * D_H) W1[e] = (bf16)P[P_W1 + e];
    if (e < D_H * D_H) W2[e] = (bf16)P[P_W2 + e];
    if (e < D_H * D_OUTP) {
        const int r = e / D_OUTP, c = e % D_OUTP;
        W3[e] = (c < D_OUT) ? (bf16)P[P_W3 + (size_t)r * D_OUT + c] : (bf16)0.0f;
    }
    if (e < D_OUTP) b3p[e] = (e < D_OUT) ? P[P_B3 + e] : 0.0f;
}

// Transposed BF16 copies for the fused small-batch forward: W1T [256][64] (k >= 50 zero),
// W2T [256][256], W3T [256][256] (rows n >= 200 zero); row n holds the weights into unit n.
__global__ void k_refresh_bf16_t(const float *P, bf16 *W1T, bf16 *W2T, bf16 *W3T) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < D_H * D_INP) {
        const int n = e / D_INP, k = e % D_INP;
        W1T[e] = (k < D_IN) ? (bf16)P[P_W1 + (size_t)k * D_H + n] : (bf16)0.0f;
    }
    if (e < D_H * D_H) {
        const int n = e / D_H, k = e % D_H;
        W2T[e] = (bf16)P[P_W2 + (size_t)k * D_H + n];
        W3T[e] = (n < D_OUT) ? (bf16)P[P_W3 + (size_t)k * D_OUT + n] : (bf16)0.0f;
    }
}

// One 16 x K x 16 product step of the fused kernels (output columns n0 .. n0 + 15): the
// B fragments of a lane come from the transposed weights (row n0 + l % 16, k 32 i + 8 (l /
// 16) .. + 7 for i = 0 .. K/32 - 1) and are loaded first, so a wave can fetch them ahead
// of the barrier or epilogue before its product; the A rows come from LDS.  Same lane ->
// (row, k) map and k order as k_gemm_bf16, so the sums are the same.
// four BF16 values (rows 4 g .. 4 g + 3 of one column of a row-blocked copy) as one
// 8-byte store
__device__ __forceinline__ void store_rows4(bf16 *dst, const bf16 (&h)[4]) {
    ushort4 u;
    u.x = __builtin_bit_cast(unsigned short, h[0]);
    u.y = __builtin_bit_cast(unsigned short, h[1]);
    u.z = __builtin_bit_cast(unsigned short, h[2]);
    u.w = __builtin_bit_cast(unsigned short, h[3]);
    *(ushort4 *)dst = u;
}

template <int K>
__device__ __forceinline__ void load_frags(const bf16 *__restrict__ WT, int n0, int l, bf16x8 (&b)[K / 32]) {
#pragma unroll
    for (int i = 0; i < K / 32; ++i) b[i] = *(const bf16x8 *)&WT[(size_t)(n0 + (l & 15)) * K + 32 * i + 8 * (l >> 4)];
}
template <int K>
__device__ __forceinline__ f32x4 mfma_frags(const bf16 *A, int lda, const bf16x8 (&b)[K / 32], int l) {
    f32x4 acc = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < K / 32; ++i) {
        const bf16x8 a = *(const bf16x8 *)&A[(l & 15) * lda + 32 * i + 8 * (l >> 4)];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[i], acc, 0, 0, 0);
    }
    return acc;
}

// Gaussian negative log-likelihood of target u for step t < 64, channel c (0 acceleration,
// 1 steering) of one row whose outputs are o[256] (mean over B rows; constant 0.5 log 2 pi
// dropped; steps t >= N do not enter, u unused): its term is returned, its gradient w.r.t.
// the outputs written as BF16 to g[4 t + c] (mean) and g[4 t + 2 + c] (log scale), and,
// when gt is not NULL, also to gt[(4 t + c) ldt] and gt[(4 t + 2 + c) ldt].
__device__ __forceinline__ float nll_term(const float *o, float u, int t, int c, int N, float sig_a, float sig_d,
                                          int B, bf16 *g, bf16 *gt = nullptr, long long ldt = 0) {
    if (t >= N) {
        g[4 * t + c] = (bf16)0.0f;
        g[4 * t + 2 + c] = (bf16)0.0f;
        if (gt) {
            gt[(4 * t + c) * ldt] = (bf16)0.0f;
            gt[(4 * t + 2 + c) * ldt] = (bf16)0.0f;
        }
        return 0.0f;
    }
    const float scale = c ? D_SCALE : A_SCALE;
    const float lsp = logf(c ? sig_d : sig_a);
    const float mu = scale * o[4 * t + c];
    const float raw = o[4 * t + 2 + c];
    const float cl = fminf(fmaxf(raw, LS_MIN), LS_MAX);
    const float ls = lsp + cl;
    const float inv_s2 = expf(-2.0f * ls);
    const float res = u - mu;
    const bf16 gm = (bf16)(-scale * res * inv_s2 / (float)B);
    const bf16 gs = (bf16)((raw > LS_MIN && raw < LS_MAX) ? (1.0f - res * res * inv_s2) / (float)B : 0.0f);
    g[4 * t + c] = gm;
    g[4 * t + 2 + c] = gs;
    if (gt) {
        gt[(4 * t + c) * ldt] = gm;
        gt[(4 * t + 2 + c) * ldt] = gs;
    }
    return 0.5f * res * res * inv_s2 + ls;
}

// What a training forward also does: where its rows come from (row b of X and U, or, with
// M > 0, a data-set row drawn as k_gather_sampled draws it, recorded in idx), the rows'
// BF16 operands it leaves for the backward pass, and the loss gradient it ends with.
struct TrainIn {
    const float *U;  // targets [.][N][2], rows indexed like the features
    long long M;     // data-set rows when the minibatch is drawn, else 0
    uint32_t k0, k1;
    const int *t;    // Adam steps taken (the draw's counter)
    int *idx;        // [B] drawn rows
    bf16 *Xb;        // [B][64] BF16 features (zero padding)
    int N;
    float sig_a, sig_d;
    bf16 *dout;       // [B][256] loss gradient w.r.t. the outputs
    float *loss_part; // [2 B] loss partials: row b steps 0-31 at 2 b, steps 32-63 at 2 b + 1
    // row-blocked copies [B / 16][columns][16] of the features, both hidden activations and
    // the output gradient
    bf16 *XB, *H1B, *H2B, *DB;
};

// Fused forward of 16 rows per workgroup: the three layers run back to back with the
// hidden activations in LDS (BF16, as the tiled path stores them).  TRAIN: the rows are
// fetched (drawn or not) from X, their BF16 operands written to Xb; the pre-activations
// (float32) and activations (BF16) of both hidden layers are also written out ([B][256]
// each), as the tiled products write them for the backward pass; and the loss and its
// gradient are taken from the output tile, as k_nll takes them (same lane -> (step,
// channel) map, same per-wave sums).
template <bool TRAIN>
__global__ void __launch_bounds__(64 * FWD_WAVES) k_mlp_fwd16(const float *X, int ldx, int B, const bf16 *W1T,
                                                             const bf16 *W2T, const bf16 *W3T, const float *b1,
                                                             const float *b2, const float *b3, float *out, int ldo,
                                                             int n_out, float *pre1, bf16 *h1o, float *pre2,
                                                             bf16 *h2o, TrainIn ti) {
    static_assert(FWD_WAVES == 16, "one 16-column tile per wave and layer");
    constexpr int LX = D_INP + 8, LH = D_H + 8, LO = D_OUTP + 4;  // padded rows
    __shared__ __align__(16) bf16 xs[16 * LX];
    __shared__ __align__(16) bf16 h1[16 * LH];
    __shared__ __align__(16) bf16 h2[16 * LH];
    __shared__ float os[TRAIN ? 16 * LO : 1];
    __shared__ __align__(16) bf16 dsb[TRAIN ? 16 * D_OUTP : 8];  // output gradient, row-blocked
    __shared__ long long src[16];
    const int r0 = blockIdx.x * 16, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int n0 = 16 * w, col = n0 + (l & 15);  // this wave's output columns in every layer
    const bool l3 = n0 < n_out;                  // layer 3 columns >= n_out are dropped
    // the wave's weight fragments and biases of all three layers, fetched while the rows
    // are drawn and fetched
    bf16x8 f1[D_INP / 32], f2[D_H / 32], f3[D_H / 32];
    load_frags<D_INP>(W1T, n0, l, f1);
    load_frags<D_H>(W2T, n0, l, f2);
    if (l3) load_frags<D_H>(W3T, n0, l, f3);
    const float c1 = b1[col], c2 = b2[col], c3 = col < n_out ? b3[col] : 0.0f;
    if (tid < 16) {
        const int b = r0 + tid;
        long long i = b;
        if (TRAIN && ti.M > 0 && b < B) {
            const uint4 r = philox4x32_10(make_uint4((uint32_t)b, (uint32_t)*ti.t, 0u, 0u), ti.k0, ti.k1);
            i = (long long)(((unsigned long long)r.x * (unsigned long long)ti.M) >> 32);
            ti.idx[b] = (int)i;
        }
        src[tid] = i;
    }
    __syncthreads();
    for (int e = tid; e < 16 * D_INP; e += 64 * FWD_WAVES) {
        const int r = e / D_INP, c = e % D_INP;
        const bf16 v = (r0 + r < B && c < D_IN) ? (bf16)X[src[r] * ldx + c] : (bf16)0.0f;
        xs[r * LX + c] = v;
        if (TRAIN && ti.Xb && r0 + r < B) ti.Xb[(long long)(r0 + r) * D_INP + c] = v;
    }
    // the targets the loss section below takes (its pairs (row, step, channel) of both of
    // the wave's groups), fetched now
    const int tt = 32 * (w & 1) + (l >> 1), cc = l & 1;
    float u[2] = {0.0f, 0.0f};
    if (TRAIN && tt < ti.N) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int row = (w >> 1) + 8 * j;
            if (r0 + row < B) u[j] = ti.U[src[row] * 2 * ti.N + 2 * tt + cc];
        }
    }
    __syncthreads();
    if (TRAIN)  // the rows' features into their row-blocked copy, 16 rows of a column contiguous
        for (int e = tid; e < 16 * D_INP; e += 64 * FWD_WAVES)
            ti.XB[(long long)r0 * D_INP + e] = xs[(e & 15) * LX + (e >> 4)];
    {  // layer 1
        const f32x4 acc = mfma_frags<D_INP>(xs, LX, f1, l);
        bf16 hb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * (l >> 4) + v;
            const float x = acc[v] + c1;
            const bf16 h = (bf16)gelu_f(x);
            hb[v] = h;
            h1[row * LH + col] = h;
            if (TRAIN && r0 + row < B) {
                pre1[(long long)(r0 + row) * D_H + col] = x;
                if (h1o) h1o[(long long)(r0 + row) * D_H + col] = h;
            }
        }
        if (TRAIN) store_rows4(ti.H1B + (long long)r0 * D_H + col * 16 + 4 * (l >> 4), hb);
    }
    __syncthreads();
    {  // layer 2
        const f32x4 acc = mfma_frags<D_H>(h1, LH, f2, l);
        bf16 hb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * (l >> 4) + v;
            const float x = acc[v] + c2;
            const bf16 h = (bf16)gelu_f(x);
            hb[v] = h;
            h2[row * LH + col] = h;
            if (TRAIN && r0 + row < B) {
                pre2[(long long)(r0 + row) * D_H + col] = x;
                if (h2o) h2o[(long long)(r0 + row) * D_H + col] = h;
            }
        }
        if (TRAIN) store_rows4(ti.H2B + (long long)r0 * D_H + col * 16 + 4 * (l >> 4), hb);
    }
    __syncthreads();
    if (l3) {  // layer 3
        const f32x4 acc = mfma_frags<D_H>(h2, LH, f3, l);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * (l >> 4) + v;
            const float o = acc[v] + c3;
            if (TRAIN) os[row * LO + col] = o;
            if (r0 + row < B && col < n_out) out[(long long)(r0 + row) * ldo + col] = o;
        }
    }
    if (TRAIN) {
        __syncthreads();
        // 32 groups of 64 (step, channel) pairs: row vg / 2, steps 32 (vg & 1) + 0..31; wave
        // w takes groups w and w + 16 (rows w / 2 and w / 2 + 8)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int vg = w + 16 * j, row = vg >> 1, b = r0 + row;
            if (b >= B) break;
            float contrib = nll_term(os + row * LO, u[j], tt, cc, ti.N, ti.sig_a, ti.sig_d, B,
                                     ti.dout + (long long)b * D_OUTP, dsb + row, 16);
            for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
            if (l == 0) ti.loss_part[2 * b + (vg & 1)] = contrib;
        }
        __syncthreads();
        // the output gradient's row-blocked copy: the block's 16 x 256 tile, contiguous
        for (int e = tid; e < 16 * D_OUTP / 8; e += 64 * FWD_WAVES)
            *(u16x8 *)&ti.DB[(long long)r0 * D_OUTP + 8 * e] = *(const u16x8 *)&dsb[8 * e];
    }
}

// The same loss and gradient from outputs in memory (the tiled path), targets U[B][N][2].
// One thread per (row, step < 64, channel); one partial per wave, summed in order by
// k_grad_finish.
__global__ void k_nll(const float *out, int ldo, const float *U, int B, int N, float sig_a, float sig_d, bf16 *dout,
                      int ldd, float *loss_part) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = e >> 7, t = (e >> 1) & 63, c = e & 1;
    float contrib = 0.0f;
    if (b < B && 4 * t < ldd)
        contrib = nll_term(out + (long long)b * ldo, t < N ? U[((long long)b * N + t) * 2 + c] : 0.0f, t, c, N, sig_a,
                           sig_d, B, dout + (long long)b * ldd);
    for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
    if ((threadIdx.x & 63) == 0) loss_part[e >> 6] = contrib;
}

// Fused input gradients of 16 rows per workgroup, the backward counterpart of k_mlp_fwd16:
// D2 = BF16((D W3^T) GELU'(pre2)), kept in LDS, then D1 = BF16((D2 W2^T) GELU'(pre1));
// both written out for the weight gradients.  Same lane -> (row, k) map and k order as the
// tiled products, so the same bits.
__global__ void __launch_bounds__(64 * FWD_WAVES) k_mlp_bwd16(const bf16 *D, const bf16 *W3, const bf16 *W2,
                                                             const float *pre2, const float *pre1, int B, bf16 *D2,
                                                             bf16 *D1, bf16 *D2B, bf16 *D1B, int *step_count) {
    static_assert(FWD_WAVES == 16, "one 16-column tile per wave and layer");
    constexpr int LH = D_H + 8;
    __shared__ __align__(16) bf16 ds[16 * LH];
    __shared__ __align__(16) bf16 d2s[16 * LH];
    const int r0 = blockIdx.x * 16, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int n0 = 16 * w, col = n0 + (l & 15);
    // in a combined training step, the Adam step count advances here: the forward before
    // has drawn its rows with the old count, the Adam step after reads the new one
    if (step_count && blockIdx.x == 0 && tid == 0) *step_count += 1;
    // everything that does not depend on the products first: the wave's weight fragments
    // and GELU'(pre-activation) of its 4 x 2 elements (rows past B read row B - 1, unused)
    bf16x8 f3[D_OUTP / 32], f2[D_H / 32];
    load_frags<D_OUTP>(W3, n0, l, f3);
    load_frags<D_H>(W2, n0, l, f2);
    float q2[4], q1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long o = (long long)min(r0 + 4 * (l >> 4) + v, B - 1) * D_H + col;
        q2[v] = pre2[o];
        q1[v] = pre1[o];
    }
    for (int e = tid; e < 16 * (D_OUTP / 8); e += 64 * FWD_WAVES) {  // 16-byte vectors of 8 columns
        const int r = e / (D_OUTP / 8), c = 8 * (e % (D_OUTP / 8));
        u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r0 + r < B) v = *(const u16x8 *)&D[(long long)(r0 + r) * D_OUTP + c];
        *(u16x8 *)&ds[r * LH + c] = v;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        q2[v] = gelu_grad_f(q2[v]);
        q1[v] = gelu_grad_f(q1[v]);
    }
    __syncthreads();
    {  // D2
        const f32x4 acc = mfma_frags<D_OUTP>(ds, LH, f3, l);
        bf16 hb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * (l >> 4) + v;
            bf16 h = (bf16)0.0f;
            if (r0 + row < B) {
                h = (bf16)(acc[v] * q2[v]);
                if (D2) D2[(long long)(r0 + row) * D_H + col] = h;
            }
            hb[v] = h;
            d2s[row * LH + col] = h;
        }
        store_rows4(D2B + (long long)r0 * D_H + col * 16 + 4 * (l >> 4), hb);
    }
    __syncthreads();
    {  // D1
        const f32x4 acc = mfma_frags<D_H>(d2s, LH, f2, l);
        bf16 hb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * (l >> 4) + v;
            hb[v] = (bf16)(acc[v] * q1[v]);
            if (D1 && r0 + row < B) D1[(long long)(r0 + row) * D_H + col] = hb[v];
        }
        store_rows4(D1B + (long long)r0 * D_H + col * 16 + 4 * (l >> 4), hb);
    }
}

// loss = (sum of the per-wave partials, in a fixed order) / B, by one block of 256 threads;
// also written to loss2 when it is given
__device__ __forceinline__ void loss_total(const float *part, int n, int B, float *loss, float *loss2) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = red[0] / (float)B;
        if (loss2) loss2[0] = red[0] / (float)B;
    }
}

// Adam step number t = *t_prev + 1 read on the device (so a captured training step can be
// replayed); k_step_count advances it after the step
// The new master weight is also written to the BF16 operand copies (plain and transposed;
// their padding stays zero), as k_refresh_bf16 and k_refresh_bf16_t would.
struct Bf16Copies {
    bf16 *W1, *W2, *W3, *W1T, *W2T, *W3T;
    float *b3p;
};
__device__ __forceinline__ void write_copies(const Bf16Copies &w, size_t e, float p) {
    const bf16 h = (bf16)p;
    if (e < P_B1) {
        const size_t k = e / D_H, n = e % D_H;
        w.W1[e] = h;
        w.W1T[n * D_INP + k] = h;
    } else if (e >= P_W2 && e < P_B2) {
        const size_t f = e - P_W2, k = f / D_H, n = f % D_H;
        w.W2[f] = h;
        w.W2T[n * D_H + k] = h;
    } else if (e >= P_W3 && e < P_B3) {
        const size_t f = e - P_W3, k = f / D_OUT, n = f % D_OUT;
        w.W3[k * D_OUTP + n] = h;
        w.W3T[n * D_H + k] = h;
    } else if (e >= P_B3) {
        w.b3p[e - P_B3] = p;
    }
}

struct AdamArgs {
    float *P, *m, *v;
    float lr, b1, b2, eps;
    const int *t_prev;
    Bf16Copies copies;
    int t_add;  // step number t = *t_prev + t_add (0 when the count was already advanced)
};
// Adam on parameter e with gradient g (bias-corrected moments, step t)
__device__ __forceinline__ void adam_update(const AdamArgs &a, size_t e, float g) {
    const float t = (float)(*a.t_prev + a.t_add);
    const float bc1 = 1.0f - powf(a.b1, t), bc2 = 1.0f - powf(a.b2, t);
    const float mm = a.b1 * a.m[e] + (1.0f - a.b1) * g;
    const float vv = a.b2 * a.v[e] + (1.0f - a.b2) * g * g;
    a.m[e] = mm;
    a.v[e] = vv;
    const float p = a.P[e] - a.lr * (mm / bc1) / (sqrtf(vv / bc2) + a.eps);
    a.P[e] = p;
    write_copies(a.copies, e, p);
}

// One launch that ends the gradient: the slice sums of the three weight-and-bias gradient
// products (dst[r][c] = the sum over slices z = 0, 1, ... in that order of src[z][r][c]; with
// dst_last the last row, the bias gradient, goes to dst_last[c]) and, in the last block,
// the loss.  Blocks [first[l], first[l + 1]) sum product l.  With adam_on, each gradient
// value also takes its Adam step at once (parameter index = its offset in G).
struct SliceSum {
    const float *src;
    long long zs;
    int n_slices, rows, cols, lds, ldd;
    float *dst, *dst_last;
};
struct FinishArgs {
    SliceSum s[3];
    int first[4];  // block ranges; block first[3] computes the loss
    const float *lp;
    int n_lp, B;
    float *loss, *loss2;
    const float *G;
    int adam_on;
    AdamArgs adam;
};
__global__ void k_grad_finish(FinishArgs f) {
    const int blk = blockIdx.x;
    if (blk >= f.first[3]) {
        loss_total(f.lp, f.n_lp, f.B, f.loss, f.loss2);
        return;
    }
    const int l = blk < f.first[1] ? 0 : blk < f.first[2] ? 1 : 2;
    const SliceSum &d = f.s[l];
    const int e = (blk - f.first[l]) * blockDim.x + threadIdx.x;
    if (e >= d.rows * d.cols) return;
    const int r = e / d.cols, c = e % d.cols;
    const float *q = d.src + (long long)r * d.lds + c;
    // loads issued up to 32 at a time, added in slice order (the sum is the same as one at
    // a time)
    constexpr int G = 32;
    const int n = d.n_slices;
    float v = q[0];
    for (int z = 1; z < n; z += G) {
        float t[G];
#pragma unroll
        for (int j = 0; j < G; ++j) t[j] = z + j < n ? q[(z + j) * d.zs] : 0.0f;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (z + j < n) v += t[j];
    }
    float *dp = (d.dst_last && r == d.rows - 1) ? d.dst_last + c : d.dst + (long long)r * d.ldd + c;
    *dp = v;
    if (f.adam_on) adam_update(f.adam, (size_t)(dp - f.G), v);
}

__global__ void k_adam(AdamArgs a, const float *G, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    adam_update(a, (size_t)e, G[e]);
}

__global__ void k_step_count(int *t) {
    if (threadIdx.x == 0) *t += 1;
}

}  // namespace

struct sgtp_mlp {
    int B_max = 0;
    std::string err;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;  // packed float32
    bf16 *W1 = nullptr, *W2 = nullptr, *W3 = nullptr;              // BF16 operands
    bf16 *W1T = nullptr, *W2T = nullptr, *W3T = nullptr;           // transposed (fused forward)
    float *b3p = nullptr;
    bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *D = nullptr, *D2 = nullptr, *D1 = nullptr;
    float *PRE1 = nullptr, *PRE2 = nullptr, *OUT = nullptr, *loss = nullptr;
    float *PART = nullptr;  // split-K partial products of the weight and bias gradients [3][64][257][256]
    float *LP = nullptr;    // per-wave loss partials [2 B_max + 4]
    int *adam_t = nullptr;  // device: Adam steps taken
    float *UB = nullptr;    // gathered targets of a sampled gradient [B_max][N_H][2]
    int *IDX = nullptr;     // rows drawn by the last sampled gradient [B_max]
    // row-blocked copies [B / 16][columns][16] of X, H1, H2, D, D2 and D1, written by the
    // fused kernels (one contiguous block per workgroup) so the weight-gradient products
    // (K = the batch) stage 16-byte vectors of k
    bf16 *XB = nullptr, *H1B = nullptr, *H2B = nullptr, *DB = nullptr, *D2B = nullptr, *D1B = nullptr;
    int last_B = 0;  // rows of the last sgtp_mlp_grad (its workspace tensors stay until the next call)
    bool last_sampled = false;  // the last gradient drew its rows on the device
    bool last_blocked = false;  // the last gradient left H1, H2, D2 and D1 only row-blocked
};

namespace {

int mfail(sgtp_mlp *m, int code, const std::string &s) {
    if (m) m->err = s;
    return code;
}
#define MCHK(m, call)                                                                                        \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return mfail(m, SGTP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// K split of a weight-gradient product (K = batch, output (M + 1) x N): slices of whole
// 64-k chunks (a part-filled last chunk in every slice costs as much as a full one), three
// per slice for the products of many tiles and two for the one of few (at a 4096-row
// batch 22, 22 and 32 slices, 1008 workgroups in the grouped launch: measured faster than
// 2 or 4 chunks, and than slices sized for a workgroup count), at most 64 slices
constexpr int MAX_SPLITS = 64;
int k_splits(int M, int N, int K) {
    const int tiles = ((N + 63) / 64) * ((M + 1 + 63) / 64);
    const int c = tiles >= 16 ? 3 : 2;
    const int chunks = (K + 63) / 64;
    return std::max(1, std::min(MAX_SPLITS, (chunks + c - 1) / c));
}

// staging of an operand with element strides (s_r along its rows, s_k along k): 16-byte
// vectors where the unit stride and the alignment allow them
int stage_mode(const void *P, long long s_r, long long s_k) {
    if (((uintptr_t)P & 15) != 0) return STAGE_ELEM;
    if (s_k == 1 && s_r % 8 == 0) return STAGE_VEC_K;
    if (s_r == 1 && s_k % 8 == 0) return STAGE_VEC_ROW;
    return STAGE_ELEM;
}

// H output: BF16 GELU(C), or with gpre BF16 C x GELU'(gpre) (an activation gradient)
void gemm(hipStream_t st, const bf16 *A, long long a_m, long long a_k, const bf16 *B, long long b_k, long long b_n,
          int M, int N, int K, const float *bias, float *C, long long ldc, bf16 *H, long long ldh,
          const float *gpre = nullptr) {
    GemmArgs g{A, a_m, a_k, B, b_k, b_n, M, N, K, bias, C, ldc, 0, H, ldh, gpre,
               stage_mode(A, a_m, a_k), stage_mode(B, b_n, b_k), -1};
    hipLaunchKernelGGL(k_gemm_bf16, dim3((N + 63) / 64, (M + 63) / 64, 1), dim3(256), 0, st, g);
}

// weight gradient dst[M][ldd] (first N columns) = A B and bias gradient bias_dst[N] =
// column sums of B, as one product with an extra row of ones in A, K split into `splits`
// slices: partial products into `part` [splits][M + 1][N]; the slices are summed in order
// by k_grad_finish (its descriptor is returned).  The product becomes member p of the
// group launch grp.  blk_mode STAGE_BLK16: both operands row-blocked (strides as that
// mode reads them).
SliceSum gemm_wgrad(GemmGroup &grp, int p, float *part, const bf16 *A, long long a_m, long long a_k, const bf16 *B,
                    long long b_k, long long b_n, int M, int N, int K, float *dst, int ldd, float *bias_dst,
                    int splits, int blk_mode = -1) {
    const int R = M + 1;  // row M of A reads as 1: the bias gradient
    const int am = blk_mode >= 0 ? blk_mode : stage_mode(A, a_m, a_k);
    const int bm = blk_mode >= 0 ? blk_mode : stage_mode(B, b_n, b_k);
    grp.g[p] = GemmArgs{A, a_m, a_k, B, b_k, b_n, R, N, K, nullptr, part, N, (long long)R * N, nullptr, 0, nullptr,
                        am, bm, M};
    grp.gx[p] = (N + 63) / 64;
    grp.gy[p] = (R + 63) / 64;
    grp.gz[p] = splits;
    grp.first[p + 1] = grp.first[p] + grp.gx[p] * grp.gy[p] * splits;
    return SliceSum{part, (long long)R * N, splits, R, N, N, ldd, dst, bias_dst};
}

// forward of B rows (features float32 [B][ldx]) into out[B][ldo], n_out columns (200, or
// 256 with the zero padding for the loss)
// (products only: the BF16 operands are already in m->X)
int forward_bf16(sgtp_mlp *m, int B, float *out, int ldo, int n_out, hipStream_t st) {
    gemm(st, m->X, D_INP, 1, m->W1, D_H, 1, B, D_H, D_IN, m->P + P_B1, m->PRE1, D_H, m->H1, D_H);
    gemm(st, m->H1, D_H, 1, m->W2, D_H, 1, B, D_H, D_H, m->P + P_B2, m->PRE2, D_H, m->H2, D_H);
    gemm(st, m->H2, D_H, 1, m->W3, D_OUTP, 1, B, n_out, D_H, m->b3p, out, ldo, nullptr, 0);
    MCHK(m, hipGetLastError());
    return SGTP_OK;
}
int forward(sgtp_mlp *m, const float *X, int ldx, int B, float *out, int ldo, int n_out, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16_rows, dim3((B * D_INP + 255) / 256), dim3(256), 0, st, X, B, D_IN, ldx, m->X, D_INP);
    return forward_bf16(m, B, out, ldo, n_out, st);
}

}  // namespace

extern "C" {

int sgtp_mlp_create(int B_max, sgtp_mlp **out) {
    if (!out || B_max < 1) return SGTP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return SGTP_EDEVICE;
    sgtp_mlp *m = new sgtp_mlp();
    m->B_max = B_max;
    bool ok = true;
    auto al = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
        if (ok && hipMemset(*p, 0, bytes) != hipSuccess) ok = false;
    };
    al((void **)&m->P, P_TOTAL * 4);
    al((void **)&m->G, P_TOTAL * 4);
    al((void **)&m->Mm, P_TOTAL * 4);
    al((void **)&m->Vv, P_TOTAL * 4);
    al((void **)&m->W1, (size_t)D_IN * D_H * 2);
    al((void **)&m->W2, (size_t)D_H * D_H * 2);
    al((void **)&m->W3, (size_t)D_H * D_OUTP * 2);
    al((void **)&m->b3p, D_OUTP * 4);
    al((void **)&m->W1T, (size_t)D_H * D_INP * 2);
    al((void **)&m->W2T, (size_t)D_H * D_H * 2);
    al((void **)&m->W3T, (size_t)D_H * D_H * 2);
    al((void **)&m->X, (size_t)B_max * D_INP * 2);
    al((void **)&m->H1, (size_t)B_max * D_H * 2);
    al((void **)&m->H2, (size_t)B_max * D_H * 2);
    al((void **)&m->D, (size_t)B_max * D_OUTP * 2);
    al((void **)&m->D2, (size_t)B_max * D_H * 2);
    al((void **)&m->D1, (size_t)B_max * D_H * 2);
    al((void **)&m->PRE1, (size_t)B_max * D_H * 4);
    al((void **)&m->PRE2, (size_t)B_max * D_H * 4);
    al((void **)&m->OUT, (size_t)B_max * D_OUTP * 4);
    al((void **)&m->PART, (size_t)3 * MAX_SPLITS * (D_H + 1) * D_OUTP * 4);
    al((void **)&m->LP, (size_t)(2 * B_max + 4) * 4);
    al((void **)&m->adam_t, 4);
    al((void **)&m->UB, (size_t)B_max * N_H * 2 * 4);
    al((void **)&m->IDX, (size_t)B_max * 4);
    al((void **)&m->loss, 4);
    const size_t rows16 = (size_t)(B_max + 15) / 16 * 16;
    al((void **)&m->XB, rows16 * D_INP * 2);
    al((void **)&m->H1B, rows16 * D_H * 2);
    al((void **)&m->H2B, rows16 * D_H * 2);
    al((void **)&m->DB, rows16 * D_OUTP * 2);
    al((void **)&m->D2B, rows16 * D_H * 2);
    al((void **)&m->D1B, rows16 * D_H * 2);
    if (!ok) {
        sgtp_mlp_destroy(m);
        return SGTP_ENOMEM;
    }
    *out = m;
    return SGTP_OK;
}

int sgtp_mlp_destroy(sgtp_mlp *m) {
    if (!m) return SGTP_EINVAL;
    (void)hipDeviceSynchronize();
    void *bufs[] = {m->P,  m->G,  m->Mm, m->Vv,   m->W1,   m->W2,  m->W3, m->b3p, m->X,    m->H1,   m->H2,
                    m->D,  m->D1, m->PRE1, m->PRE2, m->OUT, m->PART, m->loss, m->W1T, m->W2T, m->W3T,
                    m->D2, m->LP, m->adam_t, m->UB, m->IDX, m->XB, m->H1B, m->H2B, m->DB, m->D2B, m->D1B};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete m;
    return SGTP_OK;
}

const char *sgtp_mlp_last_error(const sgtp_mlp *m) { return m ? m->err.c_str() : "null network"; }

int sgtp_mlp_num_params(void) { return (int)P_TOTAL; }

int sgtp_mlp_batch_max(const sgtp_mlp *m) { return m ? m->B_max : 0; }

int sgtp_mlp_set_params(sgtp_mlp *m, const float *host) {
    if (!m || !host) return SGTP_EINVAL;
    MCHK(m, hipMemcpy(m->P, host, P_TOTAL * 4, hipMemcpyHostToDevice));
    MCHK(m, hipMemset(m->Mm, 0, P_TOTAL * 4));
    MCHK(m, hipMemset(m->Vv, 0, P_TOTAL * 4));
    MCHK(m, hipMemset(m->adam_t, 0, 4));
    hipLaunchKernelGGL(k_refresh_bf16, dim3((D_H * D_OUTP + 255) / 256), dim3(256), 0, nullptr, m->P, m->W1, m->W2,
                       m->W3, m->b3p);
    hipLaunchKernelGGL(k_refresh_bf16_t, dim3((D_H * D_H + 255) / 256), dim3(256), 0, nullptr, m->P, m->W1T, m->W2T,
                       m->W3T);
    MCHK(m, hipGetLastError());
    MCHK(m, hipDeviceSynchronize());
    return SGTP_OK;
}

int sgtp_mlp_get_params(sgtp_mlp *m, float *host) {
    if (!m || !host) return SGTP_EINVAL;
    MCHK(m, hipDeviceSynchronize());
    MCHK(m, hipMemcpy(host, m->P, P_TOTAL * 4, hipMemcpyDeviceToHost));
    return SGTP_OK;
}

int sgtp_mlp_forward(sgtp_mlp *m, const float *X, int B, float *out, int ld_out, void *stream) {
    if (!m || !X || !out) return SGTP_EINVAL;
    if (B < 1 || B > m->B_max) return mfail(m, SGTP_ESHAPE, "batch larger than the network workspace");
    if (ld_out < D_OUT) return mfail(m, SGTP_EINVAL, "ld_out < 200");
    hipStream_t st = (hipStream_t)stream;
    if (B <= FUSED_MAX_ROWS) {  // planning-size batches: one fused kernel
        hipLaunchKernelGGL(k_mlp_fwd16<false>, dim3((B + 15) / 16), dim3(64 * FWD_WAVES), 0, st, X,
                           D_IN, B, m->W1T, m->W2T, m->W3T, m->P + P_B1, m->P + P_B2, m->P + P_B3, out, ld_out, D_OUT,
                           nullptr, nullptr, nullptr, nullptr, TrainIn{});
        MCHK(m, hipGetLastError());
        return SGTP_OK;
    }
    return forward(m, X, D_IN, B, out, ld_out, D_OUT, st);
}

namespace {
// Training batches up to this many rows take the fused forward (one launch, the hidden
// layers written out for the backward pass); larger ones the tiled products.  Both give
// the same bits.
constexpr int FUSED_TRAIN_MAX = 8192;

// Where the B rows of a gradient come from: features X [.][50] and targets U [.][N][2],
// row b of each, or (M > 0) rows drawn from a data set of M rows with Philox key (k0, k1)
struct RowSrc {
    const float *X, *U;
    long long M;
    uint32_t k0, k1;
};

// Adam's arguments over the network's parameters and moments
AdamArgs adam_args(sgtp_mlp *m, float lr, float beta1, float beta2, float eps) {
    const Bf16Copies copies{m->W1, m->W2, m->W3, m->W1T, m->W2T, m->W3T, m->b3p};
    return AdamArgs{m->P, m->Mm, m->Vv, lr, beta1, beta2, eps, m->adam_t, copies, 1};
}

// The gradient of B rows into m->G (and the loss); with ad, each gradient value also takes
// its Adam step inside the slice-sum launch, and *counted tells whether the step count was
// advanced on the way (by the fused input-gradient kernel) or is the caller's to advance.
int grad_rows(sgtp_mlp *m, const RowSrc &rs, int B, int N, float sig_a, float sig_d, float *loss, float *grads,
              hipStream_t st, const AdamArgs *ad = nullptr, bool *counted = nullptr) {
    if (counted) *counted = false;
    int n_lp;
    if (B <= FUSED_TRAIN_MAX) {  // fetch, forward and loss gradient in one launch
        // the weight gradients read the row-blocked copies; the row layouts of the features,
        // hidden activations and input gradients are not written (sgtp_mlp_workspace
        // rebuilds them from the blocked copies)
        const TrainIn ti{rs.U,  rs.M,  rs.k0, rs.k1, m->adam_t, m->IDX, nullptr, N,
                         sig_a, sig_d, m->D,  m->LP, m->XB,  m->H1B,    m->H2B,  m->DB};
        hipLaunchKernelGGL(k_mlp_fwd16<true>, dim3((B + 15) / 16), dim3(64 * FWD_WAVES), 0, st, rs.X,
                           D_IN, B, m->W1T, m->W2T, m->W3T, m->P + P_B1, m->P + P_B2, m->b3p, m->OUT, D_OUTP, D_OUTP,
                           m->PRE1, nullptr, m->PRE2, nullptr, ti);
        n_lp = 2 * B;
    } else {
        const float *U = rs.U;
        if (rs.M > 0) {
            hipLaunchKernelGGL(k_gather_sampled, dim3(B), dim3(128), 0, st, rs.X, rs.U, rs.M, N, rs.k0, rs.k1,
                               m->adam_t, m->X, m->UB, m->IDX);
            U = m->UB;
        } else {
            hipLaunchKernelGGL(k_to_bf16_rows, dim3((B * D_INP + 255) / 256), dim3(256), 0, st, rs.X, B, D_IN, D_IN,
                               m->X, D_INP);
        }
        int rc = forward_bf16(m, B, m->OUT, D_OUTP, D_OUTP, st);
        if (rc) return rc;
        const int nll_blocks = (B * 128 + 255) / 256;
        hipLaunchKernelGGL(k_nll, dim3(nll_blocks), dim3(256), 0, st, m->OUT, D_OUTP, U, B, N, sig_a, sig_d, m->D,
                           D_OUTP, m->LP);
        n_lp = 4 * nll_blocks;
    }
    // partial products of the three weight-and-bias gradients go to separate thirds of PART
    const size_t third = (size_t)MAX_SPLITS * (D_H + 1) * D_OUTP;
    if (B <= FUSED_TRAIN_MAX) {  // dH2 = D W3^T and dH1 = D2 W2^T in one launch
        hipLaunchKernelGGL(k_mlp_bwd16, dim3((B + 15) / 16), dim3(64 * FWD_WAVES), 0, st, m->D, m->W3, m->W2,
                           m->PRE2, m->PRE1, B, nullptr, nullptr, m->D2B, m->D1B, ad ? m->adam_t : nullptr);
        if (counted) *counted = ad != nullptr;
    } else {
        gemm(st, m->D, D_OUTP, 1, m->W3, 1, D_OUTP, B, D_H, D_OUTP, nullptr, nullptr, 0, m->D2, D_H, m->PRE2);
        gemm(st, m->D2, D_H, 1, m->W2, 1, D_H, B, D_H, D_H, nullptr, nullptr, 0, m->D1, D_H, m->PRE1);
    }
    FinishArgs fa{};
    GemmGroup grp{};
    // gW3 = H2^T D and gb3 = column sums of D (one product); gW2 = H1^T D2, gb2;
    // gW1 = X^T D1, gb1.  After the fused kernels the operands are read from their
    // row-blocked copies (same products, 16 consecutive k contiguous).
    if (B <= FUSED_TRAIN_MAX) {
        fa.s[0] = gemm_wgrad(grp, 0, m->PART, m->H2B, 16, 16 * D_H, m->DB, 16 * D_OUTP, 16, D_H, D_OUT, B,
                             m->G + P_W3, D_OUT, m->G + P_B3, k_splits(D_H, D_OUT, B), STAGE_BLK16);
        fa.s[1] = gemm_wgrad(grp, 1, m->PART + third, m->H1B, 16, 16 * D_H, m->D2B, 16 * D_H, 16, D_H, D_H, B,
                             m->G + P_W2, D_H, m->G + P_B2, k_splits(D_H, D_H, B), STAGE_BLK16);
        fa.s[2] = gemm_wgrad(grp, 2, m->PART + 2 * third, m->XB, 16, 16 * D_INP, m->D1B, 16 * D_H, 16, D_IN, D_H,
                             B, m->G + P_W1, D_H, m->G + P_B1, k_splits(D_IN, D_H, B), STAGE_BLK16);
    } else {
        fa.s[0] = gemm_wgrad(grp, 0, m->PART, m->H2, 1, D_H, m->D, D_OUTP, 1, D_H, D_OUT, B, m->G + P_W3, D_OUT,
                             m->G + P_B3, k_splits(D_H, D_OUT, B));
        fa.s[1] = gemm_wgrad(grp, 1, m->PART + third, m->H1, 1, D_H, m->D2, D_H, 1, D_H, D_H, B, m->G + P_W2, D_H,
                             m->G + P_B2, k_splits(D_H, D_H, B));
        fa.s[2] = gemm_wgrad(grp, 2, m->PART + 2 * third, m->X, 1, D_INP, m->D1, D_H, 1, D_IN, D_H, B,
                             m->G + P_W1, D_H, m->G + P_B1, k_splits(D_IN, D_H, B));
    }
    hipLaunchKernelGGL(k_gemm_bf16_group, dim3(grp.first[3]), dim3(256), 0, st, grp);
    // the slice sums and the loss in one launch
    fa.first[0] = 0;
    for (int l = 0; l < 3; ++l) fa.first[l + 1] = fa.first[l] + (fa.s[l].rows * fa.s[l].cols + 255) / 256;
    fa.lp = m->LP;
    fa.n_lp = n_lp;
    fa.B = B;
    fa.loss = m->loss;
    fa.loss2 = loss;
    fa.G = m->G;
    fa.adam_on = ad != nullptr;
    if (ad) {
        fa.adam = *ad;
        if (counted && *counted) fa.adam.t_add = 0;
    }
    hipLaunchKernelGGL(k_grad_finish, dim3(fa.first[3] + 1), dim3(256), 0, st, fa);
    MCHK(m, hipGetLastError());
    m->last_B = B;
    m->last_blocked = B <= FUSED_TRAIN_MAX;
    if (grads) MCHK(m, hipMemcpyAsync(grads, m->G, P_TOTAL * 4, hipMemcpyDeviceToDevice, st));
    return SGTP_OK;
}

int check_grad_args(sgtp_mlp *m, int B, int N, float sig_a, float sig_d) {
    if (B < 1 || B > m->B_max) return mfail(m, SGTP_ESHAPE, "batch larger than the network workspace");
    if (N < 1 || N > N_H) return mfail(m, SGTP_ESHAPE, "horizon outside [1, 50]");
    if (!(sig_a > 0.0f) || !(sig_d > 0.0f)) return mfail(m, SGTP_EINVAL, "plain scales must be positive");
    return SGTP_OK;
}
}  // namespace

int sgtp_mlp_grad(sgtp_mlp *m, const float *X, const float *U, int B, int N, float sig_a, float sig_d, float *loss,
                  float *grads, void *stream) {
    if (!m || !X || !U) return SGTP_EINVAL;
    if (int rc = check_grad_args(m, B, N, sig_a, sig_d)) return rc;
    m->last_sampled = false;
    return grad_rows(m, RowSrc{X, U, 0, 0, 0}, B, N, sig_a, sig_d, loss, grads, (hipStream_t)stream);
}

int sgtp_mlp_grad_sampled(sgtp_mlp *m, const float *X_all, const float *U_all, long long M, int B, int N,
                          unsigned long long seed, float sig_a, float sig_d, float *loss, float *grads, void *stream) {
    if (!m || !X_all || !U_all) return SGTP_EINVAL;
    if (M < 1 || M > 0x7fffffffLL) return mfail(m, SGTP_ESHAPE, "data set rows outside [1, 2^31 - 1]");
    if (int rc = check_grad_args(m, B, N, sig_a, sig_d)) return rc;
    m->last_sampled = true;
    return grad_rows(m, RowSrc{X_all, U_all, M, (uint32_t)seed, (uint32_t)(seed >> 32)}, B, N, sig_a, sig_d, loss,
                     grads, (hipStream_t)stream);
}

int sgtp_mlp_workspace(sgtp_mlp *m, int which, void *dst, void *stream) {
    if (!m || !dst) return SGTP_EINVAL;
    if (m->last_B < 1) return mfail(m, SGTP_EINVAL, "no gradient computed yet");
    const void *src = nullptr;
    size_t row = 0;
    if (m->last_blocked && (which == SGTP_MLP_WS_H1 || which == SGTP_MLP_WS_H2 || which == SGTP_MLP_WS_D2 ||
                            which == SGTP_MLP_WS_D1)) {
        const bf16 *blk = which == SGTP_MLP_WS_H1 ? m->H1B : which == SGTP_MLP_WS_H2 ? m->H2B
                          : which == SGTP_MLP_WS_D2 ? m->D2B : m->D1B;
        const long long n = (long long)m->last_B * D_H;
        hipLaunchKernelGGL(k_unblock, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, blk, D_H,
                           m->last_B, (bf16 *)dst);
        MCHK(m, hipGetLastError());
        return SGTP_OK;
    }
    switch (which) {
        case SGTP_MLP_WS_H1: src = m->H1; row = D_H * 2; break;
        case SGTP_MLP_WS_H2: src = m->H2; row = D_H * 2; break;
        case SGTP_MLP_WS_OUT: src = m->OUT; row = D_OUTP * 4; break;
        case SGTP_MLP_WS_D3: src = m->D; row = D_OUTP * 2; break;
        case SGTP_MLP_WS_D2: src = m->D2; row = D_H * 2; break;
        case SGTP_MLP_WS_D1: src = m->D1; row = D_H * 2; break;
        case SGTP_MLP_WS_IDX:
            if (!m->last_sampled) return mfail(m, SGTP_EINVAL, "the last gradient did not draw its rows");
            src = m->IDX;
            row = 4;
            break;
        default: return mfail(m, SGTP_EINVAL, "unknown workspace tensor");
    }
    MCHK(m, hipMemcpyAsync(dst, src, row * m->last_B, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SGTP_OK;
}

int sgtp_mlp_adam(sgtp_mlp *m, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!m) return SGTP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adam, dim3((P_TOTAL + 255) / 256), dim3(256), 0, st, adam_args(m, lr, beta1, beta2, eps),
                       m->G, (int)P_TOTAL);
    hipLaunchKernelGGL(k_step_count, dim3(1), dim3(64), 0, st, m->adam_t);
    MCHK(m, hipGetLastError());
    return SGTP_OK;
}

int sgtp_mlp_train_step_sampled(sgtp_mlp *m, const float *X_all, const float *U_all, long long M, int B, int N,
                                unsigned long long seed, float sig_a, float sig_d, float lr, float beta1, float beta2,
                                float eps, float *loss, void *stream) {
    if (!m || !X_all || !U_all) return SGTP_EINVAL;
    if (M < 1 || M > 0x7fffffffLL) return mfail(m, SGTP_ESHAPE, "data set rows outside [1, 2^31 - 1]");
    if (int rc = check_grad_args(m, B, N, sig_a, sig_d)) return rc;
    hipStream_t st = (hipStream_t)stream;
    m->last_sampled = true;
    const AdamArgs ad = adam_args(m, lr, beta1, beta2, eps);
    bool counted = false;
    if (int rc = grad_rows(m, RowSrc{X_all, U_all, M, (uint32_t)seed, (uint32_t)(seed >> 32)}, B, N, sig_a, sig_d,
                           loss, nullptr, st, &ad, &counted))
        return rc;
    if (!counted) hipLaunchKernelGGL(k_step_count, dim3(1), dim3(64), 0, st, m->adam_t);
    MCHK(m, hipGetLastError());
    return SGTP_OK;
}

int sgtp_gemm_bf16(const void *A, long long a_m, long long a_k, const void *B, long long b_k, long long b_n, int M,
                   int N, int K, const float *bias, float *C, long long ldc, void *stream) {
    if (!A || !B || !C || M < 1 || N < 1 || K < 1) return SGTP_EINVAL;
    gemm((hipStream_t)stream, (const bf16 *)A, a_m, a_k, (const bf16 *)B, b_k, b_n, M, N, K, bias, C, ldc, nullptr, 0);
    return hipGetLastError() == hipSuccess ? SGTP_OK : SGTP_EDEVICE;
}

}  // extern "C"
