// Rollout-value surrogate: an MLP 64 -> 256 -> 256 -> 256 -> 1 with ReLU,
// BF16 weights and activations on MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, FP32 master weights and Adam; plus the state features it
// reads.  Forward, backward and the optimizer are hand-written kernels.
#include <math.h>
#include <string.h>

#include <vector>

#include "mlp.hpp"
#include "models.hpp"

namespace hdx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even; NaN stays NaN
    const uint32_t u = __float_as_uint(f);
    const uint32_t rn = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t special = (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);  // Inf, NaN
    return (uint16_t)(((u & 0x7f800000u) == 0x7f800000u) ? special : rn);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] = op(A)[M x K] * op(B)[K x N], BF16 inputs, FP32 accumulation.
// A is [M][K] (lda) or, if a_t, [K][M]; B is [K][N] (ldb) or, if b_t, [N][K].
// N must be a multiple of 64 and K of 32; rows m >= M are zero / not stored.
// blockIdx.z selects the k range [z kslice, (z + 1) kslice) (split K); with
// EPI_F32 slice z writes its partial product at out_f + z M ldo.
enum { EPI_BIAS_RELU_BF16 = 0, EPI_MASK_BF16 = 1, EPI_F32 = 2 };

constexpr int TM = 64, TN = 64, TK = 32, KP = TK + 8;  // LDS row pad against bank conflicts

__global__ __launch_bounds__(256) void gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                                                 int a_t, const uint16_t *__restrict__ B, int ldb, int b_t,
                                                 int epi, const float *__restrict__ bias,
                                                 const uint16_t *__restrict__ mask, int ldm, uint16_t *out_bf,
                                                 float *out_f, int ldo, int kslice) {
    __shared__ __align__(16) uint16_t As[TM][KP];
    __shared__ __align__(16) uint16_t Bs[TN][KP];  // n-major: Bs[n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kbeg = blockIdx.z * kslice, kend = min(K, kbeg + kslice);
    if (epi == EPI_F32) out_f += (size_t)blockIdx.z * M * ldo;
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        // A tile: 64 x 32 -> As[m][k]; 256 threads x 8 elements
        if (!a_t) {
            const int r = tid >> 2, c = (tid & 3) * 8;
            const int m = m0 + r;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (m < M) v = *(const uint4 *)(A + (size_t)m * lda + k0 + c);
            *(uint4 *)&As[r][c] = v;
        } else {
            const int k = tid >> 3, c = (tid & 7) * 8;  // 32 k rows x 64 m
            const int m = m0 + c;
            const uint16_t *src = A + (size_t)(k0 + k) * lda + m;
            if (m + 8 <= M) {
                const uint4 v = *(const uint4 *)src;
                const uint16_t *e = (const uint16_t *)&v;
                for (int i = 0; i < 8; ++i) As[c + i][k] = e[i];
            } else {
                for (int i = 0; i < 8; ++i) As[c + i][k] = (m + i < M) ? src[i] : (uint16_t)0;
            }
        }
        // B tile: 32 x 64 -> Bs[n][k]
        if (b_t) {
            const int r = tid >> 2, c = (tid & 3) * 8;  // B stored [N][K]
            *(uint4 *)&Bs[r][c] = *(const uint4 *)(B + (size_t)(n0 + r) * ldb + k0 + c);
        } else {
            const int k = tid >> 3, c = (tid & 7) * 8;  // B stored [K][N]
            const uint4 v = *(const uint4 *)(B + (size_t)(k0 + k) * ldb + n0 + c);
            const uint16_t *e = (const uint16_t *)&v;
            for (int i = 0; i < 8; ++i) Bs[c + i][k] = e[i];
        }
        __syncthreads();
        const int g = lane >> 4, q = lane & 15;
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8 *)&As[wm + i * 16 + q][g * 8];
        for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8 *)&Bs[wn + j * 16 + q][g * 8];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D layout: lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 tile
    const int g = lane >> 4, q = lane & 15;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + g * 4 + r;
                const int n = n0 + wn + j * 16 + q;
                if (m >= M) continue;
                const float v = acc[i][j][r];
                if (epi == EPI_BIAS_RELU_BF16) {
                    const float z = v + bias[n];
                    out_bf[(size_t)m * ldo + n] = f2bf(z > 0.f ? z : 0.f);
                } else if (epi == EPI_MASK_BF16) {
                    const bool on = mask[(size_t)m * ldm + n] != 0 && !(mask[(size_t)m * ldm + n] & 0x8000);
                    out_bf[(size_t)m * ldo + n] = f2bf(on ? v : 0.f);
                } else {
                    out_f[(size_t)m * ldo + n] = v;
                }
            }
}

// ---- fused forward --------------------------------------------------------
// One workgroup of four wavefronts takes kFR = 128 rows.  The layer input
// (X, then H1, H2) sits in LDS; wavefront w computes all 128 rows x columns
// [64 w, +64) with 16x16x32 BF16 MFMAs (8 x 4 accumulator tiles), its weight
// fragments read straight from the transposed BF16 weights, each fragment
// feeding eight row tiles.  The MFMA is
// fed (weights, activations), i.e. it produces the transposed tile, so a
// lane ends up holding four consecutive output columns of one row: the
// epilogue (bias, ReLU, BF16) writes them as one 8-byte LDS store.  The
// output layer sums each row's 256 products over a lane's 16 columns, the
// four lanes of the row, then the four column wavefronts, in a fixed order,
// so a row's value does not depend on the other rows.
constexpr int kFR = 128, kHP = kMlpHidden + 8, kFwdThreads = 256, kMI = kFR / 16;

// acc[i][j][r] = output (row 16 i + q, column nb + 16 j + 4 g + r)
template <int K>
__device__ __forceinline__ void fused_layer(const uint16_t (*Hs)[kHP], const uint16_t *__restrict__ wt, int nb,
                                            int lane, f32x4 (&acc)[kMI][4]) {
    const int g = lane >> 4, q = lane & 15;
#pragma unroll
    for (int i = 0; i < kMI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *wrow = wt + (size_t)(nb + q) * K + g * 8;
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8 *)(wrow + (size_t)j * 16 * K + k0);
#pragma unroll
        for (int i = 0; i < kMI; ++i) {
            const bf16x8 a = *(const bf16x8 *)&Hs[i * 16 + q][k0 + g * 8];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a, acc[i][j], 0, 0, 0);
        }
    }
}

// Two FP32 values rounded to BF16 (nearest even) and packed, lo in bits
// 0-15: one v_cvt_pk_bf16_f32 on gfx950.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const f32x2_t v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// h = bf16(relu(acc + bias)) into LDS (and, when STORE, to Hout)
template <bool STORE>
__device__ __forceinline__ void fused_store(uint16_t (*Hs)[kHP], const f32x4 (&acc)[kMI][4],
                                            const float *__restrict__ bias, int nb, int lane, uint16_t *Hout,
                                            int64_t r0, int64_t n) {
    const int g = lane >> 4, q = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = nb + j * 16 + g * 4;
        const float4 bv = *(const float4 *)(bias + col);
#pragma unroll
        for (int i = 0; i < kMI; ++i) {
            const int row = i * 16 + q;
            const uint2 v = make_uint2(pack_bf16(fmaxf(acc[i][j][0] + bv.x, 0.f), fmaxf(acc[i][j][1] + bv.y, 0.f)),
                                       pack_bf16(fmaxf(acc[i][j][2] + bv.z, 0.f), fmaxf(acc[i][j][3] + bv.w, 0.f)));
            *(uint2 *)&Hs[row][col] = v;
            if (STORE && r0 + row < n) *(uint2 *)(Hout + (r0 + row) * kMlpHidden + col) = v;
        }
    }
}

// STORE: also write H1..H3 (training); the inference form writes only y.
template <bool STORE>
__global__ __launch_bounds__(kFwdThreads, 2) void mlp_fused_fwd(const uint16_t *__restrict__ X, int64_t n,
                                                             const MlpDev P, float *__restrict__ y, uint16_t *H1,
                                                             uint16_t *H2, uint16_t *H3) {
    __shared__ __align__(16) uint16_t Hs[kFR][kHP];
    __shared__ float yp[4][kFR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, q = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * kFR;
    const int cw = wave, nb = cw * 64;
    constexpr int kV = kMlpIn / 8;  // uint4 per input row
    for (int i = tid; i < kFR * kV; i += kFwdThreads) {
        const int r = i / kV, c = (i % kV) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r0 + r < n) v = *(const uint4 *)(X + (r0 + r) * kMlpIn + c);
        *(uint4 *)&Hs[r][c] = v;
    }
    __syncthreads();
    f32x4 acc[kMI][4];
    fused_layer<kMlpIn>(Hs, P.w1t, nb, lane, acc);
    __syncthreads();
    fused_store<STORE>(Hs, acc, P.b1, nb, lane, H1, r0, n);
    __syncthreads();
    fused_layer<kMlpHidden>(Hs, P.w2t, nb, lane, acc);
    __syncthreads();
    fused_store<STORE>(Hs, acc, P.b2, nb, lane, H2, r0, n);
    __syncthreads();
    fused_layer<kMlpHidden>(Hs, P.w3t, nb, lane, acc);
    // output layer: y = bf16(h3) . bf16(w4) + b4
    float rowsum[kMI];
#pragma unroll
    for (int i = 0; i < kMI; ++i) rowsum[i] = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = nb + j * 16 + g * 4;
        const float4 bv = *(const float4 *)(P.b3 + col);
        const uint2 wv = *(const uint2 *)(P.w4b + col);
        const float w0 = __uint_as_float(wv.x << 16), w1 = __uint_as_float(wv.x & 0xffff0000u);
        const float w2 = __uint_as_float(wv.y << 16), w3 = __uint_as_float(wv.y & 0xffff0000u);
#pragma unroll
        for (int i = 0; i < kMI; ++i) {
            const int row = i * 16 + q;
            const uint32_t h01 = pack_bf16(fmaxf(acc[i][j][0] + bv.x, 0.f), fmaxf(acc[i][j][1] + bv.y, 0.f));
            const uint32_t h23 = pack_bf16(fmaxf(acc[i][j][2] + bv.z, 0.f), fmaxf(acc[i][j][3] + bv.w, 0.f));
            if (STORE && r0 + row < n) *(uint2 *)(H3 + (r0 + row) * kMlpHidden + col) = make_uint2(h01, h23);
            float s = rowsum[i];
            s += __uint_as_float(h01 << 16) * w0;
            s += __uint_as_float(h01 & 0xffff0000u) * w1;
            s += __uint_as_float(h23 << 16) * w2;
            s += __uint_as_float(h23 & 0xffff0000u) * w3;
            rowsum[i] = s;
        }
    }
#pragma unroll
    for (int i = 0; i < kMI; ++i) {
        float s = rowsum[i];
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (g == 0) yp[cw][i * 16 + q] = s;
    }
    __syncthreads();
    if (tid < kFR && r0 + tid < n) y[r0 + tid] = (((yp[0][tid] + yp[1][tid]) + yp[2][tid]) + yp[3][tid]) + P.b4[0];
}

// W1..W3 transposed to [out][in] (BF16), for the fused forward
__global__ void transpose_weights(const uint16_t *__restrict__ pb, uint16_t *__restrict__ pt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpWtElems) return;
    constexpr int64_t n1 = (int64_t)kMlpHidden * kMlpIn, n2 = (int64_t)kMlpHidden * kMlpHidden;
    int64_t o = i, base = kOffW1;
    int K = kMlpIn;
    if (o >= n1) {
        o -= n1;
        base = kOffW2;
        K = kMlpHidden;
        if (o >= n2) {
            o -= n2;
            base = kOffW3;
        }
    }
    const int64_t col = o / K, k = o % K;  // pt[col][k] = W[k][col]
    pt[i] = pb[base + k * kMlpHidden + col];
}

// dy = 2 (y - t) / B; per-block partial losses
__global__ void loss_grad(const float *y, const float *t, int B, float *dy, float *loss_part) {
    __shared__ float part[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < B) {
        const float e = y[i] - t[i];
        dy[i] = 2.f * e / (float)B;
        l = e * e / (float)B;
    }
    for (int d = 32; d > 0; d >>= 1) l += __shfl_xor(l, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// G3[b][j] = dy[b] w4[j] [H3[b][j] > 0]  (bf16)
__global__ void out_layer_back(const float *dy, const uint16_t *w4, const uint16_t *H, int B, uint16_t *G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * kMlpHidden) return;
    const int64_t b = i / kMlpHidden;
    const int j = (int)(i % kMlpHidden);
    const uint16_t h = H[i];
    const bool on = h != 0 && !(h & 0x8000);
    G[i] = f2bf(on ? dy[b] * bf2f(w4[j]) : 0.f);
}

// Partial weighted column sums over kMlpColRows-row slices:
// part[slice][j] = sum_b v(b, j) w(b), v = bf16 M[b][j] (1 without M),
// w = w[b] (1 without w); 64 columns x 4 row groups per block, fixed order.
__global__ __launch_bounds__(256) void wcolsum_part(const uint16_t *__restrict__ Mx, const float *__restrict__ w,
                                                    int B, int N, float *__restrict__ part) {
    __shared__ float red[4][64];
    const int tid = threadIdx.x, l = tid & 63, rg = tid >> 6;
    const int c = blockIdx.x * 64 + l;
    const int b0 = blockIdx.y * kMlpColRows, b1 = min(B, b0 + kMlpColRows);
    float s = 0.f;
    if (c < N)
        for (int b = b0 + rg; b < b1; b += 4) {
            float v = Mx ? bf2f(Mx[(size_t)b * N + c]) : 1.f;
            if (w) v *= w[b];
            s += v;
        }
    red[rg][l] = s;
    __syncthreads();
    if (rg == 0 && c < N) part[(size_t)blockIdx.y * N + c] = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
}

// out[i] = sum over slices z of part[z n + i], in slice order
__global__ void sum_slices(const float *__restrict__ part, int S, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(size_t)z * n + i];
    out[i] = s;
}

// Adam on FP32 master weights; refresh the BF16 copy of weight matrices
__global__ void adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                          float eps, float c1, float c2, const int64_t *bf_ranges, uint16_t *pbf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    const float np = p[i] - upd;
    p[i] = np;
    pbf[i] = f2bf(np);
}

__global__ void to_bf16(const float *src, int64_t n, uint16_t *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

// State features for the surrogate (64 values, BF16): RockSample x/n, y/n,
// terminal, remaining depth/100, rock qualities, rock offsets dx/n, dy/n;
// crowd driving s/path_len, speed level/(levels-1), terminal, remaining
// depth/100, then per pedestrian (px - s)/10, py/10, goal/n_goals; zeros
// to 64.  Feature j is a compile-time index, so nothing lives in private
// memory; a row is written as eight 16-byte stores.
template <int J>
__device__ __forceinline__ float rs_feature(const HDX_CONST ModelHdr *M, int32_t w, int x, int y, float inv,
                                            float remain) {
    if (J == 0) return (float)x * inv;
    if (J == 1) return (float)y * inv;
    if (J == 2) return (float)((w >> 30) & 1);
    if (J == 3) return remain;
    const int m = M->n_rocks, i = J - 4;
    if (i < m) return (float)((w >> ((10 + i) & 31)) & 1);  // i < m <= 20
    if (i < 2 * m) return (float)(M->rock_x[i - m] - x) * inv;
    if (i < 3 * m) return (float)(M->rock_y[i - 2 * m] - y) * inv;
    return 0.f;
}

template <int J>
__device__ __forceinline__ float ped_feature(const HDX_CONST ModelHdr *M, const StatesPtr &S, int64_t k, float s,
                                             int32_t car, float remain) {
    if (J == 0) return s / M->path_len;
    if (J == 1) return (float)(car & 0xff) / (float)max(M->n_levels - 1, 1);
    if (J == 2) return (float)((car >> 8) & 1);
    if (J == 3) return remain;
    constexpr int p = (J - 4) / 3, c = (J - 4) % 3;
    if (p >= M->n_peds) return 0.f;
    if (c == 0) return (S.px[p * S.stride + k] - s) * 0.1f;
    if (c == 1) return S.py[p * S.stride + k] * 0.1f;
    return (float)S.goal[p * S.stride + k] / (float)M->n_goals;
}

template <int J0>
__device__ __forceinline__ uint4 feature_chunk(const HDX_CONST ModelHdr *M, const StatesPtr &S, int64_t k, bool rs,
                                               int32_t w, int x, int y, float inv, float s, int32_t car, float remain) {
    float f[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = 0.f;
    if (rs) {
        f[0] = rs_feature<J0 + 0>(M, w, x, y, inv, remain);
        f[1] = rs_feature<J0 + 1>(M, w, x, y, inv, remain);
        f[2] = rs_feature<J0 + 2>(M, w, x, y, inv, remain);
        f[3] = rs_feature<J0 + 3>(M, w, x, y, inv, remain);
        f[4] = rs_feature<J0 + 4>(M, w, x, y, inv, remain);
        f[5] = rs_feature<J0 + 5>(M, w, x, y, inv, remain);
        f[6] = rs_feature<J0 + 6>(M, w, x, y, inv, remain);
        f[7] = rs_feature<J0 + 7>(M, w, x, y, inv, remain);
    } else {
        f[0] = ped_feature<J0 + 0>(M, S, k, s, car, remain);
        f[1] = ped_feature<J0 + 1>(M, S, k, s, car, remain);
        f[2] = ped_feature<J0 + 2>(M, S, k, s, car, remain);
        f[3] = ped_feature<J0 + 3>(M, S, k, s, car, remain);
        f[4] = ped_feature<J0 + 4>(M, S, k, s, car, remain);
        f[5] = ped_feature<J0 + 5>(M, S, k, s, car, remain);
        f[6] = ped_feature<J0 + 6>(M, S, k, s, car, remain);
        f[7] = ped_feature<J0 + 7>(M, S, k, s, car, remain);
    }
    uint4 v;
    v.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
    v.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
    v.z = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
    v.w = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
    return v;
}

// blockIdx.y selects the pack entry; rows of that entry by blockIdx.x.
__global__ __launch_bounds__(128) void features_kernel(const FeatPack P) {
    const FeatArgs &A = P.a[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.n) return;
    const HDX_CONST ModelHdr *M = (const HDX_CONST ModelHdr *)&A.model->h;
    const int depth = A.depths ? A.depths[k] : A.depth_const;
    const float remain = (float)max(A.horizon - depth, 0) * 0.01f;
    const bool rs = M->kind == HDX_ROCKSAMPLE;
    int32_t w = 0, car = 0;
    int x = 0, y = 0;
    float inv = 0.f, s = 0.f;
    if (rs) {
        w = A.states.w[k];
        x = w & 31;
        y = (w >> 5) & 31;
        inv = 1.0f / (float)M->grid;
    } else {
        s = A.states.s[k];
        car = A.states.car[k];
    }
    uint4 *dst = (uint4 *)(A.X + k * kMlpIn);
    dst[0] = feature_chunk<0>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[1] = feature_chunk<8>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[2] = feature_chunk<16>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[3] = feature_chunk<24>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[4] = feature_chunk<32>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[5] = feature_chunk<40>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[6] = feature_chunk<48>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
    dst[7] = feature_chunk<56>(M, A.states, k, rs, w, x, y, inv, s, car, remain);
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t mlp_gemm(int M, int N, int K, const uint16_t *A, int lda, int a_t, const uint16_t *B, int ldb, int b_t,
                    int epi, const float *bias, const uint16_t *mask, int ldm, uint16_t *out_bf, float *out_f, int ldo,
                    hipStream_t s, int slices) {
    if (M <= 0) return hipSuccess;
    if (slices < 1 || epi != EPI_F32) slices = 1;
    const int kslice = ((K + slices - 1) / slices + TK - 1) / TK * TK;
    slices = (K + kslice - 1) / kslice;
    dim3 grid(N / TN, (M + TM - 1) / TM, slices);
    hipLaunchKernelGGL(gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, lda, a_t, B, ldb, b_t, epi, bias, mask, ldm,
                       out_bf, out_f, ldo, kslice);
    return hipGetLastError();
}

namespace {

// dW[M x 256] = A^T G over B rows (A [B][M], G [B][256]), split over K
// into slices summed in a fixed order.
hipError_t weight_grad(int M, int B, const uint16_t *A, const uint16_t *G, float *out, float *part, hipStream_t s) {
    const int slices = std::max(1, std::min(kMlpMaxSlices, B / 512));
    if (slices == 1)
        return mlp_gemm(M, kMlpHidden, B, A, M, 1, G, kMlpHidden, 0, EPI_F32, nullptr, nullptr, 0, nullptr, out,
                        kMlpHidden, s, 1);
    hipError_t e = mlp_gemm(M, kMlpHidden, B, A, M, 1, G, kMlpHidden, 0, EPI_F32, nullptr, nullptr, 0, nullptr, part,
                            kMlpHidden, s, slices);
    if (e != hipSuccess) return e;
    const int kslice = ((B + slices - 1) / slices + TK - 1) / TK * TK;
    const int used = (B + kslice - 1) / kslice;
    const int64_t n = (int64_t)M * kMlpHidden;
    hipLaunchKernelGGL(sum_slices, dim3(blocks_for(n, 256)), dim3(256), 0, s, part, used, n, out);
    return hipGetLastError();
}

// out[j] = sum_b v(b, j) w(b) (see wcolsum_part), two passes, fixed order
hipError_t col_sum(const uint16_t *Mx, const float *w, int B, int N, float *out, float *part, hipStream_t s) {
    const int S = (B + kMlpColRows - 1) / kMlpColRows;
    hipLaunchKernelGGL(wcolsum_part, dim3((N + 63) / 64, S), dim3(256), 0, s, Mx, w, B, N, part);
    hipLaunchKernelGGL(sum_slices, dim3(blocks_for(N, 256)), dim3(256), 0, s, part, S, (int64_t)N, out);
    return hipGetLastError();
}

}  // namespace

// Forward pass of n rows: the fused kernel, 128 rows per workgroup.
hipError_t mlp_forward(const MlpDev &P, const uint16_t *X, int64_t n, uint16_t *H1, uint16_t *H2, uint16_t *H3,
                       float *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kFR - 1) / kFR;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (H1 && H2 && H3)
        hipLaunchKernelGGL(mlp_fused_fwd<true>, dim3((unsigned)blocks), dim3(kFwdThreads), 0, s, X, n, P, y, H1, H2,
                           H3);
    else
        hipLaunchKernelGGL(mlp_fused_fwd<false>, dim3((unsigned)blocks), dim3(kFwdThreads), 0, s, X, n, P, y,
                           nullptr, nullptr, nullptr);
    return hipGetLastError();
}

// Gradients of the mean squared error for one batch (B a multiple of 64).
hipError_t mlp_backward(const MlpDev &P, const uint16_t *X, const float *t, int B, MlpScratch &S, float *grads,
                        hipStream_t s) {
    const int H = kMlpHidden;
    hipError_t e = mlp_forward(P, X, B, S.h1, S.h2, S.h3, S.y, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_grad, dim3(blocks_for(B, 256)), dim3(256), 0, s, S.y, t, B, S.dy, S.loss_part);
    float *gw1 = grads + kOffW1, *gb1 = grads + kOffB1, *gw2 = grads + kOffW2, *gb2 = grads + kOffB2;
    float *gw3 = grads + kOffW3, *gb3 = grads + kOffB3, *gw4 = grads + kOffW4, *gb4 = grads + kOffB4;
    float *part = S.part, *cpart = S.part + (int64_t)kMlpMaxSlices * H * H;
    hipLaunchKernelGGL(out_layer_back, dim3(blocks_for((int64_t)B * H, 256)), dim3(256), 0, s, S.dy, P.w4b, S.h3, B,
                       S.g3);
    // output layer: dw4 = H3^T dy, db4 = sum dy
    if ((e = col_sum(S.h3, S.dy, B, H, gw4, cpart, s)) != hipSuccess) return e;
    if ((e = col_sum(nullptr, S.dy, B, 1, gb4, cpart, s)) != hipSuccess) return e;
    // layer 3: dW3 = H2^T G3, db3 = colsum G3, G2 = (G3 W3^T) [H2 > 0]
    if ((e = weight_grad(H, B, S.h2, S.g3, gw3, part, s)) != hipSuccess) return e;
    if ((e = col_sum(S.g3, nullptr, B, H, gb3, cpart, s)) != hipSuccess) return e;
    e = mlp_gemm(B, H, H, S.g3, H, 0, P.w3b, H, 1, EPI_MASK_BF16, nullptr, S.h2, H, S.g2, nullptr, H, s, 1);
    if (e != hipSuccess) return e;
    // layer 2
    if ((e = weight_grad(H, B, S.h1, S.g2, gw2, part, s)) != hipSuccess) return e;
    if ((e = col_sum(S.g2, nullptr, B, H, gb2, cpart, s)) != hipSuccess) return e;
    e = mlp_gemm(B, H, H, S.g2, H, 0, P.w2b, H, 1, EPI_MASK_BF16, nullptr, S.h1, H, S.g1, nullptr, H, s, 1);
    if (e != hipSuccess) return e;
    // layer 1
    if ((e = weight_grad(kMlpIn, B, X, S.g1, gw1, part, s)) != hipSuccess) return e;
    return col_sum(S.g1, nullptr, B, H, gb1, cpart, s);
}

hipError_t mlp_adam(MlpDev &P, const float *grads, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_step, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, grads, P.m, P.v,
                       (int64_t)kMlpParams, lr, b1, b2, eps, c1, c2, nullptr, P.pb);
    hipLaunchKernelGGL(transpose_weights, dim3(blocks_for(kMlpWtElems, 256)), dim3(256), 0, s, P.pb, P.pt);
    return hipGetLastError();
}

hipError_t mlp_refresh_bf16(MlpDev &P, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, (int64_t)kMlpParams, P.pb);
    hipLaunchKernelGGL(transpose_weights, dim3(blocks_for(kMlpWtElems, 256)), dim3(256), 0, s, P.pb, P.pt);
    return hipGetLastError();
}

hipError_t launch_features(const FeatArgs *a, int count, hipStream_t s) {
    for (int i0 = 0; i0 < count; i0 += kFeatPack) {
        FeatPack P;
        memset(&P, 0, sizeof(P));
        int64_t n_max = 0;
        const int c = std::min(kFeatPack, count - i0);
        for (int i = 0; i < c; ++i) {
            P.a[i] = a[i0 + i];
            n_max = std::max<int64_t>(n_max, a[i0 + i].n);
        }
        if (n_max <= 0) continue;
        const int64_t bx = (n_max + 127) / 128;
        if (bx > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(features_kernel, dim3((unsigned)bx, c), dim3(128), 0, s, P);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hdx

namespace hdx {
namespace {
__global__ void sum_parts(const float *part, int n, float *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s;
    }
}
}  // namespace

namespace {
// Surrogate lower bounds of the children of pack entry blockIdx.z: for
// action a (blockIdx.y) and child c, l0 = mean of the surrogate values of
// the child's scenarios; per-scenario values copied out on request.  With
// few children (RockSample: at most three) the wavefront takes one child at
// a time, lane l summing the child's grouped positions l, l + 64, ... in
// order and a fixed butterfly adding the lanes; with many small children
// (hashed observations) each lane sums one child in grouped order.
__global__ __launch_bounds__(64) void surrogate_reduce(const SurPack P) {
    const SurArgs &A = P.a[blockIdx.z];
    const int a = blockIdx.y;
    if (a >= A.n_actions) return;
    const int n = A.n, lane = threadIdx.x;
    const float *v = A.values + (int64_t)a * n;
    const int nch = min(A.n_children[a], A.cap);
    const int16_t *perm = A.perm + (int64_t)a * n;
    if (nch <= 16) {
        for (int c = 0; c < nch; ++c) {
            const int off = A.child_off[a * A.cap + c], cnt = A.child_n[a * A.cap + c];
            float sum = 0.f;
            for (int i = lane; i < cnt; i += 64) sum = sum + v[perm[off + i]];
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) sum = sum + __shfl_xor(sum, d, 64);
            if (lane == 0) A.child_l0[a * A.cap + c] = sum / (float)cnt;
        }
    } else {
        for (int c = lane; c < nch; c += 64) {
            const int off = A.child_off[a * A.cap + c], cnt = A.child_n[a * A.cap + c];
            float sum = 0.f;
            for (int i = 0; i < cnt; ++i) sum = sum + v[perm[off + i]];
            A.child_l0[a * A.cap + c] = sum / (float)cnt;
        }
    }
    if (A.L_out)
        for (int k = lane; k < n; k += 64) A.L_out[(int64_t)a * n + k] = v[k];
}
}  // namespace

hipError_t launch_surrogate_reduce(const SurArgs *a, int count, hipStream_t s) {
    for (int i0 = 0; i0 < count; i0 += kSurPack) {
        SurPack P;
        memset(&P, 0, sizeof(P));
        int A = 0;
        const int c = std::min(kSurPack, count - i0);
        for (int i = 0; i < c; ++i) {
            P.a[i] = a[i0 + i];
            A = std::max(A, a[i0 + i].n_actions);
        }
        if (A <= 0) continue;
        hipLaunchKernelGGL(surrogate_reduce, dim3(1, A, c), dim3(64), 0, s, P);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t mlp_sum_loss(const float *part, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(64), 0, s, part, n, out);
    return hipGetLastError();
}
}  // namespace hdx
