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

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] = op(A)[M x K] * op(B)[K x N], BF16 inputs, FP32 accumulation.
// A is [M][K] (lda) or, if a_t, [K][M]; B is [K][N] (ldb) or, if b_t, [N][K].
// N must be a multiple of 64 and K of 32; rows m >= M are zero / not stored.
enum { EPI_BIAS_RELU_BF16 = 0, EPI_MASK_BF16 = 1, EPI_F32 = 2 };

constexpr int TM = 64, TN = 64, TK = 32, KP = TK + 8;  // LDS row pad against bank conflicts

__global__ __launch_bounds__(256) void gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A, int lda,
                                                 int a_t, const uint16_t *__restrict__ B, int ldb, int b_t,
                                                 int epi, const float *__restrict__ bias,
                                                 const uint16_t *__restrict__ mask, int ldm, uint16_t *out_bf,
                                                 float *out_f, int ldo) {
    __shared__ __align__(16) uint16_t As[TM][KP];
    __shared__ __align__(16) uint16_t Bs[TN][KP];  // n-major: Bs[n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
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
            for (int i = 0; i < 8; ++i) As[c + i][k] = (m + i < M) ? src[i] : (uint16_t)0;
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

// y[b] = H3[b] . w4 + b4 (one wavefront per row)
__global__ void out_layer(const uint16_t *H, const uint16_t *w4, const float *b4, int64_t M, float *y) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= M) return;
    float s = 0.f;
    for (int j = lane; j < kMlpHidden; j += 64) s += bf2f(H[row * kMlpHidden + j]) * bf2f(w4[j]);
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) y[row] = s + b4[0];
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

// column sums: out[j] = sum_b M[b][j] (bf16 or fp32 source), FP32, fixed order
__global__ void col_sum_bf16(const uint16_t *Mx, int B, int N, float *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += bf2f(Mx[(size_t)b * N + j]);
    out[j] = s;
}

// dW4[j] = sum_b H3[b][j] dy[b]; db4 = sum_b dy[b]
__global__ void out_grad(const uint16_t *H, const float *dy, int B, float *dw4, float *db4) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kMlpHidden) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += bf2f(H[(size_t)b * kMlpHidden + j]) * dy[b];
        dw4[j] = s;
    } else if (j == kMlpHidden) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += dy[b];
        db4[0] = s;
    }
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

// State features for the surrogate (64 values, BF16).
__global__ void features_kernel(const FeatArgs A) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.n) return;
    const HDX_CONST ModelHdr *M = (const HDX_CONST ModelHdr *)&A.model->h;
    float f[kMlpIn];
    for (int i = 0; i < kMlpIn; ++i) f[i] = 0.f;
    const int depth = A.depths ? A.depths[k] : A.depth_const;
    const float remain = (float)max(A.horizon - depth, 0) * 0.01f;
    if (M->kind == HDX_ROCKSAMPLE) {
        const int32_t w = A.states.w[k];
        const int x = w & 31, y = (w >> 5) & 31;
        const float inv = 1.0f / (float)M->grid;
        f[0] = (float)x * inv;
        f[1] = (float)y * inv;
        f[2] = (float)((w >> 30) & 1);
        f[3] = remain;
        const int m = M->n_rocks;
        for (int i = 0; i < m && 4 + 3 * i + 2 < kMlpIn; ++i) {
            f[4 + i] = (float)((w >> (10 + i)) & 1);
            f[4 + m + i] = (float)(M->rock_x[i] - x) * inv;
            f[4 + 2 * m + i] = (float)(M->rock_y[i] - y) * inv;
        }
    } else {
        const float s = A.states.s[k];
        const int32_t car = A.states.car[k];
        f[0] = s / M->path_len;
        f[1] = (float)(car & 0xff) / (float)max(M->n_levels - 1, 1);
        f[2] = (float)((car >> 8) & 1);
        f[3] = remain;
        const int P = min(M->n_peds, (kMlpIn - 4) / 3);
        for (int j = 0; j < P; ++j) {
            f[4 + 3 * j] = (A.states.px[j * A.states.stride + k] - s) * 0.1f;
            f[5 + 3 * j] = A.states.py[j * A.states.stride + k] * 0.1f;
            f[6 + 3 * j] = (float)A.states.goal[j * A.states.stride + k] / (float)M->n_goals;
        }
    }
    uint16_t *dst = A.X + k * kMlpIn;
    for (int i = 0; i < kMlpIn; ++i) dst[i] = f2bf(f[i]);
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t mlp_gemm(int M, int N, int K, const uint16_t *A, int lda, int a_t, const uint16_t *B, int ldb, int b_t,
                    int epi, const float *bias, const uint16_t *mask, int ldm, uint16_t *out_bf, float *out_f, int ldo,
                    hipStream_t s) {
    if (M <= 0) return hipSuccess;
    dim3 grid(N / TN, (M + TM - 1) / TM);
    hipLaunchKernelGGL(gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, lda, a_t, B, ldb, b_t, epi, bias, mask, ldm,
                       out_bf, out_f, ldo);
    return hipGetLastError();
}

// Forward pass of n rows in chunks of kMlpChunkRows; H1..H3 are scratch of
// min(n, kMlpChunkRows) rows x 256 bf16 (they hold the last chunk).
hipError_t mlp_forward(const MlpDev &P, const uint16_t *X, int64_t n, uint16_t *H1, uint16_t *H2, uint16_t *H3,
                       float *y, hipStream_t s) {
    const int H = kMlpHidden;
    for (int64_t r0 = 0; r0 < n; r0 += kMlpChunkRows) {
        const int rows = (int)std::min<int64_t>(kMlpChunkRows, n - r0);
        const uint16_t *x = X + r0 * kMlpIn;
        hipError_t e = mlp_gemm(rows, H, kMlpIn, x, kMlpIn, 0, P.w1b, H, 0, EPI_BIAS_RELU_BF16, P.b1, nullptr, 0,
                                H1, nullptr, H, s);
        if (e == hipSuccess)
            e = mlp_gemm(rows, H, H, H1, H, 0, P.w2b, H, 0, EPI_BIAS_RELU_BF16, P.b2, nullptr, 0, H2, nullptr, H, s);
        if (e == hipSuccess)
            e = mlp_gemm(rows, H, H, H2, H, 0, P.w3b, H, 0, EPI_BIAS_RELU_BF16, P.b3, nullptr, 0, H3, nullptr, H, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(out_layer, dim3(blocks_for(rows, 4)), dim3(256), 0, s, H3, P.w4b, P.b4, (int64_t)rows,
                           y + r0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
    hipLaunchKernelGGL(out_layer_back, dim3(blocks_for((int64_t)B * H, 256)), dim3(256), 0, s, S.dy, P.w4b, S.h3, B,
                       S.g3);
    hipLaunchKernelGGL(out_grad, dim3(blocks_for(H + 1, 256)), dim3(256), 0, s, S.h3, S.dy, B, gw4, gb4);
    // layer 3: dW3 = H2^T G3, db3 = colsum G3, G2 = (G3 W3^T) [H2 > 0]
    e = mlp_gemm(H, H, B, S.h2, H, 1, S.g3, H, 0, EPI_F32, nullptr, nullptr, 0, nullptr, gw3, H, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_sum_bf16, dim3(1), dim3(256), 0, s, S.g3, B, H, gb3);
    e = mlp_gemm(B, H, H, S.g3, H, 0, P.w3b, H, 1, EPI_MASK_BF16, nullptr, S.h2, H, S.g2, nullptr, H, s);
    if (e != hipSuccess) return e;
    // layer 2
    e = mlp_gemm(H, H, B, S.h1, H, 1, S.g2, H, 0, EPI_F32, nullptr, nullptr, 0, nullptr, gw2, H, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_sum_bf16, dim3(1), dim3(256), 0, s, S.g2, B, H, gb2);
    e = mlp_gemm(B, H, H, S.g2, H, 0, P.w2b, H, 1, EPI_MASK_BF16, nullptr, S.h1, H, S.g1, nullptr, H, s);
    if (e != hipSuccess) return e;
    // layer 1
    e = mlp_gemm(kMlpIn, H, B, X, kMlpIn, 1, S.g1, H, 0, EPI_F32, nullptr, nullptr, 0, nullptr, gw1, H, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_sum_bf16, dim3(1), dim3(256), 0, s, S.g1, B, H, gb1);
    return hipGetLastError();
}

hipError_t mlp_adam(MlpDev &P, const float *grads, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_step, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, grads, P.m, P.v,
                       (int64_t)kMlpParams, lr, b1, b2, eps, c1, c2, nullptr, P.pb);
    return hipGetLastError();
}

hipError_t mlp_refresh_bf16(MlpDev &P, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, (int64_t)kMlpParams, P.pb);
    return hipGetLastError();
}

hipError_t launch_features(const FeatArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(a.n, 128)), dim3(128), 0, s, a);
    return hipGetLastError();
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
// Surrogate lower bounds of one leaf's children: for action a (blockIdx.y)
// and child c, l0 = mean of the surrogate values of the child's scenarios,
// summed in grouped order; per-scenario values copied out on request.
__global__ void surrogate_reduce(const SurArgs A) {
    const int a = blockIdx.y;
    const int n = A.n;
    const float *v = A.values + (int64_t)a * n;
    const int nch = A.n_children[a];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nch && c < A.cap; c += gridDim.x * blockDim.x) {
        const int off = A.child_off[a * A.cap + c], cnt = A.child_n[a * A.cap + c];
        const int32_t *perm = A.perm + (int64_t)a * n;
        float s = 0.f;
        for (int i = 0; i < cnt; ++i) s = s + v[perm[off + i]];
        A.child_l0[a * A.cap + c] = s / (float)cnt;
    }
    if (A.L_out)
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
            A.L_out[(int64_t)a * n + k] = v[k];
}
}  // namespace

hipError_t launch_surrogate_reduce(const SurArgs &a, int n_actions, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(surrogate_reduce, dim3(1, n_actions), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t mlp_sum_loss(const float *part, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(64), 0, s, part, n, out);
    return hipGetLastError();
}
}  // namespace hdx
