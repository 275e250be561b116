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

// A block's 128 rows of Hs out to H (rows below n), 16 bytes per thread
// per store: whole rows, coalesced.
__device__ __forceinline__ void copy_rows_out(const uint16_t (*Hs)[kHP], uint16_t *H, int64_t r0, int64_t n) {
    constexpr int kV = kMlpHidden / 8;
    for (int i = threadIdx.x; i < kFR * kV; i += kFwdThreads) {
        const int r = i / kV, c = (i % kV) * 8;
        if (r0 + r < n) *(uint4 *)(H + (r0 + r) * kMlpHidden + c) = *(const uint4 *)&Hs[r][c];
    }
}

// STORE: also write H1..H3 (training), through LDS as whole rows; the
// inference form writes only y.
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
    fused_store<false>(Hs, acc, P.b1, nb, lane, nullptr, r0, n);
    __syncthreads();
    if (STORE) copy_rows_out(Hs, H1, r0, n);
    fused_layer<kMlpHidden>(Hs, P.w2t, nb, lane, acc);
    __syncthreads();
    fused_store<false>(Hs, acc, P.b2, nb, lane, nullptr, r0, n);
    __syncthreads();
    if (STORE) copy_rows_out(Hs, H2, r0, n);
    fused_layer<kMlpHidden>(Hs, P.w3t, nb, lane, acc);
    if (STORE) __syncthreads();  // H3 goes through Hs once every wavefront has read H2
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
            if (STORE) *(uint2 *)&Hs[row][col] = make_uint2(h01, h23);
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
    if (STORE) copy_rows_out(Hs, H3, r0, n);
    if (tid < kFR && r0 + tid < n) y[r0 + tid] = (((yp[0][tid] + yp[1][tid]) + yp[2][tid]) + yp[3][tid]) + P.b4[0];
}

// ---- training step: fused backward, weight gradients, reductions --------
// Backward of one 128-row block, laid out as the fused forward: dy, then
// G3 = dy w4 [H3 > 0], G2 = (G3 W3^T) [H2 > 0] and G1 = (G2 W2^T) [H1 > 0]
// with 16x16x32 BF16 MFMAs (a row of W_l as stored, [in][out], holds an
// output column's products contiguously), each G rounded to BF16 and written
// out for the weight gradients; the block's column sums of G1..G3 (bias
// gradients), of dy H3 (dw4), of dy (db4) and its share of the loss go to
// its row of `part`, each sum in a fixed order.
constexpr int kBwdPart = kMlpBwdPart;  // db1, db2, db3, dw4 | db4, loss

__device__ __forceinline__ bool bf_on(uint32_t h) { return (h & 0xffffu) != 0 && !(h & 0x8000u); }

// A block's 128 rows of H (rows below B; zeros past them) into Hs, whole
// rows, 16 bytes per thread per load.
__device__ __forceinline__ void copy_rows_in(uint16_t (*Hs)[kHP], const uint16_t *H, int64_t r0, int64_t B) {
    constexpr int kV = kMlpHidden / 8;
    for (int i = threadIdx.x; i < kFR * kV; i += kFwdThreads) {
        const int r = i / kV, c = (i % kV) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < B) v = *(const uint4 *)(H + (r0 + r) * kMlpHidden + c);
        *(uint4 *)&Hs[r][c] = v;
    }
}

// One layer's G: the accumulators masked where H > 0 and rounded to BF16,
// H read from Hs (staged there by the caller), G written back into Hs; the
// block's column sums into colsum[col].  Hs is read, then (after a
// barrier) rewritten.
__device__ __forceinline__ void bwd_mask(uint16_t (*Hs)[kHP], const f32x4 (&acc)[kMI][4], int nb, int lane,
                                         float *colsum) {
    const int g = lane >> 4, q = lane & 15;
    uint2 gv[kMI][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = nb + j * 16 + g * 4;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
        for (int i = 0; i < kMI; ++i) {
            const uint2 hv = *(const uint2 *)&Hs[i * 16 + q][col];
            const uint32_t lo = pack_bf16(bf_on(hv.x) ? acc[i][j][0] : 0.f, bf_on(hv.x >> 16) ? acc[i][j][1] : 0.f);
            const uint32_t hi = pack_bf16(bf_on(hv.y) ? acc[i][j][2] : 0.f, bf_on(hv.y >> 16) ? acc[i][j][3] : 0.f);
            gv[i][j] = make_uint2(lo, hi);
            s0 += __uint_as_float(lo << 16);
            s1 += __uint_as_float(lo & 0xffff0000u);
            s2 += __uint_as_float(hi << 16);
            s3 += __uint_as_float(hi & 0xffff0000u);
        }
        // the 16 lanes of this column group hold the 128 rows: fixed butterfly
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            s0 += __shfl_xor(s0, d, 64);
            s1 += __shfl_xor(s1, d, 64);
            s2 += __shfl_xor(s2, d, 64);
            s3 += __shfl_xor(s3, d, 64);
        }
        if (q == 0) *(float4 *)(colsum + col) = make_float4(s0, s1, s2, s3);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < kMI; ++i) *(uint2 *)&Hs[i * 16 + q][nb + j * 16 + g * 4] = gv[i][j];
}

__global__ __launch_bounds__(kFwdThreads, 2) void mlp_fused_bwd(const float *__restrict__ y,
                                                             const float *__restrict__ t, int B,
                                                             const uint16_t *H1, const uint16_t *H2,
                                                             const uint16_t *H3, const MlpDev P, uint16_t *G1,
                                                             uint16_t *G2, uint16_t *G3, float *part) {
    __shared__ __align__(16) uint16_t Gs[kFR][kHP];
    __shared__ float dys[kFR];
    __shared__ float red[8][kMlpHidden];
    __shared__ float wred[2][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kFR;
    float *pb = part + (size_t)blockIdx.x * kBwdPart;
    // dy = 2 (y - t) / B; this block's db4 and loss
    if (tid < kFR) {
        const int64_t row = r0 + tid;
        float d = 0.f, l = 0.f;
        if (row < B) {
            const float e = y[row] - t[row];
            d = 2.f * e / (float)B;
            l = e * e / (float)B;
        }
        dys[tid] = d;
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            d += __shfl_xor(d, s, 64);
            l += __shfl_xor(l, s, 64);
        }
        if (lane == 0) {
            wred[wave][0] = d;
            wred[wave][1] = l;
        }
    }
    __syncthreads();
    if (tid == 0) {
        pb[4 * kMlpHidden] = wred[0][0] + wred[1][0];
        pb[4 * kMlpHidden + 1] = wred[0][1] + wred[1][1];
    }
    // G3 = bf16(dy w4) where H3 > 0: thread (row group rg of 16 rows, 8 columns c8)
    {
        const int c8 = (tid & 31) * 8, rg = tid >> 5;
        float w4[8];
        const uint4 wv = *(const uint4 *)(P.w4b + c8);
        const uint32_t wvw[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            w4[2 * e] = __uint_as_float(wvw[e] << 16);
            w4[2 * e + 1] = __uint_as_float(wvw[e] & 0xffff0000u);
        }
        float s3[8], s4[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s3[e] = s4[e] = 0.f;
        for (int rr = 0; rr < 16; ++rr) {
            const int row = rg * 16 + rr;
            const int64_t grow = r0 + row;
            uint4 hv = make_uint4(0u, 0u, 0u, 0u);
            if (grow < B) hv = *(const uint4 *)(H3 + grow * kMlpHidden + c8);
            const uint32_t hw[4] = {hv.x, hv.y, hv.z, hv.w};
            const float d = dys[row];
            uint32_t gw[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t h0 = hw[e] & 0xffffu, h1 = hw[e] >> 16;
                gw[e] = pack_bf16(bf_on(h0) ? d * w4[2 * e] : 0.f, bf_on(h1) ? d * w4[2 * e + 1] : 0.f);
                s3[2 * e] += __uint_as_float(gw[e] << 16);
                s3[2 * e + 1] += __uint_as_float(gw[e] & 0xffff0000u);
                s4[2 * e] += __uint_as_float(h0 << 16) * d;
                s4[2 * e + 1] += __uint_as_float(h1 << 16) * d;
            }
            const uint4 gv = make_uint4(gw[0], gw[1], gw[2], gw[3]);
            *(uint4 *)&Gs[row][c8] = gv;
            if (grow < B) *(uint4 *)(G3 + grow * kMlpHidden + c8) = gv;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) red[rg][c8 + e] = s3[e];
        __syncthreads();
        {
            float s = 0.f;
            for (int r = 0; r < 8; ++r) s += red[r][tid];
            pb[2 * kMlpHidden + tid] = s;  // db3
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) red[rg][c8 + e] = s4[e];
        __syncthreads();
        {
            float s = 0.f;
            for (int r = 0; r < 8; ++r) s += red[r][tid];
            pb[3 * kMlpHidden + tid] = s;  // dw4
        }
    }
    const int nb = wave * 64;
    f32x4 acc[kMI][4];
    __syncthreads();
    // G2 = (G3 W3^T) [H2 > 0]
    fused_layer<kMlpHidden>(Gs, P.w3b, nb, lane, acc);
    __syncthreads();
    copy_rows_in(Gs, H2, r0, B);
    __syncthreads();
    bwd_mask(Gs, acc, nb, lane, pb + kMlpHidden);
    __syncthreads();
    copy_rows_out(Gs, G2, r0, B);
    // G1 = (G2 W2^T) [H1 > 0]
    fused_layer<kMlpHidden>(Gs, P.w2b, nb, lane, acc);
    __syncthreads();
    copy_rows_in(Gs, H1, r0, B);
    __syncthreads();
    bwd_mask(Gs, acc, nb, lane, pb);
    __syncthreads();
    copy_rows_out(Gs, G1, r0, B);
}

// Weight gradients dW_l[M][256] = A_l^T G_l over the batch rows, split into
// row slices: workgroup (m tile of 64 rows of dW, slice, layer) accumulates
// its 64 x 256 tile over its slice with 16x16x32 BF16 MFMAs, wavefront w
// owning columns [64 w, 64 w + 64).  Per step of 32 batch rows the A and G
// tiles are staged in LDS transposed (k contiguous), two batch rows packed
// per 32-bit store.  Each slice writes its partial product; the slices are
// summed in order afterwards.
struct WgradArgs {
    const uint16_t *A[3];
    const uint16_t *G[3];
    float *out[3];
    int32_t M[3];
    int32_t B, kslice, slices;
};
constexpr int kWK = 32, kWP = kWK + 8;

// Tiles in a 1-D grid: the four m tiles of a slice of dW3, then of dW2, then
// dW1's one tile per slice.  Workgroup b runs on XCD b mod 8, each XCD with
// its own L2; consecutive tiles are dealt to one XCD so the m tiles of a
// slice read its G rows through one L2.
__global__ __launch_bounds__(256, 2) void wgrad_bf16(const WgradArgs W) {
    __shared__ __align__(16) uint16_t As[64][kWP];
    __shared__ __align__(16) uint16_t Gt[kMlpHidden][kWP];
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x8 = b & 7, base = nb >> 3, extra = nb & 7;
    const int J = x8 * base + min(x8, extra) + (b >> 3);
    const int S = W.slices;
    int layer, slice, mt;
    if (J < 8 * S) {
        layer = 2 - J / (4 * S);
        slice = (J % (4 * S)) >> 2;
        mt = J & 3;
    } else {
        layer = 0;
        slice = J - 8 * S;
        mt = 0;
    }
    const int M = W.M[layer], m0 = mt * 64;
    const uint16_t *A = W.A[layer], *G = W.G[layer];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, q = lane & 15;
    const int kbeg = slice * W.kslice, kend = min(W.B, kbeg + W.kslice);
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this thread's loads of one step: A (threads below 128: a row pair and a
    // chunk of 8 columns), G (two units of a row pair and a chunk)
    const int pa = tid & 15, ca = tid >> 4;
    uint4 ra[2], rg[2][2];
    auto load = [&](int k0) {
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        ra[0] = ra[1] = z;
        if (tid < 128) {
            const int r = k0 + 2 * pa;
            if (r < kend) ra[0] = *(const uint4 *)(A + (size_t)r * M + m0 + ca * 8);
            if (r + 1 < kend) ra[1] = *(const uint4 *)(A + (size_t)(r + 1) * M + m0 + ca * 8);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = tid + 256 * h, r = k0 + 2 * (u & 15), ch = u >> 4;
            rg[h][0] = rg[h][1] = z;
            if (r < kend) rg[h][0] = *(const uint4 *)(G + (size_t)r * kMlpHidden + ch * 8);
            if (r + 1 < kend) rg[h][1] = *(const uint4 *)(G + (size_t)(r + 1) * kMlpHidden + ch * 8);
        }
    };
    // two batch rows of 8 columns into 8 LDS rows (k contiguous), packed
    auto stash = [](uint16_t (*T)[kWP], int row0, int pr, const uint4 &v0, const uint4 &v1) {
        const uint32_t a0[4] = {v0.x, v0.y, v0.z, v0.w}, a1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            *(uint32_t *)&T[row0 + 2 * e][2 * pr] = (a0[e] & 0xffffu) | (a1[e] << 16);
            *(uint32_t *)&T[row0 + 2 * e + 1][2 * pr] = (a0[e] >> 16) | (a1[e] & 0xffff0000u);
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kWK) {
        if (tid < 128) stash(As, ca * 8, pa, ra[0], ra[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = tid + 256 * h;
            stash(Gt, (u >> 4) * 8, u & 15, rg[h][0], rg[h][1]);
        }
        __syncthreads();
        if (k0 + kWK < kend) load(k0 + kWK);  // the next step's loads fly during this step's products
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8 *)&As[i * 16 + q][g * 8];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8 *)&Gt[wave * 64 + j * 16 + q][g * 8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D: lane holds rows 4 g + r of each 16 x 16 tile, column q
    float *out = W.out[layer] + (size_t)slice * M * kMlpHidden;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(size_t)(m0 + i * 16 + g * 4 + r) * kMlpHidden + wave * 64 + j * 16 + q] = acc[i][j][r];
}

// The gradient vector from the partials, each sum in a fixed order.
// Weight matrices: element by element over the row slices, in slice order.
__global__ void reduce_wgrads(const float *__restrict__ wpart0, const float *__restrict__ wpart1,
                              const float *__restrict__ wpart2, int slices, float *__restrict__ grads) {
    constexpr int64_t n0 = (int64_t)kMlpIn * kMlpHidden, n1 = (int64_t)kMlpHidden * kMlpHidden;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0 + 2 * n1) return;
    const float *wp;
    int64_t o, n, dst;
    if (i < n0) {
        wp = wpart0, o = i, n = n0, dst = kOffW1 + i;
    } else if (i < n0 + n1) {
        wp = wpart1, o = i - n0, n = n1, dst = kOffW2 + o;
    } else {
        wp = wpart2, o = i - n0 - n1, n = n1, dst = kOffW3 + o;
    }
    // loads issued eight slices ahead; the sum stays in slice order
    float s = 0.f;
    int z = 0;
    for (; z + 8 <= slices; z += 8) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = wp[(size_t)(z + u) * n + o];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; z < slices; ++z) s += wp[(size_t)z * n + o];
    grads[dst] = s;
}

// Biases, w4, b4 and the loss over the blocks' partial rows: workgroup x
// takes 16 entries of a row, its 64 segments of consecutive blocks are
// summed in block order, then the segment sums in segment order.
constexpr int kRedSeg = 64, kRedCols = 16;
__global__ __launch_bounds__(kRedCols * kRedSeg) void reduce_bias(const float *__restrict__ bpart, int blocks,
                                                                   float *__restrict__ grads, float *loss) {
    __shared__ float seg[kRedSeg][kRedCols];
    const int c = threadIdx.x % kRedCols, sg = threadIdx.x / kRedCols;
    const int e = blockIdx.x * kRedCols + c;  // entry of a partial row
    const int per = (blocks + kRedSeg - 1) / kRedSeg;
    float s = 0.f;
    if (e < 4 * kMlpHidden + 2)
        for (int b = sg * per; b < min(blocks, (sg + 1) * per); ++b) s += bpart[(size_t)b * kBwdPart + e];
    seg[sg][c] = s;
    __syncthreads();
    if (sg == 0 && e < 4 * kMlpHidden + 2) {
        float t = 0.f;
        for (int k = 0; k < kRedSeg; ++k) t += seg[k][c];
        if (e < kMlpHidden) grads[kOffB1 + e] = t;
        else if (e < 2 * kMlpHidden) grads[kOffB2 + e - kMlpHidden] = t;
        else if (e < 3 * kMlpHidden) grads[kOffB3 + e - 2 * kMlpHidden] = t;
        else if (e < 4 * kMlpHidden) grads[kOffW4 + e - 3 * kMlpHidden] = t;
        else if (e == 4 * kMlpHidden) grads[kOffB4] = t;
        else if (loss) *loss = t;
    }
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

// Place of packed parameter i (an element of W1..W3) in the transposed
// BF16 weights ([out][in]), or -1 for the other parameters.
__device__ __forceinline__ int64_t transposed_at(int64_t i) {
    constexpr int64_t n1 = (int64_t)kMlpIn * kMlpHidden, n2 = (int64_t)kMlpHidden * kMlpHidden;
    int64_t o, base;
    int K;
    if (i >= kOffW1 && i < kOffB1) {
        o = i - kOffW1, base = 0, K = kMlpIn;
    } else if (i >= kOffW2 && i < kOffB2) {
        o = i - kOffW2, base = n1, K = kMlpHidden;
    } else if (i >= kOffW3 && i < kOffB3) {
        o = i - kOffW3, base = n1 + n2, K = kMlpHidden;
    } else {
        return -1;
    }
    const int64_t k = o / kMlpHidden, col = o % kMlpHidden;  // W[k][col]
    return base + col * K + k;
}

// Adam on FP32 master weights; the BF16 copy and its transpose refreshed in
// the same pass
__global__ void adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                          float eps, float c1, float c2, uint16_t *pbf, uint16_t *pt) {
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
    const uint16_t b = f2bf(np);
    pbf[i] = b;
    const int64_t ti = transposed_at(i);
    if (ti >= 0) pt[ti] = b;
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

// Features of row k of one state array.
template <class Args>
__device__ __forceinline__ void features_row(const Args &A, int64_t k) {
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

// One state array, its arguments by value.
__global__ __launch_bounds__(128) void features_one(const FeatArgs A) {
    features_row(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Many state arrays, their arguments in device memory (read through the
// constant address space); blockIdx.y selects the array.
__global__ __launch_bounds__(128) void features_many(const FeatArgs *args) {
    const HDX_CONST FeatArgs &A = ((const HDX_CONST FeatArgs *)args)[blockIdx.y];
    features_row(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// A few state arrays, their arguments in the kernel arguments.
__global__ __launch_bounds__(128) void features_pack(const FeatPack P) {
    features_row(P.a[blockIdx.y], (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

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

// Gradients of the mean squared error for one batch (B a multiple of 64):
// the fused forward storing H1..H3, the fused backward (G1..G3 and the
// per-block column sums), the split-K weight gradients of all three layers
// in one launch, and one pass summing every partial in a fixed order; the
// loss (when wanted) with it.
hipError_t mlp_backward(const MlpDev &P, const uint16_t *X, const float *t, int B, MlpScratch &S, float *grads,
                        float *loss, hipStream_t s) {
    hipError_t e = mlp_forward(P, X, B, S.h1, S.h2, S.h3, S.y, s);
    if (e != hipSuccess) return e;
    const int blocks = (B + kFR - 1) / kFR;
    float *wpart0 = S.part;
    int slices = std::max(1, std::min(kMlpMaxSlices, B / 1024));
    const int kslice = ((B + slices - 1) / slices + kWK - 1) / kWK * kWK;
    slices = (B + kslice - 1) / kslice;
    float *wpart1 = wpart0 + (size_t)slices * kMlpIn * kMlpHidden;
    float *wpart2 = wpart1 + (size_t)slices * kMlpHidden * kMlpHidden;
    float *bpart = wpart2 + (size_t)slices * kMlpHidden * kMlpHidden;
    hipLaunchKernelGGL(mlp_fused_bwd, dim3(blocks), dim3(kFwdThreads), 0, s, S.y, t, B, S.h1, S.h2, S.h3, P, S.g1,
                       S.g2, S.g3, bpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    WgradArgs W;
    W.A[0] = X, W.A[1] = S.h1, W.A[2] = S.h2;
    W.G[0] = S.g1, W.G[1] = S.g2, W.G[2] = S.g3;
    W.out[0] = wpart0, W.out[1] = wpart1, W.out[2] = wpart2;
    W.M[0] = kMlpIn, W.M[1] = kMlpHidden, W.M[2] = kMlpHidden;
    W.B = B;
    W.kslice = kslice;
    W.slices = slices;
    hipLaunchKernelGGL(wgrad_bf16, dim3(9 * slices), dim3(256), 0, s, W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_wgrads, dim3(blocks_for((int64_t)(kMlpIn + 2 * kMlpHidden) * kMlpHidden, 256)),
                       dim3(256), 0, s, wpart0, wpart1, wpart2, slices, grads);
    hipLaunchKernelGGL(reduce_bias, dim3((4 * kMlpHidden + 2 + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedSeg), 0,
                       s, bpart, blocks, grads, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(MlpDev &P, const float *grads, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_step, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, grads, P.m, P.v,
                       (int64_t)kMlpParams, lr, b1, b2, eps, c1, c2, P.pb, P.pt);
    return hipGetLastError();
}

hipError_t mlp_refresh_bf16(MlpDev &P, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, s, P.p, (int64_t)kMlpParams, P.pb);
    hipLaunchKernelGGL(transpose_weights, dim3(blocks_for(kMlpWtElems, 256)), dim3(256), 0, s, P.pb, P.pt);
    return hipGetLastError();
}

hipError_t launch_features(const FeatArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int64_t bx = (a.n + 127) / 128;
    if (bx > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(features_one, dim3((unsigned)bx), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_features_pack(const FeatPack &P, int count, int64_t n_max, hipStream_t s) {
    if (count <= 0 || n_max <= 0) return hipSuccess;
    const int64_t bx = (n_max + 127) / 128;
    if (bx > 0x7fffffff || count > kArgPack) return hipErrorInvalidValue;
    hipLaunchKernelGGL(features_pack, dim3((unsigned)bx, count), dim3(128), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_features_many(const FeatArgs *d_args, int count, int64_t n_max, hipStream_t s) {
    if (count <= 0 || n_max <= 0) return hipSuccess;
    const int64_t bx = (n_max + 127) / 128;
    if (bx > 0x7fffffff) return hipErrorInvalidValue;
    for (int i0 = 0; i0 < count; i0 += kMaxGridY) {
        const int c = std::min(kMaxGridY, count - i0);
        hipLaunchKernelGGL(features_many, dim3((unsigned)bx, c), dim3(128), 0, s, d_args + i0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
// Surrogate lower bounds of the children of one leaf: for action a
// (blockIdx.y) and child c, l0 = mean of the surrogate values of the
// child's scenarios; per-scenario values copied out on request.  With few
// children (RockSample: at most three) the wavefront takes one child at a
// time, lane l summing the child's grouped positions l, l + 64, ... in
// order and a fixed butterfly adding the lanes; with many small children
// (hashed observations) each lane sums one child in grouped order.
template <class Args>
__device__ __forceinline__ void child_means(const Args &A) {
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

// Leaf blockIdx.z of an argument array in device memory.
__global__ __launch_bounds__(64) void surrogate_reduce(const SurArgs *args) {
    child_means(((const HDX_CONST SurArgs *)args)[blockIdx.z]);
}

// Leaf blockIdx.z of a pack in the kernel arguments.
__global__ __launch_bounds__(64) void surrogate_reduce_pack(const SurPack P) { child_means(P.a[blockIdx.z]); }
}  // namespace

hipError_t launch_surrogate_reduce_pack(const SurPack &P, int count, int32_t n_actions_max, hipStream_t s) {
    if (count <= 0 || n_actions_max <= 0) return hipSuccess;
    if (count > kArgPack) return hipErrorInvalidValue;
    hipLaunchKernelGGL(surrogate_reduce_pack, dim3(1, n_actions_max, count), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_surrogate_reduce(const SurArgs *d_args, int count, int32_t n_actions_max, hipStream_t s) {
    if (count <= 0 || n_actions_max <= 0) return hipSuccess;
    for (int i0 = 0; i0 < count; i0 += kMaxGridY) {
        const int c = std::min(kMaxGridY, count - i0);
        hipLaunchKernelGGL(surrogate_reduce, dim3(1, n_actions_max, c), dim3(64), 0, s, d_args + i0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hdx
