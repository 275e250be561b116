// Surrogate MLP: parameter layout, device buffers and kernel launchers.
#pragma once

#include "internal.hpp"

namespace hdx {

constexpr int kMlpIn = HDX_MLP_IN;          // 64 features
constexpr int kMlpHidden = HDX_MLP_HIDDEN;  // 256
constexpr int64_t kMlpChunkRows = 1 << 16;  // largest training batch
// packed parameter vector: W1 [64][256], b1, W2 [256][256], b2, W3, b3, w4 [256], b4
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kMlpIn * kMlpHidden;
constexpr int64_t kOffW2 = kOffB1 + kMlpHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kMlpHidden * kMlpHidden;
constexpr int64_t kOffW3 = kOffB2 + kMlpHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kMlpHidden * kMlpHidden;
constexpr int64_t kOffW4 = kOffB3 + kMlpHidden;
constexpr int64_t kOffB4 = kOffW4 + kMlpHidden;
constexpr int64_t kMlpParams = kOffB4 + 1;
static_assert(kMlpParams == HDX_MLP_PARAMS, "parameter count");

constexpr int64_t kMlpWtElems = (int64_t)kMlpHidden * kMlpIn + 2 * (int64_t)kMlpHidden * kMlpHidden;
// partials of one training step: the weight gradients of the three layers
// over at most kMlpMaxSlices row slices, then the backward's per-block
// column sums (kMlpBwdPart floats per 128-row block)
constexpr int kMlpMaxSlices = 64;
constexpr int kMlpBwdPart = 4 * kMlpHidden + 8;
constexpr int64_t kMlpPartFloats =
    (int64_t)kMlpMaxSlices * (kMlpIn + 2 * kMlpHidden) * kMlpHidden + (kMlpChunkRows / 128) * (int64_t)kMlpBwdPart;

struct MlpDev {
    float *p;      // FP32 master parameters
    uint16_t *pb;  // BF16 copy
    uint16_t *pt;  // BF16 W1..W3 transposed ([out][in]) for the fused forward
    float *m, *v;  // Adam moments
    float *g;      // gradients
    const uint16_t *w1b, *w2b, *w3b, *w4b;
    const uint16_t *w1t, *w2t, *w3t;
    const float *b1, *b2, *b3, *b4;
};

struct MlpScratch {
    int64_t rows = 0;
    uint16_t *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
    float *y = nullptr;
    float *part = nullptr;  // kMlpPartFloats
};

struct FeatArgs {
    const DevModel *model;
    StatesPtr states;
    const int32_t *depths;  // per state, or NULL to use depth_const
    int64_t n;
    int32_t horizon, depth_const;
    uint16_t *X;
};

// y = MLP(X) for n rows; H1..H3 (row stride 256) receive the activations
// when non-NULL (then they hold n rows).
hipError_t mlp_forward(const MlpDev &P, const uint16_t *X, int64_t n, uint16_t *H1, uint16_t *H2, uint16_t *H3,
                       float *y, hipStream_t s);
hipError_t mlp_backward(const MlpDev &P, const uint16_t *X, const float *t, int B, MlpScratch &S, float *grads,
                        float *loss, hipStream_t s);
hipError_t mlp_adam(MlpDev &P, const float *grads, float lr, int step, hipStream_t s);
hipError_t mlp_refresh_bf16(MlpDev &P, hipStream_t s);
// Features of one state array (arguments by value), of up to kArgPack
// arrays (arguments in the kernel arguments), or of `count` arrays whose
// arguments are in device memory (n_max: the longest array).
constexpr int kArgPack = 8;       // a surrogate expansion of this many leaves takes the packs
constexpr int kMaxGridY = 65535;  // arrays per launch of the argument-array kernels
struct FeatPack {
    FeatArgs a[kArgPack];
};
static_assert(sizeof(FeatPack) <= 1024, "kernel argument pack too large");
hipError_t launch_features(const FeatArgs &a, hipStream_t s);
hipError_t launch_features_pack(const FeatPack &P, int count, int64_t n_max, hipStream_t s);
hipError_t launch_features_many(const FeatArgs *d_args, int count, int64_t n_max, hipStream_t s);

struct SurArgs {
    const float *values;  // [A][n] surrogate value per (action, scenario)
    const int16_t *perm;
    const int32_t *n_children, *child_n, *child_off;
    float *child_l0;
    float *L_out;  // optional [A][n]
    int32_t n, cap, n_actions, pad;
};
// Child means of up to kArgPack leaves (a pack in the kernel arguments) or
// of `count` leaves whose arguments are in device memory.
struct SurPack {
    SurArgs a[kArgPack];
};
static_assert(sizeof(SurPack) <= 1024, "kernel argument pack too large");
hipError_t launch_surrogate_reduce_pack(const SurPack &P, int count, int32_t n_actions_max, hipStream_t s);
hipError_t launch_surrogate_reduce(const SurArgs *d_args, int count, int32_t n_actions_max, hipStream_t s);

}  // namespace hdx
