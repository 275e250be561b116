// C ABI of the rollout-value surrogate: create, parameters, forward,
// gradients, training step (Adam) and state features.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "mlp.hpp"

using namespace hdx;

struct hdx_mlp {
    MlpDev P;
    MlpScratch S;
    float *grads = nullptr;
    float *loss = nullptr;
    int step = 0;
    void *sur = nullptr;  // scratch of surrogate expansions
    size_t sur_bytes = 0;
    // pinned staging of a surrogate expansion's per-leaf arguments (features,
    // child means), copied into `sur` in one transfer; rewritten once the
    // previous call's copy has run
    void *h_args = nullptr;
    size_t h_args_bytes = 0;
    hipEvent_t args_done = nullptr;
    bool args_used = false;
    hipEvent_t last = nullptr;  // completion of the latest call (orders calls across streams)
    std::mutex mu;
};

namespace {

// He-uniform initialisation from a splitmix64 sequence (host, deterministic)
uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void init_params(uint32_t seed, std::vector<float> &p) {
    uint64_t s = 0x6D6C7000ull ^ seed;
    auto uni = [&]() { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0; };
    auto fill = [&](int64_t off, int64_t n, double bound) {
        for (int64_t i = 0; i < n; ++i) p[off + i] = (float)(bound * uni());
    };
    fill(kOffW1, kOffB1 - kOffW1, sqrt(6.0 / kMlpIn));
    fill(kOffW2, kOffB2 - kOffW2, sqrt(6.0 / kMlpHidden));
    fill(kOffW3, kOffB3 - kOffW3, sqrt(6.0 / kMlpHidden));
    fill(kOffW4, kOffB4 - kOffW4, sqrt(3.0 / kMlpHidden));
}

bool grow_scratch(MlpScratch &S, int64_t rows) {
    if (S.rows >= rows) return true;
    for (void *ptr : {(void *)S.h1, (void *)S.h2, (void *)S.h3, (void *)S.g1, (void *)S.g2, (void *)S.g3,
                      (void *)S.y, (void *)S.part})
        if (ptr) hipFree(ptr);
    S = MlpScratch();
    const size_t hb = (size_t)rows * kMlpHidden * sizeof(uint16_t);
    if (hipMalloc(&S.h1, hb) != hipSuccess || hipMalloc(&S.h2, hb) != hipSuccess || hipMalloc(&S.h3, hb) != hipSuccess ||
        hipMalloc(&S.g1, hb) != hipSuccess || hipMalloc(&S.g2, hb) != hipSuccess || hipMalloc(&S.g3, hb) != hipSuccess ||
        hipMalloc(&S.y, rows * sizeof(float)) != hipSuccess ||
        hipMalloc(&S.part, kMlpPartFloats * sizeof(float)) != hipSuccess)
        return false;
    S.rows = rows;
    return true;
}

void bind(MlpDev &P) {
    P.w1b = P.pb + kOffW1;
    P.w2b = P.pb + kOffW2;
    P.w3b = P.pb + kOffW3;
    P.w4b = P.pb + kOffW4;
    P.w1t = P.pt;
    P.w2t = P.pt + (int64_t)kMlpHidden * kMlpIn;
    P.w3t = P.w2t + (int64_t)kMlpHidden * kMlpHidden;
    P.b1 = P.p + kOffB1;
    P.b2 = P.p + kOffB2;
    P.b3 = P.p + kOffB3;
    P.b4 = P.p + kOffB4;
}

StatesPtr to_states(const hdx_states &s) {
    StatesPtr p;
    p.w = s.w;
    p.s = s.s;
    p.car = s.car;
    p.px = s.px;
    p.py = s.py;
    p.goal = s.goal;
    p.stride = s.stride;
    return p;
}

// The handle's weights and scratch are shared by every call: each call
// waits for the previous one's work, whichever stream it ran on, and marks
// its own end.  Under stream capture the caller orders the work.
// HDX_E_DEVICE with the failing step and HIP's text in hdx_last_error.
hdx_status dev_fail(hdx_ctx *ctx, hipError_t e, const char *what) {
    char msg[256];
    snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    hdx_internal_set_error(ctx, msg);
    return HDX_E_DEVICE;
}

struct Ordered {
    hdx_mlp *m;
    hipStream_t s;
    bool on;
    Ordered(hdx_mlp *m_, hipStream_t s_) : m(m_), s(s_), on(false) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
        on = cs == hipStreamCaptureStatusNone && m->last != nullptr;
        if (on) hipStreamWaitEvent(s, m->last, 0);
    }
    ~Ordered() {
        if (on) hipEventRecord(m->last, s);
    }
};

}  // namespace

extern "C" {

hdx_status hdx_mlp_create(hdx_ctx *ctx, uint32_t seed, hdx_mlp **out) {
    if (!ctx || !out) return HDX_E_INVALID;
    *out = nullptr;
    hdx_mlp *m = new hdx_mlp();
    const size_t pbytes = kMlpParams * sizeof(float);
    if (hipMalloc(&m->P.p, pbytes) != hipSuccess || hipMalloc(&m->P.pb, kMlpParams * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&m->P.pt, kMlpWtElems * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&m->P.m, pbytes) != hipSuccess || hipMalloc(&m->P.v, pbytes) != hipSuccess ||
        hipMalloc(&m->grads, pbytes) != hipSuccess || hipMalloc(&m->loss, sizeof(float)) != hipSuccess ||
        hipEventCreateWithFlags(&m->last, hipEventDisableTiming) != hipSuccess) {
        hdx_mlp_destroy(ctx, m);
        return HDX_E_NOMEM;
    }
    bind(m->P);
    std::vector<float> p(kMlpParams, 0.0f);
    init_params(seed, p);
    hdx_status st = hdx_mlp_set_params(ctx, m, p.data());
    if (st != HDX_OK) {
        hdx_mlp_destroy(ctx, m);
        return st;
    }
    *out = m;
    return HDX_OK;
}

hdx_status hdx_mlp_destroy(hdx_ctx *ctx, hdx_mlp *m) {
    if (!ctx || !m) return HDX_E_INVALID;
    hipDeviceSynchronize();
    for (void *ptr : {(void *)m->P.p, (void *)m->P.pb, (void *)m->P.pt, (void *)m->P.m, (void *)m->P.v, (void *)m->grads,
                      (void *)m->loss, m->sur})
        if (ptr) hipFree(ptr);
    if (m->last) hipEventDestroy(m->last);
    if (m->args_done) hipEventDestroy(m->args_done);
    if (m->h_args) hipHostFree(m->h_args);
    for (void *ptr : {(void *)m->S.h1, (void *)m->S.h2, (void *)m->S.h3, (void *)m->S.g1, (void *)m->S.g2,
                      (void *)m->S.g3, (void *)m->S.y, (void *)m->S.part})
        if (ptr) hipFree(ptr);
    delete m;
    return HDX_OK;
}

hdx_status hdx_mlp_get_params(hdx_ctx *ctx, const hdx_mlp *m, float *host) {
    if (!ctx || !m || !host) return HDX_E_INVALID;
    return hipMemcpy(host, m->P.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? HDX_OK
                                                                                                   : HDX_E_DEVICE;
}

hdx_status hdx_mlp_set_params(hdx_ctx *ctx, hdx_mlp *m, const float *host) {
    if (!ctx || !m || !host) return HDX_E_INVALID;
    const size_t pbytes = kMlpParams * sizeof(float);
    if (hipMemcpy(m->P.p, host, pbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->P.m, 0, pbytes) != hipSuccess || hipMemset(m->P.v, 0, pbytes) != hipSuccess ||
        mlp_refresh_bf16(m->P, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return HDX_E_DEVICE;
    m->step = 0;
    return HDX_OK;
}

// Checkpoint file: magic, parameter count, Adam step, then the FP32
// parameters and the two Adam moments (little-endian, as in memory).
static const char kMlpMagic[8] = {'H', 'D', 'X', 'M', 'L', 'P', '0', '1'};

hdx_status hdx_mlp_save(hdx_ctx *ctx, hdx_mlp *m, const char *path) {
    if (!ctx || !m || !path) return HDX_E_INVALID;
    std::lock_guard<std::mutex> g(m->mu);
    const size_t n = kMlpParams;
    std::vector<float> buf(3 * n);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(buf.data(), m->P.p, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + n, m->P.m, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + 2 * n, m->P.v, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return HDX_E_DEVICE;
    FILE *f = fopen(path, "wb");
    if (!f) return HDX_E_INVALID;
    const int64_t count = (int64_t)n, step = m->step;
    const bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(&count, sizeof(count), 1, f) == 1 &&
                    fwrite(&step, sizeof(step), 1, f) == 1 && fwrite(buf.data(), sizeof(float), 3 * n, f) == 3 * n;
    return (fclose(f) == 0 && ok) ? HDX_OK : HDX_E_INVALID;
}

hdx_status hdx_mlp_load(hdx_ctx *ctx, hdx_mlp *m, const char *path) {
    if (!ctx || !m || !path) return HDX_E_INVALID;
    FILE *f = fopen(path, "rb");
    if (!f) return HDX_E_INVALID;
    char magic[8];
    int64_t count = 0, step = 0;
    const size_t n = kMlpParams;
    std::vector<float> buf(3 * n);
    const bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 &&
                    fread(&count, sizeof(count), 1, f) == 1 && count == (int64_t)n &&
                    fread(&step, sizeof(step), 1, f) == 1 && step >= 0 && step < (1ll << 31) &&
                    fread(buf.data(), sizeof(float), 3 * n, f) == 3 * n;
    fclose(f);
    if (!ok) return HDX_E_SHAPE;
    std::lock_guard<std::mutex> g(m->mu);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(m->P.p, buf.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->P.m, buf.data() + n, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->P.v, buf.data() + 2 * n, n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        mlp_refresh_bf16(m->P, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return HDX_E_DEVICE;
    m->step = (int)step;
    return HDX_OK;
}

hdx_status hdx_mlp_forward(hdx_ctx *ctx, hdx_mlp *m, const uint16_t *X, int64_t n, float *y, hdx_stream stream) {
    if (!ctx || !m || (n > 0 && (!X || !y)) || n < 0) return HDX_E_INVALID;
    if (n == 0) return HDX_OK;
    std::lock_guard<std::mutex> g(m->mu);
    Ordered o(m, (hipStream_t)stream);
    return mlp_forward(m->P, X, n, nullptr, nullptr, nullptr, y, (hipStream_t)stream) == hipSuccess ? HDX_OK
                                                                                                   : HDX_E_DEVICE;
}

hdx_status hdx_mlp_gradients(hdx_ctx *ctx, hdx_mlp *m, const uint16_t *X, const float *t, int32_t batch, float *grads,
                             float *loss, hdx_stream stream) {
    if (!ctx || !m || !X || !t || !grads) return HDX_E_INVALID;
    if (batch < 64 || batch % 64 != 0 || batch > kMlpChunkRows) return HDX_E_SHAPE;
    std::lock_guard<std::mutex> g(m->mu);
    if (!grow_scratch(m->S, batch)) return HDX_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    Ordered o(m, s);
    return mlp_backward(m->P, X, t, batch, m->S, grads, loss, s) == hipSuccess ? HDX_OK : HDX_E_DEVICE;
}

hdx_status hdx_mlp_train_step(hdx_ctx *ctx, hdx_mlp *m, const uint16_t *X, const float *t, int32_t batch, float lr,
                              float *loss, hdx_stream stream) {
    if (!ctx || !m || !X || !t || !(lr > 0.0f)) return HDX_E_INVALID;
    if (batch < 64 || batch % 64 != 0 || batch > kMlpChunkRows) return HDX_E_SHAPE;
    std::lock_guard<std::mutex> g(m->mu);
    if (!grow_scratch(m->S, batch)) return HDX_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    Ordered o(m, s);
    if (mlp_backward(m->P, X, t, batch, m->S, m->grads, loss, s) != hipSuccess) return HDX_E_DEVICE;
    m->step += 1;
    return mlp_adam(m->P, m->grads, lr, m->step, s) == hipSuccess ? HDX_OK : HDX_E_DEVICE;
}

hdx_status hdx_features(hdx_ctx *ctx, const hdx_model *model, hdx_states states, const int32_t *depths, int64_t n,
                        int32_t horizon, uint16_t *X, hdx_stream stream) {
    if (!ctx || !model || n < 0 || (n > 0 && (!depths || !X))) return HDX_E_INVALID;
    if (hdx_internal_desc(model)->kind == HDX_MARS || hdx_internal_desc(model)->kind == HDX_NAV) {
        hdx_internal_set_error(ctx, "no surrogate features for this model");
        return HDX_E_UNSUPPORTED;
    }
    if (n == 0) return HDX_OK;
    FeatArgs a;
    a.model = hdx_internal_devmodel(model);
    a.states = to_states(states);
    a.depths = depths;
    a.n = n;
    a.horizon = horizon;
    a.depth_const = 0;
    a.X = X;
    return launch_features(a, (hipStream_t)stream) == hipSuccess ? HDX_OK : HDX_E_DEVICE;
}

hdx_status hdx_expand_leaf_surrogate(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, hdx_mlp *mlp,
                                     int32_t horizon, hdx_stream stream) {
    if (!ctx || !mlp || n_leaves < 0 || (n_leaves > 0 && !leaves)) return HDX_E_INVALID;
    if (n_leaves == 0) return HDX_OK;
    // scratch: stepped states of every (action, scenario), their features and values
    std::vector<size_t> st_off(n_leaves), pair_off(n_leaves);
    size_t st_bytes = 0;
    int64_t pairs = 0;
    for (int32_t i = 0; i < n_leaves; ++i) {
        if (!leaves[i].model) return HDX_E_INVALID;
        const hdx_model_desc &d = *hdx_internal_desc(leaves[i].model);
        if (d.kind == HDX_MARS || d.kind == HDX_NAV) {
            hdx_internal_set_error(ctx, "no surrogate features for this model");
            return HDX_E_UNSUPPORTED;
        }
        const int64_t np = (int64_t)d.n_actions * (leaves[i].n > 0 ? leaves[i].n : 0);
        st_off[i] = st_bytes;
        pair_off[i] = (size_t)pairs;
        const size_t per = d.kind == HDX_ROCKSAMPLE ? 4 : (size_t)(8 + 9 * d.n_peds);
        st_bytes += ((size_t)np * per + 64) & ~(size_t)15;
        pairs += np;
    }
    std::lock_guard<std::mutex> g(mlp->mu);
    Ordered o(mlp, (hipStream_t)stream);
    const size_t args_off = (st_bytes + (size_t)pairs * (kMlpIn * sizeof(uint16_t) + sizeof(float)) + 255) & ~(size_t)255;
    const size_t args_bytes = (size_t)n_leaves * (sizeof(FeatArgs) + sizeof(SurArgs));
    const size_t need = args_off + args_bytes;
    if (mlp->sur_bytes < need) {
        if (mlp->sur) hipFree(mlp->sur);
        mlp->sur = nullptr;
        mlp->sur_bytes = 0;
        if (hipMalloc(&mlp->sur, need) != hipSuccess) return HDX_E_NOMEM;
        mlp->sur_bytes = need;
    }
    char *base = (char *)mlp->sur;
    uint16_t *X = (uint16_t *)(base + st_bytes);
    float *vals = (float *)(base + st_bytes + (size_t)pairs * kMlpIn * sizeof(uint16_t));
    // expansion without rollouts, stepped states kept
    std::vector<hdx_leaf> mod(leaves, leaves + n_leaves);
    for (int32_t i = 0; i < n_leaves; ++i) {
        const hdx_model_desc &d = *hdx_internal_desc(leaves[i].model);
        const int64_t np = (int64_t)d.n_actions * (leaves[i].n > 0 ? leaves[i].n : 0);
        hdx_leaf &L = mod[i];
        L.rollout.max_steps = 0;
        L.L = nullptr;
        if (d.kind == HDX_ROCKSAMPLE ? L.sprime.w != nullptr : L.sprime.s != nullptr) continue;  // caller's
        memset(&L.sprime, 0, sizeof(L.sprime));
        char *p = base + st_off[i];
        if (d.kind == HDX_ROCKSAMPLE) {
            L.sprime.w = (int32_t *)p;
        } else {
            L.sprime.s = (float *)p;
            L.sprime.car = (int32_t *)(p + 4 * np);
            L.sprime.px = (float *)(p + 8 * np);
            L.sprime.py = (float *)(p + (8 + 4 * (size_t)d.n_peds) * np);
            L.sprime.goal = (uint8_t *)(p + (8 + 8 * (size_t)d.n_peds) * np);
        }
        L.sprime.stride = np;
    }
    hdx_status st = hdx_expand_leaf(ctx, mod.data(), n_leaves, stream);
    if (st != HDX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<FeatArgs> fa;
    std::vector<SurArgs> sa;
    fa.reserve(n_leaves);
    sa.reserve(n_leaves);
    for (int32_t i = 0; i < n_leaves; ++i) {
        const int32_t A = hdx_model_actions(leaves[i].model);
        const int64_t np = (int64_t)A * (leaves[i].n > 0 ? leaves[i].n : 0);
        if (np == 0) continue;
        FeatArgs a;
        a.model = hdx_internal_devmodel(leaves[i].model);
        a.states = to_states(mod[i].sprime);
        a.depths = nullptr;
        a.depth_const = leaves[i].depth + 1;
        a.n = np;
        a.horizon = horizon;
        a.X = X + pair_off[i] * kMlpIn;
        fa.push_back(a);
        SurArgs r;
        r.values = vals + pair_off[i];
        r.perm = leaves[i].perm;
        r.n_children = leaves[i].n_children;
        r.child_n = leaves[i].child_n;
        r.child_off = leaves[i].child_off;
        r.child_l0 = leaves[i].child_l0;
        r.L_out = leaves[i].L;
        r.n = leaves[i].n;
        r.cap = leaves[i].cap;
        r.n_actions = A;
        r.pad = 0;
        sa.push_back(r);
    }
    if (fa.empty()) return HDX_OK;
    int64_t n_max = 0;
    int32_t a_max = 0;
    for (const FeatArgs &a : fa) n_max = std::max<int64_t>(n_max, a.n);
    for (const SurArgs &r : sa) a_max = std::max(a_max, r.n_actions);
    hipError_t e = hipSuccess;
    if (fa.size() <= (size_t)kArgPack) {
        // a few leaves (a search's expansion): the arguments travel in the
        // kernel arguments, no staging
        FeatPack fp;
        SurPack sp;
        memset(&fp, 0, sizeof(fp));
        memset(&sp, 0, sizeof(sp));
        std::copy(fa.begin(), fa.end(), fp.a);
        std::copy(sa.begin(), sa.end(), sp.a);
        if ((e = launch_features_pack(fp, (int)fa.size(), n_max, s)) != hipSuccess) return dev_fail(ctx, e, "features");
        if (pairs > 0 && (e = mlp_forward(mlp->P, X, pairs, nullptr, nullptr, nullptr, vals, s)) != hipSuccess)
            return dev_fail(ctx, e, "forward");
        if ((e = launch_surrogate_reduce_pack(sp, (int)sa.size(), a_max, s)) != hipSuccess)
            return dev_fail(ctx, e, "child means");
        return HDX_OK;
    }
    // many leaves: both argument arrays in one transfer from pinned staging
    if (mlp->args_used && (e = hipEventSynchronize(mlp->args_done)) != hipSuccess)
        return dev_fail(ctx, e, "argument staging wait");
    mlp->args_used = false;
    if (mlp->h_args_bytes < args_bytes) {
        if (mlp->h_args) hipHostFree(mlp->h_args);
        mlp->h_args = nullptr;
        mlp->h_args_bytes = 0;
        if (hipHostMalloc(&mlp->h_args, args_bytes) != hipSuccess) return HDX_E_NOMEM;
        mlp->h_args_bytes = args_bytes;
    }
    if (!mlp->args_done && (e = hipEventCreateWithFlags(&mlp->args_done, hipEventDisableTiming)) != hipSuccess)
        return dev_fail(ctx, e, "event");
    const size_t fa_bytes = fa.size() * sizeof(FeatArgs), sa_bytes = sa.size() * sizeof(SurArgs);
    memcpy(mlp->h_args, fa.data(), fa_bytes);
    memcpy((char *)mlp->h_args + fa_bytes, sa.data(), sa_bytes);
    FeatArgs *d_fa = (FeatArgs *)(base + args_off);
    SurArgs *d_sa = (SurArgs *)(base + args_off + fa_bytes);
    if ((e = hipMemcpyAsync(d_fa, mlp->h_args, fa_bytes + sa_bytes, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipEventRecord(mlp->args_done, s)) != hipSuccess)
        return dev_fail(ctx, e, "argument copy");
    mlp->args_used = true;
    if ((e = launch_features_many(d_fa, (int)fa.size(), n_max, s)) != hipSuccess) return dev_fail(ctx, e, "features");
    if (pairs > 0 && (e = mlp_forward(mlp->P, X, pairs, nullptr, nullptr, nullptr, vals, s)) != hipSuccess)
        return dev_fail(ctx, e, "forward");
    if ((e = launch_surrogate_reduce(d_sa, (int)sa.size(), a_max, s)) != hipSuccess)
        return dev_fail(ctx, e, "child means");
    return HDX_OK;
}

}  // extern "C"
