// Host runtime behind the C ABI: context, model upload (device tables),
// argument validation, descriptor staging and kernel launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace hdx;

namespace {

constexpr int kSlots = 16;  // concurrent expand calls in flight per context
constexpr int kArgSlots = 8;  // argument blocks staged in device memory per context

// Pinned staging and device copy of one launch's argument block.
struct ArgSlot {
    void *h = nullptr, *d = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
};

// Pinned staging + device copy of one call's leaf descriptors and tiles.
struct Slot {
    LeafTask *h_tasks = nullptr, *d_tasks = nullptr;
    Tile *h_tiles = nullptr, *d_tiles = nullptr;
    TileQueue *h_queue = nullptr, *d_queue = nullptr;
    int64_t cap_tasks = 0, cap_tiles = 0;
    hipEvent_t done = nullptr;
    hipEvent_t fork = nullptr, join[kGroups] = {};  // launch groups run side by side
    bool used = false;
};

bool create_events(hipEvent_t *fork, hipEvent_t *join) {
    if (hipEventCreateWithFlags(fork, hipEventDisableTiming) != hipSuccess) return false;
    for (int c = 0; c < kGroups; ++c)
        if (hipEventCreateWithFlags(&join[c], hipEventDisableTiming) != hipSuccess) return false;
    return true;
}

void destroy_events(hipEvent_t *fork, hipEvent_t *join) {
    if (*fork) hipEventDestroy(*fork);
    *fork = nullptr;
    for (int c = 0; c < kGroups; ++c) {
        if (join[c]) hipEventDestroy(join[c]);
        join[c] = nullptr;
    }
}

uint64_t prob_threshold(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

}  // namespace

// ---- Fixed scratch of the expansion entry point that allocates nothing ----
// Leaf descriptors, the tile list and the tile queues of one call, at fixed
// offsets.  Each GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: host code uses only the per-device address that
// hipGetSymbolAddress returns (kept in g_scratch_addr).
namespace {
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaTasksOff = 0;
constexpr size_t kNaTilesOff = align256((size_t)HDX_NOALLOC_MAX_LEAVES * sizeof(LeafTask));
constexpr size_t kNaQueueOff = kNaTilesOff + align256((size_t)HDX_NOALLOC_MAX_TILES * sizeof(Tile));
constexpr size_t kNaBytes = kNaQueueOff + align256((size_t)kGroups * sizeof(TileQueue));
static_assert(kNaBytes <= HDX_NOALLOC_SCRATCH_BYTES, "no-allocation scratch larger than documented");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_addr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of this device's scratch copy; call with `device` current.
static hipError_t scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = (unsigned char *)ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

struct hdx_ctx {
    int32_t device = 0;
    int32_t n_cu = 256;
    std::string err;
    std::mutex mu;
    Slot slots[kSlots];
    int next_slot = 0;
    hipStream_t cls_stream[kGroups] = {};  // one stream per launch group (default priority)
    Schedule sched{256, 0, 1};
    bool sched_fixed = false;
    ArgSlot arg_slots[kArgSlots];
    int next_arg_slot = 0;
    // expansion without allocation: the device's fixed scratch array (its
    // address from hipGetSymbolAddress), pinned host staging and events made
    // here at set-up, and fixed host arrays for planning
    unsigned char *na_scratch = nullptr;
    LeafTask *na_h_tasks = nullptr;
    Tile *na_h_tiles = nullptr;
    TileQueue *na_h_queue = nullptr;
    hipEvent_t na_done = nullptr, na_fork = nullptr, na_join[kGroups] = {};
    bool na_used = false;
    int8_t na_var[HDX_NOALLOC_MAX_LEAVES];
    int32_t na_order[HDX_NOALLOC_MAX_LEAVES];
};

struct hdx_model {
    hdx_model_desc desc;
    DevModel *d_model = nullptr;
};

// Error texts go into a string whose capacity hdx_init reserves, so
// reporting an error allocates nothing.
constexpr size_t kErrCap = 512;

static hdx_status fail(hdx_ctx *ctx, hdx_status code, const char *msg) {
    if (ctx) ctx->err.assign(msg, strnlen(msg, kErrCap - 1));
    return code;
}

static hdx_status hip_fail(hdx_ctx *ctx, hipError_t e, const char *what) {
    char buf[kErrCap];
    snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    return fail(ctx, HDX_E_DEVICE, buf);
}

extern "C" {

const char *hdx_version(void) { return "hdx 0.1 (gfx950)"; }

hdx_status hdx_init(int32_t device, hdx_ctx **out) {
    if (!out) return HDX_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HDX_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HDX_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HDX_E_DEVICE;
    hdx_ctx *ctx = new hdx_ctx();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    for (int c = 0; c < kGroups; ++c)
        if (hipStreamCreateWithFlags(&ctx->cls_stream[c], hipStreamNonBlocking) != hipSuccess) {
            hdx_fini(ctx);
            return HDX_E_DEVICE;
        }
    for (auto &s : ctx->slots) {
        if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess || !create_events(&s.fork, s.join)) {
            hdx_fini(ctx);
            return HDX_E_DEVICE;
        }
        if (hipMalloc(&s.d_queue, kGroups * sizeof(TileQueue)) != hipSuccess ||
            hipHostMalloc(&s.h_queue, kGroups * sizeof(TileQueue)) != hipSuccess ||
            hipMemset(s.d_queue, 0, kGroups * sizeof(TileQueue)) != hipSuccess) {
            hdx_fini(ctx);
            return HDX_E_NOMEM;
        }
    }
    if (configure_expand_kernels() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        hdx_fini(ctx);
        return HDX_E_DEVICE;
    }
    for (auto &a : ctx->arg_slots)
        if (hipHostMalloc(&a.h, sizeof(SampleArgs)) != hipSuccess || hipMalloc(&a.d, sizeof(SampleArgs)) != hipSuccess ||
            hipEventCreateWithFlags(&a.done, hipEventDisableTiming) != hipSuccess) {
            hdx_fini(ctx);
            return HDX_E_NOMEM;
        }
    // set-up of hdx_expand_leaf_noalloc: the scratch's device address, host
    // staging and events, so that the call itself allocates nothing
    ctx->err.reserve(kErrCap);
    if (scratch_address(device, &ctx->na_scratch) != hipSuccess) {
        hdx_fini(ctx);
        return HDX_E_DEVICE;
    }
    if (hipHostMalloc((void **)&ctx->na_h_tasks, HDX_NOALLOC_MAX_LEAVES * sizeof(LeafTask)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->na_h_tiles, HDX_NOALLOC_MAX_TILES * sizeof(Tile)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->na_h_queue, kGroups * sizeof(TileQueue)) != hipSuccess) {
        hdx_fini(ctx);
        return HDX_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&ctx->na_done, hipEventDisableTiming) != hipSuccess ||
        !create_events(&ctx->na_fork, ctx->na_join)) {
        hdx_fini(ctx);
        return HDX_E_DEVICE;
    }
    *out = ctx;
    return HDX_OK;
}

hdx_status hdx_fini(hdx_ctx *ctx) {
    if (!ctx) return HDX_E_INVALID;
    hipSetDevice(ctx->device);
    for (auto &s : ctx->slots) {
        if (s.done) hipEventSynchronize(s.done);
        if (s.h_tasks) hipHostFree(s.h_tasks);
        if (s.h_tiles) hipHostFree(s.h_tiles);
        if (s.d_tasks) hipFree(s.d_tasks);
        if (s.d_tiles) hipFree(s.d_tiles);
        if (s.d_queue) hipFree(s.d_queue);
        if (s.h_queue) hipHostFree(s.h_queue);
        if (s.done) hipEventDestroy(s.done);
        destroy_events(&s.fork, s.join);
    }
    if (ctx->na_done) {
        hipEventSynchronize(ctx->na_done);
        hipEventDestroy(ctx->na_done);
    }
    for (auto &a : ctx->arg_slots) {
        if (a.done) {
            hipEventSynchronize(a.done);
            hipEventDestroy(a.done);
        }
        if (a.h) hipHostFree(a.h);
        if (a.d) hipFree(a.d);
    }
    destroy_events(&ctx->na_fork, ctx->na_join);
    if (ctx->na_h_tasks) hipHostFree(ctx->na_h_tasks);
    if (ctx->na_h_tiles) hipHostFree(ctx->na_h_tiles);
    if (ctx->na_h_queue) hipHostFree(ctx->na_h_queue);
    for (int c = 0; c < kGroups; ++c)
        if (ctx->cls_stream[c]) hipStreamDestroy(ctx->cls_stream[c]);
    delete ctx;
    return HDX_OK;
}

const char *hdx_last_error(const hdx_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hdx_status hdx_upload_model(hdx_ctx *ctx, const hdx_model_desc *d, hdx_model **out) {
    if (!ctx || !d || !out) return fail(ctx, HDX_E_INVALID, "null argument");
    *out = nullptr;
    if (!(d->gamma > 0.0 && d->gamma <= 1.0)) return fail(ctx, HDX_E_INVALID, "gamma must be in (0, 1]");
    DevModel *dm = new DevModel();
    memset(dm, 0, sizeof(DevModel));
    ModelHdr *h = &dm->h;
    h->kind = d->kind;
    if (d->kind == HDX_ROCKSAMPLE || d->kind == HDX_MARS) {
        const int g_min = d->kind == HDX_MARS ? 2 : 1;
        if (d->grid < g_min || d->grid > kMaxGrid || d->n_rocks < 0 || d->n_rocks > kMaxRocks) {
            delete dm;
            return fail(ctx, HDX_E_SHAPE, "grid must be 1..31 (2..31 for two robots) and rocks 0..20");
        }
        h->n_actions = d->kind == HDX_MARS ? (5 + d->n_rocks) * (5 + d->n_rocks) : 5 + d->n_rocks;
        // exact for every a < (5 + n_rocks)^2 with 5 + n_rocks <= 25 (checked exhaustively)
        h->joint_inv = (65536 + 4 + d->n_rocks) / (5 + d->n_rocks);
        h->grid = d->grid;
        h->n_rocks = d->n_rocks;
        std::vector<int8_t> rock_at(kMaxGrid * kMaxGrid, -1);
        for (int i = 0; i < d->n_rocks; ++i) {
            const int x = d->rock_x[i], y = d->rock_y[i];
            if (x < 0 || x >= d->grid || y < 0 || y >= d->grid || rock_at[x + y * d->grid] >= 0) {
                delete dm;
                return fail(ctx, HDX_E_INVALID, "rocks must lie on distinct grid cells");
            }
            h->rock_x[i] = x;
            h->rock_y[i] = y;
            rock_at[x + y * d->grid] = (int8_t)i;
        }
        // sensor accuracy 0.5 + 0.5 * 2^(-d/20) as a threshold on a 32-bit word
        for (int d2 = 0; d2 < kSenseEntries; ++d2) {
            const double acc = 0.5 + 0.5 * pow(2.0, -sqrt((double)d2) / 20.0);
            dm->sense_thr_m1[d2] = (uint32_t)(prob_threshold(acc) - 1);
        }
    } else if (d->kind == HDX_NAV) {
        const int n = d->grid;
        if (n < 5 || n > HDX_MAX_NAV_GRID) {
            delete dm;
            return fail(ctx, HDX_E_SHAPE, "navigation grid must be 5..16");
        }
        int n_unknown = 0;
        bool ok = d->nav_wall >= 1 && d->nav_wall <= n - 2 && d->nav_goal_x >= 0 && d->nav_goal_x < n &&
                  d->nav_gate_x[0] >= 0 && d->nav_gate_x[0] < n && d->nav_gate_x[1] >= 0 && d->nav_gate_x[1] < n &&
                  d->p_fail >= 0.0 && d->p_fail < 1.0 && d->p_err >= 0.0 && d->p_err < 1.0;
        std::vector<int> seen(HDX_MAX_NAV_UNKNOWN, 0);
        for (int c = 0; ok && c < n * n; ++c) {
            const int v = d->nav_cell[c];
            if (v >= HDX_MAX_NAV_UNKNOWN || v < -2 || (v >= 0 && seen[v]++)) ok = false;
            else if (v >= 0) ++n_unknown;
        }
        // unknown cells are numbered 0..n_unknown-1; 0 and 1 are the gates; the goal is known free
        for (int v = 0; ok && v < n_unknown; ++v) ok = seen[v] == 1;
        ok = ok && n_unknown >= 2 && d->nav_cell[d->nav_wall * n + d->nav_gate_x[0]] == 0 &&
             d->nav_cell[d->nav_wall * n + d->nav_gate_x[1]] == 1 && d->nav_cell[(n - 1) * n + d->nav_goal_x] == -1;
        if (!ok) {
            delete dm;
            return fail(ctx, HDX_E_INVALID, "navigation map, gates, goal or probabilities");
        }
        h->n_actions = 9;
        h->grid = n;
        h->nav_goal_x = d->nav_goal_x;
        h->nav_wall = d->nav_wall;
        h->nav_gate_x[0] = d->nav_gate_x[0];
        h->nav_gate_x[1] = d->nav_gate_x[1];
        for (int c = 0; c < HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID; ++c) h->nav_cell[c] = c < n * n ? d->nav_cell[c] : -2;
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int v = d->nav_cell[y * n + x], bit = 16 * y + x;
                if (v == -2) h->nav_wall_bits[bit >> 6] |= 1ull << (bit & 63);
                if (v >= 0) h->nav_unknown_pos[v] = (uint8_t)bit;
            }
        h->fail_thr = prob_threshold(d->p_fail);
        h->err_thr = prob_threshold(d->p_err);
    } else if (d->kind == HDX_PEDNAV) {
        if (d->n_peds < 0 || d->n_peds > kMaxPeds || d->n_goals < 1 || d->n_goals > kMaxGoals ||
            d->n_levels < 1 || d->n_levels > 255) {
            delete dm;
            return fail(ctx, HDX_E_SHAPE, "pedestrians 0..32, goals 1..8, levels 1..255");
        }
        if (!(d->p_fail >= 0.0 && d->p_fail < 1.0) || !(d->dt > 0.0f)) {
            delete dm;
            return fail(ctx, HDX_E_INVALID, "p_fail must be in [0, 1) and dt > 0");
        }
        h->n_actions = 3;
        h->n_peds = d->n_peds;
        h->n_goals = d->n_goals;
        h->n_levels = d->n_levels;
        for (int g = 0; g < d->n_goals; ++g) {
            h->goal_x[g] = d->goal_x[g];
            h->goal_y[g] = d->goal_y[g];
        }
        h->path_len = d->path_len;
        h->dt = d->dt;
        h->step_len = d->ped_speed * d->dt;
        h->half_sigma = 0.5f * d->sigma_h;
        h->coll_r2 = d->coll_radius * d->coll_radius;
        h->reach = (0.5f * (float)(d->n_levels - 1)) * d->dt;
        if (!(h->reach > 0.0f)) {
            delete dm;
            return fail(ctx, HDX_E_INVALID, "need at least two speed levels");
        }
        h->ih_scale = (float)(sqrt(3.0) / 16777216.0);
        h->r_collision = d->r_collision;
        h->r_step = d->r_step;
        h->r_goal = d->r_goal;
        h->fail_thr = prob_threshold(d->p_fail);
    } else {
        delete dm;
        return fail(ctx, HDX_E_UNSUPPORTED, "unknown model kind");
    }
    if (d->n_actions != h->n_actions) {
        delete dm;
        return fail(ctx, HDX_E_INVALID, "n_actions does not match the model");
    }
    for (int j = 0; j < kHorizon; ++j) dm->gpow[j] = (float)pow(d->gamma, j);
    hipSetDevice(ctx->device);
    hdx_model *m = new hdx_model();
    m->desc = *d;
    hipError_t e = hipMalloc(&m->d_model, sizeof(DevModel));
    if (e == hipSuccess) e = hipMemcpy(m->d_model, dm, sizeof(DevModel), hipMemcpyHostToDevice);
    delete dm;
    if (e != hipSuccess) {
        if (m->d_model) hipFree(m->d_model);
        delete m;
        return hip_fail(ctx, e, "model upload");
    }
    *out = m;
    return HDX_OK;
}

hdx_status hdx_free_model(hdx_ctx *ctx, hdx_model *m) {
    if (!ctx || !m) return HDX_E_INVALID;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    hipFree(m->d_model);
    delete m;
    return HDX_OK;
}

int32_t hdx_model_actions(const hdx_model *m) { return m ? m->desc.n_actions : -1; }

}  // extern "C"

const hdx_model_desc *hdx_internal_desc(const hdx_model *m) { return &m->desc; }

const hdx::DevModel *hdx_internal_devmodel(const hdx_model *m) { return m->d_model; }

void hdx_internal_set_error(hdx_ctx *ctx, const char *msg) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->err = msg;
}

// Wait for every staged call of the context and forget the streams its
// events were recorded on (call before destroying those streams).
void hdx_internal_quiesce(hdx_ctx *ctx) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (auto &s : ctx->slots) {
        if (s.used) hipEventSynchronize(s.done);
        s.used = false;
    }
    for (auto &a : ctx->arg_slots) {
        if (a.used) hipEventSynchronize(a.done);
        a.used = false;
    }
}

extern "C" {

int32_t hdx_model_max_children(const hdx_model *m, int32_t n) {
    if (!m || n < 0) return -1;
    if (m->desc.kind == HDX_ROCKSAMPLE) return n < 3 ? n : 3;  // none, good, bad
    if (m->desc.kind == HDX_MARS) return n < 9 ? n : 9;        // one reading per robot
    if (m->desc.kind == HDX_NAV) return n < 257 ? n : 257;     // eight reading bits, or terminal
    return n;                                                  // hashed observations
}

size_t hdx_expand_out_bytes(const hdx_model *m, int32_t K, int32_t n_leaves) {
    if (!m || K < 0 || n_leaves < 0) return 0;
    const hdx_model_desc &d = m->desc;
    const size_t A = (size_t)d.n_actions, n = (size_t)K;
    const size_t cap = (size_t)std::max(hdx_model_max_children(m, K), 1);
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t states;
    if (d.kind == HDX_ROCKSAMPLE) states = r(4 * n);
    else if (d.kind == HDX_MARS) states = r(8 * n);
    else if (d.kind == HDX_NAV) states = r(20 * n);
    else states = 2 * r(4 * n) + 2 * r(4 * (size_t)d.n_peds * n) + r((size_t)d.n_peds * n);
    const size_t per_leaf = states + r(4 * n) + r(2 * A * n) + r(4 * A) + r(8 * A * cap) + 4 * r(4 * A * cap) +
                            r(4 * A) + r(16 * A);
    return per_leaf * (size_t)n_leaves;
}

static StatesPtr to_ptr(const hdx_states &s) {
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

static bool states_ok(const hdx_model *m, const hdx_states &s, int64_t n) {
    if (m->desc.kind == HDX_ROCKSAMPLE) return s.w != nullptr;
    if (m->desc.kind == HDX_MARS || m->desc.kind == HDX_NAV) return s.w != nullptr && s.stride >= n;
    if (!s.s || !s.car) return false;
    if (m->desc.n_peds > 0 && (!s.px || !s.py || !s.goal || s.stride < n)) return false;
    return true;
}

hdx_status hdx_sample_scenarios(hdx_ctx *ctx, const hdx_model *m, const hdx_belief *b, int32_t K, uint32_t seed,
                                uint32_t step, hdx_states out, hdx_stream stream) {
    if (!ctx || !m || !b) return fail(ctx, HDX_E_INVALID, "null argument");
    if (K <= 0 || K > (1 << 24)) return fail(ctx, HDX_E_SHAPE, "K must be in 1..2^24");
    if (!states_ok(m, out, K)) return fail(ctx, HDX_E_INVALID, "missing output state arrays");
    SampleArgs A;
    memset(&A, 0, sizeof(A));
    A.model = m->d_model;
    A.k0 = seed;
    A.k1 = step;
    A.K = K;
    A.out = to_ptr(out);
    const hdx_model_desc &d = m->desc;
    if (d.kind == HDX_ROCKSAMPLE) {
        if (b->x < 0 || b->x >= d.grid || b->y < 0 || b->y >= d.grid) return fail(ctx, HDX_E_INVALID, "robot cell");
        if (d.n_rocks > 0 && !b->p_good) return fail(ctx, HDX_E_INVALID, "p_good is null");
        A.x0 = b->x;
        A.y0 = b->y;
        for (int i = 0; i < d.n_rocks; ++i) A.rock_thr[i] = prob_threshold(b->p_good[i]);
    } else if (d.kind == HDX_MARS) {
        if (b->x < 0 || b->x >= d.grid || b->y < 0 || b->y >= d.grid || b->x2 < 0 || b->x2 >= d.grid ||
            b->y2 < 0 || b->y2 >= d.grid || b->gone < 0 || b->gone > 3)
            return fail(ctx, HDX_E_INVALID, "robot cells");
        if (d.n_rocks > 0 && !b->p_good) return fail(ctx, HDX_E_INVALID, "p_good is null");
        A.x0 = b->x | (b->y << 5) | (b->x2 << 10) | (b->y2 << 15) | (b->gone << 20) | (b->gone == 3 ? 1 << 30 : 0);
        for (int i = 0; i < d.n_rocks; ++i) A.rock_thr[i] = prob_threshold(b->p_good[i]);
    } else if (d.kind == HDX_NAV) {
        int nu = 0;
        for (int c = 0; c < d.grid * d.grid; ++c)
            if (d.nav_cell[c] >= 0) ++nu;
        if (nu > 2 && !b->p_good) return fail(ctx, HDX_E_INVALID, "p_good is null");
        A.n_unknown = nu;
        for (int i = 2; i < nu; ++i) A.cell_thr[i] = prob_threshold(b->p_good[i]);
    } else {
        if (d.n_peds > 0 && (!b->px || !b->py || !b->goal_p)) return fail(ctx, HDX_E_INVALID, "belief arrays");
        if (b->level < 0 || b->level >= d.n_levels) return fail(ctx, HDX_E_INVALID, "speed level");
        A.s0 = b->s;
        A.level0 = b->level;
        for (int j = 0; j < d.n_peds; ++j) {
            A.px0[j] = b->px[j];
            A.py0[j] = b->py[j];
            double cum = 0.0;
            for (int q = 0; q < d.n_goals; ++q) {
                cum += b->goal_p[j * d.n_goals + q];
                A.goal_thr[j][q] = prob_threshold(cum);
            }
        }
    }
    hipSetDevice(ctx->device);
    // the arguments go through a device slot (they are too large to travel
    // comfortably in the kernel-argument segment); the slot is reused once
    // the kernel that read it has run
    std::lock_guard<std::mutex> lock(ctx->mu);
    ArgSlot &slot = ctx->arg_slots[ctx->next_arg_slot];
    ctx->next_arg_slot = (ctx->next_arg_slot + 1) % kArgSlots;
    hipError_t e = hipSuccess;
    if (slot.used && (e = hipEventSynchronize(slot.done)) != hipSuccess) return hip_fail(ctx, e, "argument slot wait");
    memcpy(slot.h, &A, sizeof(A));
    e = hipMemcpyAsync(slot.d, slot.h, sizeof(A), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = launch_sample((const SampleArgs *)slot.d, K, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(slot.done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "sample_scenarios launch");
    slot.used = true;
    return HDX_OK;
}

static int64_t horizon_of(const hdx_rollout_cfg &c, int64_t d0) {
    int64_t h = c.max_steps;
    if (c.max_depth >= 0 && c.max_depth - d0 < h) h = c.max_depth - d0;
    return h;
}

static hdx_status check_cfg(hdx_ctx *ctx, const hdx_model *m, const hdx_rollout_cfg &c) {
    if (c.policy < HDX_POLICY_DEFAULT || c.policy > HDX_POLICY_RANDOM) return fail(ctx, HDX_E_INVALID, "policy");
    if (c.policy == HDX_POLICY_CONST && (c.const_action < 0 || c.const_action >= m->desc.n_actions))
        return fail(ctx, HDX_E_INVALID, "const_action");
    if (c.max_steps < 0) return fail(ctx, HDX_E_INVALID, "max_steps < 0");
    return HDX_OK;
}

}  // extern "C"

namespace {

struct Shape {
    int64_t n_tiles = 0;
    int32_t n_max = 1, has_rs = 0, has_ped = 0, ped_max = 0, has_mars = 0, has_nav = 0;
};

hdx_status validate_leaves(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, Shape *sh) {
    if (!leaves && n_leaves > 0) return fail(ctx, HDX_E_INVALID, "null leaves");
    if (n_leaves < 0) return fail(ctx, HDX_E_INVALID, "negative leaf count");
    Shape s;
    for (int32_t i = 0; i < n_leaves; ++i) {
        const hdx_leaf &L = leaves[i];
        if (!L.model) return fail(ctx, HDX_E_INVALID, "leaf without model");
        const hdx_model_desc &d = L.model->desc;
        const int A = d.n_actions;
        if (L.n < 0 || L.n > (d.kind == HDX_NAV ? kMaxNavLeaf : kMaxLeaf))
            return fail(ctx, HDX_E_SHAPE, "leaf scenario count out of range");
        if (L.depth < 0 || L.last_action < -1 || L.last_action >= A || (L.last_action >= 0 && L.depth < 1))
            return fail(ctx, HDX_E_INVALID, "depth / last_action");
        if (L.cap < hdx_model_max_children(L.model, L.n)) return fail(ctx, HDX_E_CAPACITY, "cap too small");
        hdx_status st = check_cfg(ctx, L.model, L.rollout);
        if (st != HDX_OK) return st;
        if (horizon_of(L.rollout, (int64_t)L.depth + 1) > kHorizon)
            return fail(ctx, HDX_E_SHAPE, "rollout horizon exceeds HDX_MAX_HORIZON");
        if (!L.n_children || !L.r_mean || !L.steps) return fail(ctx, HDX_E_INVALID, "missing output arrays");
        if (L.n > 0) {
            if (!L.parent_ids || !L.idx || !L.ids_out || !L.perm || !L.child_z || !L.child_n || !L.child_off ||
                !L.child_u0 || !L.child_l0)
                return fail(ctx, HDX_E_INVALID, "missing leaf arrays");
            if (!states_ok(L.model, L.parent, 0) || !states_ok(L.model, L.states_out, L.n))
                return fail(ctx, HDX_E_INVALID, "missing state arrays");
            if ((L.sprime.w || L.sprime.s) && !states_ok(L.model, L.sprime, (int64_t)A * L.n))
                return fail(ctx, HDX_E_INVALID, "incomplete sprime arrays");
        }
        s.n_tiles += A;
        if (L.n > s.n_max) s.n_max = L.n;
        if (d.kind == HDX_PEDNAV) {
            s.has_ped = 1;
            if (d.n_peds > s.ped_max) s.ped_max = d.n_peds;
        } else if (d.kind == HDX_MARS) {
            s.has_mars = 1;
        } else if (d.kind == HDX_NAV) {
            s.has_nav = 1;
        } else {
            s.has_rs = 1;
        }
    }
    if (s.n_tiles > (1ll << 30)) return fail(ctx, HDX_E_SHAPE, "too many tiles");
    *sh = s;
    return HDX_OK;
}

void pack_leaves(const hdx_leaf *leaves, int32_t n_leaves, LeafTask *tasks, Tile *tiles) {
    int64_t t = 0;
    for (int32_t i = 0; i < n_leaves; ++i) {
        const hdx_leaf &L = leaves[i];
        LeafTask &T = tasks[i];
        memset(&T, 0, sizeof(T));
        T.model = L.model->d_model;
        T.kind = L.model->desc.kind;
        T.n_actions = L.model->desc.n_actions;
        T.k0 = L.seed;
        T.k1 = L.step;
        T.policy = L.rollout.policy;
        T.const_action = L.rollout.const_action;
        T.max_steps = L.rollout.max_steps;
        T.max_depth = L.rollout.max_depth;
        T.parent = to_ptr(L.parent);
        T.parent_ids = L.parent_ids;
        T.idx = L.idx;
        T.n = L.n;
        T.depth = L.depth;
        T.last_action = L.last_action;
        T.cap = L.cap;
        T.out = to_ptr(L.states_out);
        T.ids_out = L.ids_out;
        T.perm = L.perm;
        T.n_children = L.n_children;
        T.child_z = L.child_z;
        T.child_n = L.child_n;
        T.child_off = L.child_off;
        T.child_u0 = L.child_u0;
        T.child_l0 = L.child_l0;
        T.r_mean = L.r_mean;
        T.steps = L.steps;
        T.sprime = to_ptr(L.sprime);
        T.r = L.r;
        T.z = L.z;
        T.U = L.U;
        T.L = L.L;
        T.child_of = L.child_of;
        if (tiles)
            for (int a = 0; a < T.n_actions; ++a) tiles[t++] = Tile{i, a};
    }
}

}  // namespace

void hdx::plan_classes(const LeafTask *tasks, const int8_t *variant, Tile *tiles, int64_t n_tiles,
                       ClassPlan *plan, bool split) {
    int32_t vmax[kModelVariants] = {0};
    if (!split)
        for (int64_t t = 0; t < n_tiles; ++t)
            vmax[variant[tiles[t].leaf]] = std::max(vmax[variant[tiles[t].leaf]], tasks[tiles[t].leaf].n);
    auto group = [&](const Tile &t) {
        const int v = variant[t.leaf];
        return v * kSizeClasses + size_class(split ? tasks[t.leaf].n : vmax[v]);
    };
    int64_t cnt[kGroups] = {0};
    for (int g = 0; g < kGroups; ++g) plan->n_max[g] = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int g = group(tiles[t]);
        cnt[g]++;
        plan->n_max[g] = std::max(plan->n_max[g], tasks[tiles[t].leaf].n);
    }
    int64_t at = 0;
    for (int g = 0; g < kGroups; ++g) {
        plan->begin[g] = at;
        plan->count[g] = cnt[g];
        at += cnt[g];
    }
    std::stable_sort(tiles, tiles + n_tiles, [&](const Tile &x, const Tile &y) {
        const int gx = group(x), gy = group(y);
        if (gx != gy) return gx < gy;
        return tasks[x.leaf].n > tasks[y.leaf].n;
    });
    // Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD
    // b mod 8), each XCD with its own L2.  Inside a group, deal the leaves
    // (largest first) to the XCDs in turn and interleave the XCDs' tile
    // lists, so every tile of a leaf runs where its parent data is cached
    // while each XCD still sees the sizes largest first.
    std::vector<Tile> lists[kXcds];
    for (int g = 0; g < kGroups; ++g) {
        Tile *t = tiles + plan->begin[g];
        const int64_t count = plan->count[g];
        if (count < 2 * kXcds) continue;
        for (auto &l : lists) l.clear();
        int32_t prev = -1;
        int64_t rank = -1;
        for (int64_t i = 0; i < count; ++i) {
            if (t[i].leaf != prev) {
                prev = t[i].leaf;
                ++rank;
            }
            lists[rank % kXcds].push_back(t[i]);
        }
        size_t pos[kXcds] = {};
        int64_t o = 0;
        while (o < count)
            for (int x = 0; x < kXcds; ++x)
                if (pos[x] < lists[x].size()) t[o++] = lists[x][pos[x]++];
    }
}

Schedule hdx::class_default_schedule(int32_t n_max, int32_t max_threads, int32_t mode) {
    Schedule s;
    s.threads = std::min(std::max(64, pow2_at_least(std::max(n_max, 1)) / 2), std::min(mode == 4 ? 1024 : 256, max_threads));
    s.persistent = 0;
    s.xcd_remap = mode < 0 ? 1 : 0;
    if (mode == 0 || mode == 3) s.threads = 64;
    // latency form: one scenario per lane where the model's width allows
    if (mode == -2) s.threads = std::min(std::max(64, pow2_at_least(std::max(n_max, 1))), max_threads);
    return s;
}

hipError_t hdx::launch_classes(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queues,
                               const ClassPlan &plan, const int32_t *lds_n, const Schedule *sch, int32_t n_cu,
                               hipStream_t stream, uint64_t mask) {
    for (int g = 0; g < kGroups; ++g) {
        if (plan.count[g] == 0 || !(mask & (1ull << g))) continue;
        Variant vg = group_variant(g);
        vg.n_max = std::max(lds_n[g], plan.n_max[g]);
        // driving leaves small enough for every scenario's pedestrians to
        // get lanes of their own (n times the pedestrian bound fits a
        // wavefront): the element-level instance
        vg.group = vg.mode == 1 && plan.n_max[g] * vg.pm <= 64 ? 1 : 0;
        // a workgroup no wider than the group's leaves need
        const int need = std::min(variant_max_threads(vg), std::max(64, pow2_at_least(std::max(vg.n_max, 1))));
        Schedule sc = sch[g];
        if (sc.threads > need) sc.threads = need;
        const hipError_t e = launch_expand(d_tasks, d_tiles + plan.begin[g], d_queues + g, (int32_t)plan.count[g], vg,
                                           sc, n_cu, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {

// Each non-empty group of `mask` on a stream of its own, forked from `st`
// and joined back into it (inside a stream capture this becomes parallel
// graph branches), so one group's slow tail overlaps the others; a single
// group launches on `st` directly.
hipError_t launch_classes_forked(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queues,
                                 const ClassPlan &plan, const int32_t *lds_n, const Schedule *sch, int32_t n_cu,
                                 hipStream_t st, const hipStream_t *cls, hipEvent_t fork, const hipEvent_t *join,
                                 uint64_t mask = ~0ull) {
    int active = 0;
    for (int g = 0; g < kGroups; ++g)
        if (plan.count[g] > 0 && (mask & (1ull << g))) ++active;
    if (active <= 1) return launch_classes(d_tasks, d_tiles, d_queues, plan, lds_n, sch, n_cu, st, mask);
    hipError_t e = hipEventRecord(fork, st);
    // largest leaves first: their tails are the longest
    for (int c = kSizeClasses - 1; c >= 0 && e == hipSuccess; --c)
        for (int v = kModelVariants - 1; v >= 0 && e == hipSuccess; --v) {
            const int g = v * kSizeClasses + c;
            if (plan.count[g] == 0 || !(mask & (1ull << g))) continue;
            e = hipStreamWaitEvent(cls[g], fork, 0);
            if (e == hipSuccess) e = launch_classes(d_tasks, d_tiles, d_queues, plan, lds_n, sch, n_cu, cls[g], 1ull << g);
            if (e == hipSuccess) e = hipEventRecord(join[g], cls[g]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, join[g], 0);
        }
    return e;
}

// Model variant of each leaf (its launch-group row).
void leaf_variants(const hdx_leaf *leaves, int32_t n_leaves, int8_t *out) {
    for (int32_t i = 0; i < n_leaves; ++i) {
        const hdx_model_desc &d = *hdx_internal_desc(leaves[i].model);
        out[i] = (int8_t)model_variant(d.kind, d.n_peds);
    }
}

hdx_status grow_pinned(hdx_ctx *ctx, LeafTask **h_tasks, LeafTask **d_tasks, int64_t *cap_tasks, Tile **h_tiles,
                       Tile **d_tiles, int64_t *cap_tiles, int64_t need_tasks, int64_t need_tiles) {
    if (*cap_tasks >= need_tasks && *cap_tiles >= need_tiles) return HDX_OK;
    int64_t ct = *cap_tasks, cl = *cap_tiles;
    while (ct < need_tasks) ct = ct ? 2 * ct : 64;
    while (cl < need_tiles) cl = cl ? 2 * cl : 1024;
    if (*h_tasks) hipHostFree(*h_tasks);
    if (*h_tiles) hipHostFree(*h_tiles);
    if (*d_tasks) hipFree(*d_tasks);
    if (*d_tiles) hipFree(*d_tiles);
    *h_tasks = *d_tasks = nullptr;
    *h_tiles = *d_tiles = nullptr;
    *cap_tasks = *cap_tiles = 0;
    if (hipHostMalloc((void **)h_tasks, ct * sizeof(LeafTask)) != hipSuccess ||
        hipHostMalloc((void **)h_tiles, cl * sizeof(Tile)) != hipSuccess ||
        hipMalloc((void **)d_tasks, ct * sizeof(LeafTask)) != hipSuccess ||
        hipMalloc((void **)d_tiles, cl * sizeof(Tile)) != hipSuccess)
        return fail(ctx, HDX_E_NOMEM, "descriptor staging allocation");
    *cap_tasks = ct;
    *cap_tiles = cl;
    return HDX_OK;
}

}  // namespace

namespace {

// Small calls of one kernel carry their descriptors in the kernel arguments
// (the multi-agent and navigation models have kernels of their own;
// RockSample and driving share one).  Returns false if the call is not such
// a call; otherwise launches and sets *st.
bool launch_in_args(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, const Shape &sh, hipStream_t stream,
                    hdx_status *st) {
    const int kernels = (sh.has_rs || sh.has_ped ? 1 : 0) + sh.has_mars + sh.has_nav;
    if (n_leaves > kArgLeaves || kernels > 1) return false;
    const Variant v0 = pick_variant(sh.has_rs, sh.has_ped, sh.ped_max, sh.n_max, sh.has_mars, sh.has_nav);
    static_assert(sizeof(ArgPack) <= 4096, "kernel argument pack too large");
    ArgPack pack;
    memset(&pack, 0, sizeof(pack));
    pack_leaves(leaves, n_leaves, pack.t, nullptr);
    pack.tile_begin[0] = 0;
    for (int32_t i = 0; i < n_leaves; ++i) pack.tile_begin[i + 1] = pack.tile_begin[i] + pack.t[i].n_actions;
    pack.n_leaves = n_leaves;
    pack.n_max = v0.n_max;
    const Schedule sch =
        ctx->sched_fixed ? ctx->sched : class_default_schedule(v0.n_max, variant_max_threads(v0), -2);
    pack.xcd_remap = sch.xcd_remap;
    const hipError_t e = launch_expand_args(pack, v0, sch, stream);
    *st = e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "expand launch");
    return true;
}

// Copy a planned call's descriptors, tiles and queue heads from host staging
// to their device buffers on `hs`, launch its groups, and record `done`
// after the launch (the host staging may be rewritten once it has fired).
hdx_status launch_staged(hdx_ctx *ctx, const LeafTask *h_tasks, const Tile *h_tiles, TileQueue *h_queue,
                         LeafTask *d_tasks, Tile *d_tiles, TileQueue *d_queue, int32_t n_leaves, int64_t n_tiles,
                         const ClassPlan &plan, hipStream_t hs, hipEvent_t fork, const hipEvent_t *join,
                         hipEvent_t done) {
    for (int g = 0; g < kGroups; ++g) h_queue[g] = TileQueue{0, 0, (int32_t)plan.count[g], 0};
    hipError_t e = hipMemcpyAsync(d_tasks, h_tasks, n_leaves * sizeof(LeafTask), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tiles, h_tiles, n_tiles * sizeof(Tile), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(d_queue, h_queue, kGroups * sizeof(TileQueue), hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(ctx, e, "descriptor copy");
    int32_t no_lds[kGroups] = {};
    Schedule sch[kGroups];
    // a launch far smaller than the GPU (a search's leaf batch) is latency
    // bound: wider workgroups finish each tile sooner
    const bool few = n_tiles < 8 * (int64_t)ctx->n_cu;
    for (int g = 0; g < kGroups; ++g) {
        sch[g] = ctx->sched_fixed ? ctx->sched
                                  : class_default_schedule(plan.n_max[g], variant_max_threads(group_variant(g)),
                                                           few ? -2 : group_variant(g).mode);
        if (few) sch[g].xcd_remap = 0;
    }
    e = launch_classes_forked(d_tasks, d_tiles, d_queue, plan, no_lds, sch, ctx->n_cu, hs, ctx->cls_stream, fork,
                              join);
    if (e != hipSuccess) return hip_fail(ctx, e, "expand launch");
    e = hipEventRecord(done, hs);
    return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "event record");
}

// The unsplit plan of plan_classes (one group per model variant, filed
// under its largest leaf's size class; largest leaf first, a leaf's tiles in
// action order; leaves dealt to the XCDs in turn and their tile lists
// interleaved), built from the leaf descriptors with fixed arrays only:
// order[] holds n_leaves leaf indices, tiles[] receives every tile.
void plan_fixed(const LeafTask *tasks, const int8_t *variant, int32_t n_leaves, Tile *tiles, int32_t *order,
                ClassPlan *plan) {
    int32_t vmax[kModelVariants] = {0};
    for (int32_t i = 0; i < n_leaves; ++i) vmax[variant[i]] = std::max(vmax[variant[i]], tasks[i].n);
    auto group = [&](int32_t i) { return variant[i] * kSizeClasses + size_class(vmax[variant[i]]); };
    for (int g = 0; g < kGroups; ++g) {
        plan->count[g] = 0;
        plan->n_max[g] = 0;
    }
    for (int32_t i = 0; i < n_leaves; ++i) {
        plan->count[group(i)] += tasks[i].n_actions;
        plan->n_max[group(i)] = std::max(plan->n_max[group(i)], tasks[i].n);
    }
    int64_t at = 0;
    for (int g = 0; g < kGroups; ++g) {
        plan->begin[g] = at;
        at += plan->count[g];
    }
    // leaves by (group, size descending, index): insertion sort
    auto before = [&](int32_t x, int32_t y) {
        const int gx = group(x), gy = group(y);
        if (gx != gy) return gx < gy;
        if (tasks[x].n != tasks[y].n) return tasks[x].n > tasks[y].n;
        return x < y;
    };
    for (int32_t i = 0; i < n_leaves; ++i) {
        int32_t j = i;
        while (j > 0 && before(i, order[j - 1])) {
            order[j] = order[j - 1];
            --j;
        }
        order[j] = i;
    }
    int32_t lo = 0;
    for (int g = 0; g < kGroups; ++g) {
        int32_t hi = lo;
        while (hi < n_leaves && group(order[hi]) == g) ++hi;
        Tile *t = tiles + plan->begin[g];
        const int64_t count = plan->count[g];
        int64_t o = 0;
        if (count < 2 * kXcds) {
            for (int32_t r = lo; r < hi; ++r)
                for (int a = 0; a < tasks[order[r]].n_actions; ++a) t[o++] = Tile{order[r], a};
        } else {
            // XCD x takes the leaves of rank x, x + 8, ...; one tile from
            // each XCD's list in turn
            int32_t rank[kXcds], act[kXcds];
            for (int x = 0; x < kXcds; ++x) {
                rank[x] = x;
                act[x] = 0;
            }
            const int32_t nl = hi - lo;
            while (o < count)
                for (int x = 0; x < kXcds; ++x) {
                    if (rank[x] >= nl) continue;
                    const int32_t leaf = order[lo + rank[x]];
                    t[o++] = Tile{leaf, act[x]};
                    if (++act[x] == tasks[leaf].n_actions) {
                        act[x] = 0;
                        rank[x] += kXcds;
                    }
                }
        }
        lo = hi;
    }
}

}  // namespace

extern "C" {

hdx_status hdx_expand_leaf(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, hdx_stream stream) {
    if (!ctx) return HDX_E_INVALID;
    Shape sh;
    hdx_status st = validate_leaves(ctx, leaves, n_leaves, &sh);
    if (st != HDX_OK || n_leaves == 0) return st;
    hipSetDevice(ctx->device);
    if (launch_in_args(ctx, leaves, n_leaves, sh, (hipStream_t)stream, &st)) return st;
    std::lock_guard<std::mutex> lock(ctx->mu);
    Slot &s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kSlots;
    if (s.used) {
        hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
    }
    st = grow_pinned(ctx, &s.h_tasks, &s.d_tasks, &s.cap_tasks, &s.h_tiles, &s.d_tiles, &s.cap_tiles, n_leaves,
                     sh.n_tiles);
    if (st != HDX_OK) return st;
    pack_leaves(leaves, n_leaves, s.h_tasks, s.h_tiles);
    std::vector<int8_t> var(n_leaves);
    leaf_variants(leaves, n_leaves, var.data());
    ClassPlan plan;
    plan_classes(s.h_tasks, var.data(), s.h_tiles, sh.n_tiles, &plan, false);
    st = launch_staged(ctx, s.h_tasks, s.h_tiles, s.h_queue, s.d_tasks, s.d_tiles, s.d_queue, n_leaves, sh.n_tiles,
                       plan, (hipStream_t)stream, s.fork, s.join, s.done);
    if (st == HDX_OK) s.used = true;
    return st;
}

hdx_status hdx_expand_leaf_noalloc(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, hdx_stream stream) {
    if (!ctx) return HDX_E_INVALID;
    Shape sh;
    hdx_status st = validate_leaves(ctx, leaves, n_leaves, &sh);
    if (st != HDX_OK || n_leaves == 0) return st;
    if (n_leaves > HDX_NOALLOC_MAX_LEAVES) return fail(ctx, HDX_E_CAPACITY, "more than HDX_NOALLOC_MAX_LEAVES leaves");
    if (sh.n_tiles > HDX_NOALLOC_MAX_TILES)
        return fail(ctx, HDX_E_CAPACITY, "more than HDX_NOALLOC_MAX_TILES (leaf, action) tiles");
    if (!ctx->na_scratch) return fail(ctx, HDX_E_DEVICE, "no-allocation scratch not set up");
    hipSetDevice(ctx->device);
    if (launch_in_args(ctx, leaves, n_leaves, sh, (hipStream_t)stream, &st)) return st;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (ctx->na_used) {
        // the previous call's copies must have left the host staging
        const hipError_t e = hipEventSynchronize(ctx->na_done);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
    }
    pack_leaves(leaves, n_leaves, ctx->na_h_tasks, nullptr);
    leaf_variants(leaves, n_leaves, ctx->na_var);
    ClassPlan plan;
    plan_fixed(ctx->na_h_tasks, ctx->na_var, n_leaves, ctx->na_h_tiles, ctx->na_order, &plan);
    LeafTask *d_tasks = (LeafTask *)(ctx->na_scratch + kNaTasksOff);
    Tile *d_tiles = (Tile *)(ctx->na_scratch + kNaTilesOff);
    TileQueue *d_queue = (TileQueue *)(ctx->na_scratch + kNaQueueOff);
    st = launch_staged(ctx, ctx->na_h_tasks, ctx->na_h_tiles, ctx->na_h_queue, d_tasks, d_tiles, d_queue, n_leaves,
                       sh.n_tiles, plan, (hipStream_t)stream, ctx->na_fork, ctx->na_join, ctx->na_done);
    if (st == HDX_OK) ctx->na_used = true;
    return st;
}

}  // extern "C"

struct hdx_batch {
    LeafTask *h_tasks = nullptr, *d_tasks = nullptr;
    Tile *h_tiles = nullptr, *d_tiles = nullptr;
    TileQueue *h_queue = nullptr, *d_queue = nullptr;
    int64_t cap_tasks = 0, cap_tiles = 0;
    int64_t max_leaves = 0, max_tiles = 0;  // capacity the caller asked for
    int32_t n_leaves = 0;
    int64_t n_tiles = 0;
    ClassPlan plan{};
    int32_t lds_c[kGroups] = {};  // per launch group: largest leaf seen
    ClassPlan g_plan{};
    int32_t g_lds[kGroups] = {};
    Schedule sched[kGroups];  // per launch group
    bool sched_set[kGroups] = {};
    hipStream_t work = nullptr;      // capture and tuning stream
    hipStream_t cls[kGroups] = {};  // launch groups side by side
    hipEvent_t fork = nullptr, join[kGroups] = {};
    hipEvent_t staged = nullptr, t0 = nullptr, t1 = nullptr;
    bool staged_used = false;
    bool graph_on = false, graph_ok = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Schedule g_sched[kGroups];
    int64_t g_tiles = 0;
    bool split = false;         // one launch group per (model variant, size class)
    std::vector<int8_t> var;    // model variant of each staged leaf
};

namespace {

hipError_t batch_direct_launch(hdx_ctx *ctx, hdx_batch *b, const Schedule *s, hipStream_t st,
                               uint64_t mask = ~0ull) {
    return launch_classes_forked(b->d_tasks, b->d_tiles, b->d_queue, b->plan, b->lds_c, s, ctx->n_cu, st, b->cls,
                                 b->fork, b->join, mask);
}

// Widest workgroup group g can use: its model's cap and its leaves' need.
int32_t group_width_cap(const hdx_batch *b, int g) {
    const int32_t n_max = std::max(b->lds_c[g], b->plan.n_max[g]);
    return std::min(variant_max_threads(group_variant(g)), std::max(64, pow2_at_least(std::max(n_max, 1))));
}

bool same_schedule(const Schedule &a, const Schedule &b) {
    return a.threads == b.threads && a.persistent == b.persistent && a.xcd_remap == b.xcd_remap;
}

// Default schedule of every group that has none set.
void default_schedules(hdx_batch *b) {
    for (int g = 0; g < kGroups; ++g)
        if (!b->sched_set[g])
            b->sched[g] = class_default_schedule(std::max(b->lds_c[g], 1), variant_max_threads(group_variant(g)),
                                                 group_variant(g).mode);
}

// Plan the staged tiles (split or merged groups) and copy tiles and queues
// to the device on `st`.
hipError_t replan(hdx_batch *b, hipStream_t st) {
    plan_classes(b->h_tasks, b->var.data(), b->h_tiles, b->n_tiles, &b->plan, b->split);
    for (int g = 0; g < kGroups; ++g) {
        b->h_queue[g] = TileQueue{0, 0, (int32_t)b->plan.count[g], 0};
        b->lds_c[g] = std::max(b->lds_c[g], b->plan.n_max[g]);
    }
    hipError_t e = hipSuccess;
    if (b->n_tiles > 0) e = hipMemcpyAsync(b->d_tiles, b->h_tiles, b->n_tiles * sizeof(Tile), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_queue, b->h_queue, kGroups * sizeof(TileQueue), hipMemcpyHostToDevice, st);
    return e;
}

void drop_graph(hdx_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ok = false;
}

}  // namespace

extern "C" {

hdx_status hdx_batch_create(hdx_ctx *ctx, int32_t max_leaves, int64_t max_tiles, hdx_batch **out) {
    if (!ctx || !out || max_leaves < 1 || max_tiles < 1) return fail(ctx, HDX_E_INVALID, "bad argument");
    hipSetDevice(ctx->device);
    hdx_batch *b = new hdx_batch();
    b->max_leaves = max_leaves;
    b->max_tiles = max_tiles;
    hdx_status st = grow_pinned(ctx, &b->h_tasks, &b->d_tasks, &b->cap_tasks, &b->h_tiles, &b->d_tiles, &b->cap_tiles,
                                max_leaves, max_tiles);
    if (st == HDX_OK &&
        (hipHostMalloc(&b->h_queue, kGroups * sizeof(TileQueue)) != hipSuccess ||
         hipMalloc(&b->d_queue, kGroups * sizeof(TileQueue)) != hipSuccess ||
         hipMemset(b->d_queue, 0, kGroups * sizeof(TileQueue)) != hipSuccess ||
         hipStreamCreateWithFlags(&b->work, hipStreamNonBlocking) != hipSuccess || !create_events(&b->fork, b->join) ||
         hipEventCreate(&b->staged) != hipSuccess || hipEventCreate(&b->t0) != hipSuccess ||
         hipEventCreate(&b->t1) != hipSuccess))
        st = fail(ctx, HDX_E_NOMEM, "batch allocation");
    for (int c = 0; c < kGroups && st == HDX_OK; ++c)
        if (hipStreamCreateWithFlags(&b->cls[c], hipStreamNonBlocking) != hipSuccess)
            st = fail(ctx, HDX_E_NOMEM, "batch streams");
    if (st == HDX_OK && hipDeviceSynchronize() != hipSuccess) st = fail(ctx, HDX_E_DEVICE, "batch allocation");
    if (st != HDX_OK) {
        hdx_batch_destroy(ctx, b);
        return st;
    }
    *out = b;
    return HDX_OK;
}

hdx_status hdx_batch_destroy(hdx_ctx *ctx, hdx_batch *b) {
    if (!ctx || !b) return HDX_E_INVALID;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    drop_graph(b);
    if (b->h_tasks) hipHostFree(b->h_tasks);
    if (b->h_tiles) hipHostFree(b->h_tiles);
    if (b->h_queue) hipHostFree(b->h_queue);
    if (b->d_tasks) hipFree(b->d_tasks);
    if (b->d_tiles) hipFree(b->d_tiles);
    if (b->d_queue) hipFree(b->d_queue);
    if (b->work) hipStreamDestroy(b->work);
    for (int c = 0; c < kGroups; ++c)
        if (b->cls[c]) hipStreamDestroy(b->cls[c]);
    destroy_events(&b->fork, b->join);
    if (b->staged) hipEventDestroy(b->staged);
    if (b->t0) hipEventDestroy(b->t0);
    if (b->t1) hipEventDestroy(b->t1);
    delete b;
    return HDX_OK;
}

hdx_status hdx_batch_set_leaves(hdx_ctx *ctx, hdx_batch *b, const hdx_leaf *leaves, int32_t n_leaves,
                                hdx_stream stream) {
    if (!ctx || !b) return HDX_E_INVALID;
    Shape sh;
    hdx_status st = validate_leaves(ctx, leaves, n_leaves, &sh);
    if (st != HDX_OK) return st;
    if (n_leaves > b->max_leaves || sh.n_tiles > b->max_tiles) return fail(ctx, HDX_E_CAPACITY, "batch capacity");
    hipSetDevice(ctx->device);
    if (b->staged_used) {
        hipError_t e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
    }
    pack_leaves(leaves, n_leaves, b->h_tasks, b->h_tiles);
    b->var.assign(std::max(n_leaves, 1), 0);
    leaf_variants(leaves, n_leaves, b->var.data());
    b->n_leaves = n_leaves;
    b->n_tiles = sh.n_tiles;
    // LDS sized for the largest leaf a group has seen, so graphs survive smaller batches
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (n_leaves > 0) e = hipMemcpyAsync(b->d_tasks, b->h_tasks, n_leaves * sizeof(LeafTask), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = replan(b, hs);
    if (e == hipSuccess) e = hipEventRecord(b->staged, hs);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch descriptor copy");
    b->staged_used = true;
    default_schedules(b);
    return HDX_OK;
}

hdx_status hdx_batch_set_split(hdx_ctx *ctx, hdx_batch *b, int32_t split) {
    if (!ctx || !b) return HDX_E_INVALID;
    if ((split != 0) == b->split) return HDX_OK;
    hipSetDevice(ctx->device);
    if (b->staged_used) {
        hipError_t e = hipEventSynchronize(b->staged);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
    }
    hipDeviceSynchronize();  // no launch may still read the tiles
    b->split = split != 0;
    drop_graph(b);
    hipError_t e = replan(b, b->work);
    if (e == hipSuccess) e = hipStreamSynchronize(b->work);
    if (e != hipSuccess) return hip_fail(ctx, e, "replan");
    default_schedules(b);
    return HDX_OK;
}

hdx_status hdx_batch_get_split(const hdx_batch *b, int32_t *split) {
    if (!b || !split) return HDX_E_INVALID;
    *split = b->split ? 1 : 0;
    return HDX_OK;
}

hdx_status hdx_batch_set_schedule(hdx_ctx *ctx, hdx_batch *b, int32_t threads, int32_t persistent,
                                  int32_t xcd_remap) {
    if (!ctx || !b) return HDX_E_INVALID;
    if (threads < 64 || threads > 1024 || threads % 64 != 0 || persistent < 0 || persistent > 64)
        return fail(ctx, HDX_E_INVALID, "schedule");
    for (int g = 0; g < kGroups; ++g) {
        b->sched[g] = Schedule{threads, persistent, xcd_remap ? 1 : 0};
        b->sched_set[g] = true;
    }
    return HDX_OK;
}

hdx_status hdx_batch_set_class_schedule(hdx_ctx *ctx, hdx_batch *b, int32_t cls, int32_t threads, int32_t persistent,
                                        int32_t xcd_remap) {
    if (!ctx || !b) return HDX_E_INVALID;
    if (cls < 0 || cls >= kSizeClasses || threads < 64 || threads > 1024 || threads % 64 != 0 || persistent < 0 ||
        persistent > 64)
        return fail(ctx, HDX_E_INVALID, "schedule");
    for (int v = 0; v < kModelVariants; ++v) {
        b->sched[v * kSizeClasses + cls] = Schedule{threads, persistent, xcd_remap ? 1 : 0};
        b->sched_set[v * kSizeClasses + cls] = true;
    }
    return HDX_OK;
}

hdx_status hdx_batch_get_group_schedule(const hdx_batch *b, int32_t group, int32_t *threads, int32_t *persistent,
                                        int32_t *xcd_remap, int64_t *tiles) {
    if (!b || !threads || !persistent || !xcd_remap || group < 0 || group >= kGroups) return HDX_E_INVALID;
    const Schedule &s = b->sched[group];
    const int32_t cap = group_width_cap(b, group);
    *threads = s.threads > cap ? cap : s.threads;
    *persistent = s.persistent;
    *xcd_remap = s.xcd_remap;
    if (tiles) *tiles = b->plan.count[group];
    return HDX_OK;
}

hdx_status hdx_batch_get_class_schedule(const hdx_batch *b, int32_t cls, int32_t *threads, int32_t *persistent,
                                        int32_t *xcd_remap, int64_t *tiles) {
    if (!b || !threads || !persistent || !xcd_remap || cls < 0 || cls >= kSizeClasses) return HDX_E_INVALID;
    // the class's group with the most tiles
    int best = cls;
    int64_t total = 0;
    for (int v = 0; v < kModelVariants; ++v) {
        const int g = v * kSizeClasses + cls;
        total += b->plan.count[g];
        if (b->plan.count[g] > b->plan.count[best]) best = g;
    }
    const hdx_status st = hdx_batch_get_group_schedule(b, best, threads, persistent, xcd_remap, nullptr);
    if (tiles) *tiles = total;
    return st;
}

hdx_status hdx_batch_get_schedule(const hdx_batch *b, int32_t *threads, int32_t *persistent, int32_t *xcd_remap) {
    if (!b || !threads || !persistent || !xcd_remap) return HDX_E_INVALID;
    int big = 0;
    for (int g = 1; g < kGroups; ++g)
        if (b->plan.count[g] > b->plan.count[big]) big = g;
    return hdx_batch_get_group_schedule(b, big, threads, persistent, xcd_remap, nullptr);
}

hdx_status hdx_batch_use_graph(hdx_ctx *ctx, hdx_batch *b, int32_t enable) {
    if (!ctx || !b) return HDX_E_INVALID;
    b->graph_on = enable != 0;
    return HDX_OK;
}

hdx_status hdx_batch_launch(hdx_ctx *ctx, hdx_batch *b, hdx_stream stream) {
    if (!ctx || !b) return HDX_E_INVALID;
    if (b->n_tiles == 0) return HDX_OK;
    hipSetDevice(ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    if (!b->graph_on) {
        e = batch_direct_launch(ctx, b, b->sched, hs);
        return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "batch launch");
    }
    // the graph bakes in each group's tile offset, LDS size and (non-persistent) grid
    bool groups_same = true;
    for (int g = 0; g < kGroups; ++g)
        groups_same = groups_same && b->plan.begin[g] == b->g_plan.begin[g] && b->lds_c[g] == b->g_lds[g] &&
                      same_schedule(b->sched[g], b->g_sched[g]) &&
                      (b->sched[g].persistent > 0 ? (b->plan.count[g] > 0) == (b->g_plan.count[g] > 0)
                                                  : b->plan.count[g] == b->g_plan.count[g]);
    const bool same = b->graph_ok && groups_same;
    if (!same) {
        drop_graph(b);
        e = hipStreamBeginCapture(b->work, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
        hipError_t le = batch_direct_launch(ctx, b, b->sched, b->work);
        e = hipStreamEndCapture(b->work, &b->graph);
        if (le != hipSuccess) return hip_fail(ctx, le, "captured launch");
        if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(ctx, e, "graph instantiate");
        }
        b->graph_ok = true;
        b->g_tiles = b->n_tiles;
        b->g_plan = b->plan;
        for (int g = 0; g < kGroups; ++g) {
            b->g_lds[g] = b->lds_c[g];
            b->g_sched[g] = b->sched[g];
        }
    }
    e = hipGraphLaunch(b->exec, hs);
    return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "graph launch");
}

hdx_status hdx_batch_autotune(hdx_ctx *ctx, hdx_batch *b, int32_t reps, float *best_ms) {
    if (!ctx || !b || reps < 1) return HDX_E_INVALID;
    if (b->n_tiles == 0) return HDX_OK;
    hipSetDevice(ctx->device);
    if (b->staged_used) hipEventSynchronize(b->staged);
    auto candidates = [&](int c) {
        const int cap = group_width_cap(b, c);
        std::vector<Schedule> cand;
        for (int th = 64; th <= cap; th *= 2) {
            cand.push_back(Schedule{th, 0, 0});
            cand.push_back(Schedule{th, 0, 1});
            for (int p : {1, 2, 4, 8}) cand.push_back(Schedule{th, p, 0});
        }
        return cand;
    };
    // mean ms of `reps` launches of the groups in mask under schedules s
    auto time_launch = [&](const Schedule *s, uint64_t mask, float *ms) -> hipError_t {
        hipError_t e = batch_direct_launch(ctx, b, s, b->work, mask);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(b->t0, b->work);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = batch_direct_launch(ctx, b, s, b->work, mask);
        if (e == hipSuccess) e = hipEventRecord(b->t1, b->work);
        if (e == hipSuccess) e = hipEventSynchronize(b->t1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, b->t0, b->t1);
        *ms /= (float)reps;
        return e;
    };
    // schedules of the current plan's groups: 1, each group on its own
    // launch; 2, as the groups run side by side, each group's schedule once
    // more against the whole launch with the others at their choice
    auto tune_plan = [&](Schedule *trial, float *total) -> hipError_t {
        int active = 0;
        for (int c = 0; c < kGroups; ++c) active += b->plan.count[c] > 0;
        for (int k = 0; k < kGroups; ++k) trial[k] = b->sched[k];
        *total = 0.0f;
        for (int c = 0; c < kGroups; ++c) {
            if (b->plan.count[c] == 0) continue;
            float best = 1e30f;
            Schedule best_s = b->sched[c];
            for (const Schedule &s : candidates(c)) {
                trial[c] = s;
                float ms = 0.0f;
                const hipError_t e = time_launch(trial, 1ull << c, &ms);
                if (e != hipSuccess) return e;
                if (ms < best) {
                    best = ms;
                    best_s = s;
                }
            }
            trial[c] = best_s;
            *total += best;
        }
        if (active > 1) {
            float best = 0.0f;
            hipError_t e = time_launch(trial, ~0ull, &best);
            if (e != hipSuccess) return e;
            for (int c = kGroups - 1; c >= 0; --c) {
                if (b->plan.count[c] == 0) continue;
                const Schedule keep = trial[c];
                Schedule best_s = keep;
                for (const Schedule &s : candidates(c)) {
                    if (same_schedule(s, keep)) continue;
                    trial[c] = s;
                    float ms = 0.0f;
                    e = time_launch(trial, ~0ull, &ms);
                    if (e != hipSuccess) return e;
                    if (ms < best) {
                        best = ms;
                        best_s = s;
                    }
                }
                trial[c] = best_s;
            }
            *total = best;
        }
        return hipSuccess;
    };
    // both plans (one group per model, or per model and size class); the
    // faster one is kept
    hipDeviceSynchronize();
    drop_graph(b);
    const bool first = b->split;
    Schedule sa[kGroups], sb[kGroups];
    float ta = 0.0f, tb = 0.0f;
    hipError_t e = tune_plan(sa, &ta);
    if (e == hipSuccess) {
        b->split = !first;
        e = replan(b, b->work);
        if (e == hipSuccess) e = hipStreamSynchronize(b->work);
        if (e == hipSuccess) {
            default_schedules(b);
            e = tune_plan(sb, &tb);
        }
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune launch");
    const Schedule *chosen = sb;
    float total = tb;
    if (ta <= tb) {
        b->split = first;
        e = replan(b, b->work);
        if (e == hipSuccess) e = hipStreamSynchronize(b->work);
        if (e != hipSuccess) return hip_fail(ctx, e, "replan");
        chosen = sa;
        total = ta;
    }
    for (int c = 0; c < kGroups; ++c)
        if (b->plan.count[c] > 0) {
            b->sched[c] = chosen[c];
            b->sched_set[c] = true;
        }
    if (best_ms) *best_ms = total;
    return HDX_OK;
}

hdx_status hdx_rollout_bounds(hdx_ctx *ctx, const hdx_model *m, const hdx_rollout_cfg *cfg, uint32_t seed,
                              uint32_t step, hdx_states states, const uint32_t *ids, const int32_t *depths, int64_t n,
                              float *U, float *L, int32_t *steps, hdx_stream stream) {
    if (!ctx || !m || !cfg) return fail(ctx, HDX_E_INVALID, "null argument");
    if (n < 0 || n > (1ll << 31)) return fail(ctx, HDX_E_SHAPE, "n out of range");
    if (n == 0) return HDX_OK;
    if (!ids || !depths || !U || !L || !states_ok(m, states, n)) return fail(ctx, HDX_E_INVALID, "missing arrays");
    hdx_status st = check_cfg(ctx, m, *cfg);
    if (st != HDX_OK) return st;
    if (cfg->max_depth < 0 && cfg->max_steps > kHorizon)
        return fail(ctx, HDX_E_SHAPE, "rollout horizon exceeds HDX_MAX_HORIZON");
    if (cfg->max_depth > kHorizon && cfg->max_steps > kHorizon)
        return fail(ctx, HDX_E_SHAPE, "rollout horizon exceeds HDX_MAX_HORIZON");
    BoundsArgs A;
    A.model = m->d_model;
    A.k0 = seed;
    A.k1 = step;
    A.policy = cfg->policy;
    A.const_action = cfg->const_action;
    A.max_steps = cfg->max_steps;
    A.max_depth = cfg->max_depth;
    A.states = to_ptr(states);
    A.ids = ids;
    A.depths = depths;
    A.n = n;
    A.U = U;
    A.L = L;
    A.steps = steps;
    hipSetDevice(ctx->device);
    hipError_t e = launch_bounds(A, m->desc.kind, m->desc.n_peds, (hipStream_t)stream);
    return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "rollout_bounds launch");
}

hdx_status hdx_philox(hdx_ctx *ctx, const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t *out,
                      hdx_stream stream) {
    if (!ctx || (count > 0 && (!ctr || !out)) || count < 0) return fail(ctx, HDX_E_INVALID, "bad argument");
    hipSetDevice(ctx->device);
    hipError_t e = launch_philox(ctr, count, k0, k1, out, (hipStream_t)stream);
    return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "philox launch");
}

hdx_status hdx_fp32_selftest(hdx_ctx *ctx, const float *a, const float *b, const float *c, int64_t n, float *out,
                             hdx_stream stream) {
    if (!ctx || n < 0 || (n > 0 && (!a || !b || !c || !out))) return fail(ctx, HDX_E_INVALID, "bad argument");
    hipSetDevice(ctx->device);
    hipError_t e = launch_fp32_selftest(a, b, c, n, out, (hipStream_t)stream);
    return e == hipSuccess ? HDX_OK : hip_fail(ctx, e, "fp32 selftest launch");
}

}  // extern "C"
