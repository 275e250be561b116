// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hdx.h"

namespace hdx {

constexpr int kMaxRocks = HDX_MAX_ROCKS;
constexpr int kMaxGrid = HDX_MAX_GRID;
constexpr int kMaxPeds = HDX_MAX_PEDS;
constexpr int kMaxGoals = HDX_MAX_GOALS;
constexpr int kHorizon = HDX_MAX_HORIZON;
constexpr int kSenseEntries = 2 * (kMaxGrid - 1) * (kMaxGrid - 1) + 1;  // squared distances
constexpr int kMaxLeaf = HDX_MAX_LEAF_SCENARIOS;
constexpr int kMaxNavLeaf = HDX_MAX_NAV_LEAF_SCENARIOS;

enum : uint32_t { kTagStep = 0, kTagInit = 1, kTagPolicy = 2 };
constexpr uint64_t kEmptyKey = ~0ull;
constexpr uint64_t kPedTerminalObs = ~0ull;

// Model parameters and tables as the kernels read them (device memory, one
// per uploaded model).  Derived constants are computed once on the host.
// The header is read with scalar loads; per-lane lookups of the discount
// table go through an LDS copy of its first kGpowLds entries.
struct ModelHdr {
    int32_t kind, n_actions;
    // RockSample
    int32_t grid, n_rocks;
    int32_t rock_x[kMaxRocks], rock_y[kMaxRocks];
    // crowd driving
    int32_t n_peds, n_goals, n_levels;
    // multi-agent RockSample: ceil(2^16 / (5 + n_rocks)), so that robot 1's
    // action of joint action a < (5 + n_rocks)^2 is (a * joint_inv) >> 16
    int32_t joint_inv;
    float goal_x[kMaxGoals], goal_y[kMaxGoals];
    float path_len, dt, step_len, half_sigma, coll_r2, reach, ih_scale;
    float r_collision, r_step, r_goal, pad2;
    uint64_t fail_thr;  // action fails iff word < fail_thr (driving, navigation)
    // navigation: goal column (on the bottom row), wall row, gate columns,
    // per cell -1 known free / -2 known wall / unknown cell index, and the
    // reading error (a neighbour's bit flips iff word < err_thr)
    int32_t nav_goal_x, nav_wall, nav_gate_x[2];
    int16_t nav_cell[HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID];
    uint64_t err_thr;
    // navigation rollouts: the known walls as bits 16 y + x (four words) and
    // each unknown cell's bit position 16 y + x
    uint64_t nav_wall_bits[4];
    uint8_t nav_unknown_pos[HDX_MAX_NAV_UNKNOWN];
};

constexpr int kGpowLds = 256;

struct DevModel {
    ModelHdr h;
    uint32_t sense_thr_m1[kSenseEntries];  // floor(acc(d) 2^32) - 1, by squared distance
    float gpow[kHorizon];                  // discount powers gamma^j rounded to FP32
};

struct StatesPtr {
    int32_t *w;
    float *s;
    int32_t *car;
    float *px, *py;
    uint8_t *goal;
    int64_t stride;
};

// One leaf as the expansion kernel sees it (built on the host from hdx_leaf).
struct LeafTask {
    const DevModel *model;
    int32_t kind, n_actions;
    uint32_t k0, k1;
    int32_t policy, const_action, max_steps, max_depth;
    StatesPtr parent;
    const uint32_t *parent_ids;
    const int16_t *idx;
    int32_t n, depth, last_action, cap;
    StatesPtr out;
    uint32_t *ids_out;
    int16_t *perm;
    int32_t *n_children;
    uint64_t *child_z;
    int32_t *child_n, *child_off;
    float *child_u0, *child_l0;
    float *r_mean;
    int64_t *steps;
    StatesPtr sprime;
    float *r;
    uint64_t *z;
    float *U, *L;
    int32_t *child_of;
};

struct Tile {
    int32_t leaf, action;
};

// Work queue of the persistent launch; the last workgroup to leave resets
// it, so a captured graph can be replayed without a separate clear.
struct TileQueue {
    int32_t next, done, n_tiles, pad;
};

// Launch schedule of the expansion kernel; results never depend on it.
struct Schedule {
    int32_t threads;     // workgroup size, a multiple of 64
    int32_t persistent;  // 0: one workgroup per tile; >0: that many workgroups per CU
    int32_t xcd_remap;   // keep consecutive tiles (one leaf) on one XCD
};

// LDS carve-up of one tile, the same on host (for the launch size) and
// device.  General carve-up (any model); regions live in phases and are
// reused:
//   zkey | tab    observations, then the open-addressing hash; after the
//                 children are ranked the pair holds the chunk count table
//                 (cnt), and later the grouped per-scenario sums (su, sl)
//   dslot         slot of each distinct observation, then child sizes (nc)
//   off           child offsets in the grouped order
//   ubuf, lbuf    per-scenario U and L
//   child         child index of each scenario (bits 0-15) and its rank
//                 inside its 64-scenario chunk (bits 16-23)
//   perm          grouped order (or the bitonic keys of the fallback path)
// Small carve-up (RockSample-only launches: every observation key is below
// 32, no model table staged):
//   zkey          per 64-scenario chunk and key: count, U sum, L sum
//   dslot         per chunk: mask of the keys present
//   off           per key: child offset and child index
//   child         key of each scenario (bits 0-15) and its rank inside its
//                 chunk among the scenarios of that key (bits 16-23)
struct LdsLayout {
    uint32_t zkey, tab, dslot, off, ubuf, lbuf, child, perm, misc, gpow, total;
    int32_t np, p2, h, table_cap;
    int32_t small;
};

__host__ __device__ inline int32_t pow2_at_least(int32_t v) {
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

__host__ __device__ inline LdsLayout make_layout(int32_t np, bool small = false) {
    LdsLayout L;
    if (np < 1) np = 1;
    L.np = np;
    L.small = small ? 1 : 0;
    L.p2 = pow2_at_least(np) < 64 ? 64 : pow2_at_least(np);
    L.h = pow2_at_least(2 * np) < 64 ? 64 : pow2_at_least(2 * np);
    uint32_t o = 0;
    auto take = [&](uint32_t bytes) {
        uint32_t at = o;
        o += (bytes + 15u) & ~15u;
        return at;
    };
    if (small) {
        const uint32_t chunks = (uint32_t)((np + 63) / 64);
        L.zkey = take(3u * 4u * 32u * chunks);
        L.tab = L.zkey;
        L.table_cap = 0;
        L.dslot = take(4u * chunks);
        L.off = take(4u * 64u);
        L.ubuf = L.lbuf = L.perm = L.off;  // not used by the small path
        L.child = take(2u * np);  // per scenario: key | rank << 5 (int16)
        L.misc = take(64 + 4u * 64);
        L.gpow = L.misc;
        L.total = o;
        return L;
    }
    L.zkey = take(8u * L.p2);
    L.tab = take(8u * L.h + 16u);
    L.table_cap = (int32_t)((8u * L.p2 + 8u * L.h + 16u) / 4u);
    L.dslot = take(4u * L.p2);
    L.off = take(4u * L.p2);
    L.ubuf = take(4u * np);
    L.lbuf = take(4u * np);
    L.child = take(4u * np);
    L.perm = take(4u * L.p2);
    L.misc = take(64 + 4u * 64);
    // discount powers, goal points, the navigation cell table (int16) and
    // the unknown cells' grid bits
    L.gpow = take(4u * (kGpowLds + 2 * kMaxGoals) + 2u * HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID + HDX_MAX_NAV_UNKNOWN);
    L.total = o;
    return L;
}

// Medium observation alphabet (navigation: every key below kMedKeys).
// Regions, each in use for the whole tile:
//   gpow        discount powers, goal points and the navigation cell table
//   key, rank   per scenario: observation key (16 bits) and its rank among
//               the scenarios of that key in its wavefront's chunks
//   ub, lb      per scenario: U and L
//   perm        grouped order (leaf positions)
//   su, sl      segmented sums over 64-aligned chunks of the grouped order
//   wcnt        per run of chunks (one wavefront each) and key: scenario
//               count, then the key's count in earlier runs
//   kcnt, koff, kci  per key: count, child offset, child index
//   cof, cnc    per child: offset, count
//   chunk_r     per 64-scenario chunk: step reward sum
// A leaf of up to kMaxMedLeaf scenarios fits one tile.
constexpr int kMedKeys = 264;  // 257 navigation observations, rounded up
constexpr int kMedWaves = 16;  // wavefronts of the widest workgroup
constexpr int kMaxMedLeaf = kMaxNavLeaf;
struct MedLayout {
    uint32_t gpow, key, rank, ub, lb, perm, su, sl, wcnt, kcnt, koff, kci, cof, cnc, chunk_r, misc, total;
    int32_t np;
};
__host__ __device__ inline MedLayout make_med_layout(int32_t np) {
    MedLayout L;
    if (np < 1) np = 1;
    L.np = np;
    const uint32_t n = (uint32_t)np, chunks = (n + 63u) / 64u;
    uint32_t o = 0;
    auto take = [&](uint32_t bytes) {
        uint32_t at = o;
        o += (bytes + 15u) & ~15u;
        return at;
    };
    L.gpow = take(4u * (kGpowLds + 2 * kMaxGoals) + 2u * HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID + HDX_MAX_NAV_UNKNOWN);
    L.key = take(2u * n);
    L.rank = take(2u * n);
    L.ub = take(4u * n);
    L.lb = take(4u * n);
    L.perm = take(2u * n);
    L.su = take(4u * n);
    L.sl = take(4u * n);
    L.wcnt = take(4u * (chunks < (uint32_t)kMedWaves ? chunks : (uint32_t)kMedWaves) * kMedKeys);
    L.kcnt = take(4u * kMedKeys);
    L.koff = take(4u * kMedKeys);
    L.kci = take(4u * kMedKeys);
    L.cof = take(4u * kMedKeys);
    L.cnc = take(4u * kMedKeys);
    L.chunk_r = take(4u * chunks);
    L.misc = take(64 + 4u * 64);
    L.total = o;
    return L;
}

// Kernel variant a set of leaves needs: mode 0 RockSample only, 1 driving
// only, 2 both; pm = pedestrian capacity of the register state; n_max sizes
// the LDS carve-up.
struct Variant {
    int32_t mode, pm, n_max;
    // driving only: the kernel instance whose tiles expand a leaf one lane
    // per pedestrian when n times the group width fits a wavefront
    int32_t group = 0;
};
Variant pick_variant(int32_t has_rs, int32_t has_ped, int32_t ped_max, int32_t n_max, int32_t has_mars,
                     int32_t has_nav);
int32_t variant_max_threads(const Variant &v);

// Kernel launchers (kernels.hip).  The expansion kernel reads the tile
// count from d_queue->n_tiles; n_tiles here only sizes a non-persistent grid.
hipError_t launch_expand(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queue, int32_t n_tiles,
                         const Variant &v, const Schedule &sch, int32_t n_cu, hipStream_t stream);

// Tiles are launched in groups.  A group holds tiles of one model variant
// (0 RockSample, 1-3 driving with up to 8, 16, 32 pedestrians, 4
// multi-agent RockSample, 5 navigation), so
// RockSample tiles never run in the register budget of the driving model,
// and gets an LDS carve-up and workgroup size for its own largest leaf.  By
// default all leaves of a variant form one group (one dispatch, no fork and
// join between dispatches), filed under the size class of its largest leaf;
// split plans give each size class of leaf (n <= 64, 128, 256, 512, 1024,
// and larger) a group of its own, so small leaves do not pay for the largest one's
// footprint, and launch the groups side by side.  Inside a group the tiles
// are ordered largest leaf first (long tiles start early, short ones fill
// the tail), a leaf's tiles in action order, and interleaved so that the
// tiles of one leaf go to one XCD.  Group g = variant *
// kSizeClasses + size class; the tile array is ordered by group; group g
// owns tiles [begin[g], begin[g] + count[g]) and the queue d_queues[g].
constexpr int kSizeClasses = 6;
constexpr int kXcds = 8;  // accelerator dies, each with its own L2
constexpr int kModelVariants = 6;
constexpr int kGroups = kModelVariants * kSizeClasses;
__host__ __device__ inline int size_class(int32_t n) {
    int c = 0;
    while (c < kSizeClasses - 1 && n > (64 << c)) ++c;
    return c;
}
inline int model_variant(int32_t kind, int32_t n_peds) {
    return kind == HDX_ROCKSAMPLE ? 0 : kind == HDX_MARS ? 4 : kind == HDX_NAV ? 5 : n_peds <= 8 ? 1 : n_peds <= 16 ? 2 : 3;
}
inline Variant group_variant(int g) {
    const int v = g / kSizeClasses;
    if (v == 4) return Variant{3, 1, 1};
    if (v == 5) return Variant{4, 1, 1};
    return v == 0 ? Variant{0, 1, 1} : Variant{1, v == 1 ? 8 : v == 2 ? 16 : 32, 1};
}
struct ClassPlan {
    int64_t begin[kGroups], count[kGroups];
    int32_t n_max[kGroups];
};
// Reorder tiles[0, n_tiles) by group, largest leaf first inside a group
// (variant[leaf] is the leaf's model variant); fills plan.
void plan_classes(const LeafTask *tasks, const int8_t *variant, Tile *tiles, int64_t n_tiles, ClassPlan *plan,
                  bool split);
// One launch per non-empty group in mask (bit g = group g); lds_n[g] sizes
// group g's LDS (>= its n_max); sch[g] is its schedule (its width capped at
// what the group's leaves and model need).
hipError_t launch_classes(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queues, const ClassPlan &plan,
                          const int32_t *lds_n, const Schedule *sch, int32_t n_cu, hipStream_t stream,
                          uint64_t mask = ~0ull);
// Default schedule of a group whose largest leaf has n_max scenarios.
// Latency form (a few leaves, split groups): two scenarios per lane up to
// 256 lanes (navigation: 1024), one workgroup per tile, XCD-contiguous.
// Throughput form (one group per model): both RockSample models one
// wavefront per tile (the most tiles in flight, barriers of a single
// wavefront), driving and navigation as the latency form; workgroups in
// tile order (largest first spreads over the XCDs).
Schedule class_default_schedule(int32_t n_max, int32_t max_threads, int32_t mode = -1);
hipError_t configure_expand_kernels();

// Up to kArgLeaves leaves passed by value in the kernel arguments (the
// pack stays under the 4 KB kernel-argument limit).
constexpr int kArgLeaves = 11;
struct ArgPack {
    LeafTask t[kArgLeaves];
    int32_t tile_begin[kArgLeaves + 1];
    int32_t n_leaves, n_max, xcd_remap;
};
hipError_t launch_expand_args(const ArgPack &pack, const Variant &v, const Schedule &sch, hipStream_t stream);

struct SampleArgs {
    const DevModel *model;
    uint32_t k0, k1;
    int32_t K;
    int32_t x0, y0;  // RockSample: robot cell; multi-agent: x0 is the robots' row
    uint64_t rock_thr[kMaxRocks];
    float s0;
    int32_t level0;
    float px0[kMaxPeds], py0[kMaxPeds];
    uint64_t goal_thr[kMaxPeds][kMaxGoals];  // cumulative thresholds
    int32_t n_unknown;                       // navigation: unknown cells
    uint64_t cell_thr[HDX_MAX_NAV_UNKNOWN];  // navigation: P(occupied) thresholds
    StatesPtr out;
};
// Staged in device memory (d_args) before the launch.
hipError_t launch_sample(const SampleArgs *d_args, int32_t K, hipStream_t stream);

struct BoundsArgs {
    const DevModel *model;
    uint32_t k0, k1;
    int32_t policy, const_action, max_steps, max_depth;
    StatesPtr states;
    const uint32_t *ids;
    const int32_t *depths;
    int64_t n;
    float *U, *L;
    int32_t *steps;
};
hipError_t launch_bounds(const BoundsArgs &args, int32_t kind, int32_t n_peds, hipStream_t stream);

hipError_t launch_philox(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t stream);

hipError_t launch_fp32_selftest(const float *a, const float *b, const float *c, int64_t n, float *out,
                                hipStream_t stream);

int32_t max_dynamic_lds();

}  // namespace hdx

// The description a model was uploaded from (host side, runtime.cpp).
const hdx_model_desc *hdx_internal_desc(const hdx_model *m);
void hdx_internal_set_error(hdx_ctx *ctx, const char *msg);
void hdx_internal_quiesce(hdx_ctx *ctx);
const hdx::DevModel *hdx_internal_devmodel(const hdx_model *m);

namespace hdx {

}  // namespace hdx
