/*
 * hdx -- DESPOT leaf-node expansion on AMD Instinct MI355X (gfx950).
 *
 * A C ABI over hand-written HIP kernels for the data-parallel step of
 * HyP-DESPOT (Cai, Luo, Hsu, Lee; arXiv:1802.06215): a leaf of the DESPOT
 * tree is expanded one level for every action and every scenario, scenarios
 * are grouped into child nodes by observation, and each child's initial
 * upper and lower bounds are set from a heuristic and from default-policy
 * rollouts (Sec. III-D, Eq. 10-13).  The CPU side of the method -- creating
 * nodes and the Bellman backup of Eq. 4 -- is here too, as host code.
 *
 * Conventions
 *  - Every call returns an hdx_status; no exception crosses the ABI.
 *  - "device" pointers are HIP device memory (for example from
 *    torch.Tensor.data_ptr() of a CUDA/ROCm tensor); "host" pointers are
 *    ordinary process memory.  The caller owns every buffer it passes.
 *  - Device work is enqueued on the given stream (a hipStream_t; NULL = the
 *    default stream) and is asynchronous: output buffers are valid once the
 *    stream has reached the call.  Input buffers must stay valid until then.
 *  - One context may be used from several host threads if each passes its
 *    own stream; model handles are read-only after upload.
 *  - Per-call host work allocates nothing once a context has seen the
 *    largest batch it will be given (descriptor staging grows on demand).
 *
 * Scenario states: struct of arrays ("hdx_states"), one element per scenario
 *  - RockSample: w[k] packs x in bits 0-4, y in bits 5-9, rock i's quality
 *    (1 = good) in bit 10+i, terminal in bit 30.
 *  - Multi-agent RockSample: two rows of w (robots, rocks); navigation: five
 *    rows of w (robot, then the unknown cells' occupancy); see hdx_states.
 *  - Crowd driving: s[k] car position (m) along the path; car[k] = speed
 *    level (bits 0-7, speed 0.5 m/s per level) | terminal (bit 8);
 *    px/py/goal are [pedestrian][stride] arrays (FP32 metres and the index
 *    of the pedestrian's goal point), stride >= number of scenarios.
 *
 * Random numbers (the scenario's phi = (s0, numbers), Sec. III-A): one
 * Philox4x32-10 stream per scenario id with key (seed, step) and counter
 * (scenario id, absolute depth, block, tag); tag 0 = model step, 1 = initial
 * state, 2 = rollout policy.  All actions at one depth see the same numbers.
 */
#ifndef HDX_H
#define HDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hdx_status;
#define HDX_OK 0
#define HDX_E_INVALID (-1)     /* bad argument or null pointer */
#define HDX_E_DEVICE (-2)      /* a HIP call failed; see hdx_last_error */
#define HDX_E_NOMEM (-3)       /* device or pinned allocation failed */
#define HDX_E_SHAPE (-4)       /* sizes outside the supported range */
#define HDX_E_CAPACITY (-5)    /* child table too small for the leaf */
#define HDX_E_UNSUPPORTED (-6) /* model kind or option not supported */

#define HDX_ROCKSAMPLE 0
#define HDX_PEDNAV 1
#define HDX_MARS 2 /* multi-agent RockSample */
#define HDX_NAV 3  /* navigation in a partially known map */
#define HDX_MAX_NAV_GRID 16
#define HDX_MAX_NAV_UNKNOWN 128

#define HDX_MAX_ROCKS 20
#define HDX_MAX_ACTIONS 625 /* (5 + HDX_MAX_ROCKS)^2, the multi-agent model's largest */
#define HDX_MAX_GRID 31
#define HDX_MAX_PEDS 32
#define HDX_MAX_GOALS 8
#define HDX_MAX_LEAF_SCENARIOS 2048 /* scenarios of one leaf in one tile */
#define HDX_MAX_NAV_LEAF_SCENARIOS 5120 /* navigation leaves (scenario counts up to 5000 in Sec. IV,
                                           effect of the number of scenarios) */
#define HDX_MAX_HORIZON 4096        /* longest rollout (discount table size) */

#define HDX_POLICY_DEFAULT 0 /* RockSample: move east; driving: brake for a pedestrian ahead, else accelerate */
#define HDX_POLICY_CONST 1   /* always const_action */
#define HDX_POLICY_RANDOM 2  /* uniform action per step from tag-2 numbers */

typedef struct hdx_ctx hdx_ctx;
typedef struct hdx_model hdx_model;
typedef struct hdx_tree hdx_tree;
typedef void *hdx_stream; /* hipStream_t */

/* Model description (host memory; may be freed after hdx_upload_model).
 * RockSample (Sec. IV-A, one robot): grid x grid cells, n_rocks rocks at
 * (rock_x[i], rock_y[i]); actions 0 north (y+1), 1 south, 2 east (x+1),
 * 3 west, 4 sample, 5+i sense rock i; rewards +10 good sample, -10 bad
 * sample, +10 exit east (terminal); sensor accuracy 0.5 + 0.5 2^(-d/20).
 * Multi-agent RockSample (Sec. IV-A): the same grid and rocks with two
 * robots; joint action a = a1 (5 + n_rocks) + a2, each robot's own action
 * numbered as above, so n_actions = (5 + n_rocks)^2 (625 for 20 rocks);
 * robot 1 acts first, then robot 2 on the rocks robot 1 left; each robot
 * earns +10 on leaving through the east border and then does nothing; the
 * world ends when both have left; robot j (0, 1) reads word j of its step's
 * random block for a sense; observation 3 z1 + z2 (9 values); grid >= 2.
 * Navigation (Sec. IV-A): a grid x grid map (5..16; 13 in the paper), row 0
 * at the top; nav_cell[y * grid + x] = -1 known free, -2 known wall, or the
 * index (0..127) of an unknown cell; unknown cells 0 and 1 are the gates of
 * the wall on row nav_wall (columns nav_gate_x); the goal is
 * (nav_goal_x, grid - 1).  Actions 0 stay (-0.2), 1-8 move N, NE, E, SE, S,
 * SW, W, NW (-0.1; y grows downwards); a move fails with p_fail (the robot
 * stays, still -0.1); a move into a wall, an occupied unknown cell or off
 * the map is a crash (-1, the robot stays); entering the goal pays +20 and
 * ends the episode.  Observation: bit j = neighbour j+1 occupied (off the
 * map reads occupied), each flipped with p_err; 256 once terminal.
 * Crowd driving (Sec. IV-A): straight path of path_len metres, n_levels
 * speed levels, pedestrians walking at ped_speed to one of n_goals goal
 * points with Gaussian heading noise sigma_h; actions 0 accelerate,
 * 1 maintain, 2 decelerate, failing with probability p_fail. */
typedef struct {
    int32_t kind;     /* HDX_ROCKSAMPLE, HDX_PEDNAV, HDX_MARS or HDX_NAV */
    int32_t n_actions;/* 5 + n_rocks, 3, (5 + n_rocks)^2, or 9 */
    double gamma;     /* discount */
    int32_t grid, n_rocks;
    int32_t rock_x[HDX_MAX_ROCKS], rock_y[HDX_MAX_ROCKS];
    int32_t n_peds, n_goals, n_levels, reserved;
    float goal_x[HDX_MAX_GOALS], goal_y[HDX_MAX_GOALS];
    float path_len, dt, ped_speed, sigma_h, coll_radius;
    float r_collision, r_step, r_goal;
    double p_fail;    /* driving: action failure; navigation: move failure */
    int32_t nav_goal_x, nav_wall, nav_gate_x[2];
    int16_t nav_cell[HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID];
    double p_err;     /* navigation: per-neighbour reading error */
} hdx_model_desc;

/* Belief to sample start states from (host memory). */
typedef struct {
    int32_t x, y;          /* RockSample: known robot cell */
    const double *p_good;  /* RockSample: [n_rocks] P(rock i good); navigation: [unknown cells]
                              P(cell occupied), entries 0 and 1 (the gates, one open with
                              probability 1/2 each) ignored; the robot starts on row 0 at a
                              uniformly drawn column */
    float s;               /* driving: car position */
    int32_t level;         /* driving: speed level */
    const float *px, *py;  /* driving: [n_peds] pedestrian positions */
    const double *goal_p;  /* driving: [n_peds][n_goals] goal probabilities */
    int32_t x2, y2;        /* multi-agent: robot 2's cell (x, y is robot 1's) */
    int32_t gone;          /* multi-agent: bit j set if robot j+1 has left */
} hdx_belief;

/* Rollout configuration for the lower bound (Eq. 13).  A rollout from depth
 * d0 runs at most min(max_steps, max_depth - d0) steps (max_depth < 0: no
 * depth limit), stops at a terminal state, and has tail value 0. */
typedef struct {
    int32_t policy;       /* HDX_POLICY_* */
    int32_t const_action; /* for HDX_POLICY_CONST */
    int32_t max_steps;
    int32_t max_depth;
} hdx_rollout_cfg;

/* Scenario states, struct of arrays (device pointers).  RockSample: w[k],
 * the packed word.  Multi-agent RockSample: w[k] the robots' row (robot 1's
 * x, y in bits 0-4, 5-9, robot 2's in bits 10-14, 15-19, robot j gone in
 * bit 20+j, terminal in bit 30) and w[stride + k] the rocks' row (rock i's
 * quality in bit i).  Navigation: w[k] the robot (x bits 0-3, y bits 4-7,
 * terminal bit 30), then w[(1 + j) * stride + k], j = 0..3, unknown cell i
 * occupied in bit i % 32 of row 1 + i / 32.  Driving: s[k], car[k] (speed level | terminal << 8)
 * and px, py, goal [n_peds][stride]. */
typedef struct {
    int32_t *w;
    float *s;
    int32_t *car;
    float *px, *py;
    uint8_t *goal;
    int64_t stride;
} hdx_states;

/* One leaf to expand (Sec. III-D: gather, update, expand, bounds).  All
 * array members are device pointers.  With A = the model's action count and
 * n = number of the leaf's scenarios:
 *   inputs
 *     parent, parent_ids : the parent's states and scenario ids
 *     idx[n]             : positions of the leaf's scenarios in the parent
 *                          arrays (int16, so below 32768), strictly
 *                          ascending
 *     depth              : the leaf's depth (root = 0); the update step uses
 *                          depth-1, expansion depth, rollouts depth+1 on
 *     last_action        : action from the parent, or -1 for a root (states
 *                          are then taken as they are)
 *     cap                : child slots per action in the child arrays; must
 *                          be >= hdx_model_max_children(model, n)
 *   outputs
 *     states_out, ids_out[n] : the leaf's own states (materialised) and ids
 *     perm[A][n]         : leaf positions grouped by child (children in
 *                          ascending observation, positions ascending);
 *                          int16, two bytes per scenario, so a child's
 *                          segment perm[a][off..off+count) is directly the
 *                          idx of that child when it is expanded
 *     n_children[A]      : children per action (Eq. 11)
 *     child_z, child_n, child_off [A][cap] : observation, scenario count and
 *                          offset into perm[a] of each child
 *     child_u0, child_l0 [A][cap] : initial bounds (Eq. 12, 13), FP32 means
 *     r_mean[A]          : mean step reward per action (first term of Eq. 4)
 *     steps[A][2]        : model steps on non-terminal states, in expansion
 *                          and in rollouts
 *   optional outputs (NULL to skip): sprime (stride >= A*n, element a*n+k),
 *     r, z, U, L, child_of [A][n] per (action, scenario). */
typedef struct {
    const hdx_model *model;
    uint32_t seed, step;     /* random-stream key */
    hdx_rollout_cfg rollout;
    hdx_states parent;
    const uint32_t *parent_ids;
    const int16_t *idx;
    int32_t n, depth, last_action, cap;
    hdx_states states_out;
    uint32_t *ids_out;
    int16_t *perm;
    int32_t *n_children;
    uint64_t *child_z;
    int32_t *child_n, *child_off;
    float *child_u0, *child_l0;
    float *r_mean;
    int64_t *steps;
    hdx_states sprime;
    float *r;
    uint64_t *z;
    float *U, *L;
    int32_t *child_of;
} hdx_leaf;

const char *hdx_version(void);

/* Context on HIP device `device`.  The library owns *out; release it with
 * hdx_fini.  Errors: HDX_E_DEVICE if the device cannot be used. */
hdx_status hdx_init(int32_t device, hdx_ctx **out);
hdx_status hdx_fini(hdx_ctx *ctx);
/* Text of the last error on this context (valid until the next call). */
const char *hdx_last_error(const hdx_ctx *ctx);

/* Upload a model (Sec. III-A: the simulative model g).  Builds the device
 * tables (sensor thresholds, discount powers) from the description.  The
 * library owns *out; free it with hdx_free_model after the last use on any
 * stream.  Errors: HDX_E_SHAPE for sizes beyond the HDX_MAX_* limits,
 * HDX_E_UNSUPPORTED for an unknown kind. */
hdx_status hdx_upload_model(hdx_ctx *ctx, const hdx_model_desc *desc, hdx_model **out);
hdx_status hdx_free_model(hdx_ctx *ctx, hdx_model *model);
int32_t hdx_model_actions(const hdx_model *model);
/* Largest child count one action can produce for a leaf of n scenarios. */
int32_t hdx_model_max_children(const hdx_model *model, int32_t n);
/* Workspace query: device bytes the caller provides for the required
 * outputs of n_leaves leaves of K scenarios each (states_out, ids_out,
 * perm, n_children, the child table with cap = hdx_model_max_children(K),
 * r_mean, steps; each array rounded up to 256 bytes), without the optional
 * per-pair outputs.  0 for a NULL model or negative sizes. */
size_t hdx_expand_out_bytes(const hdx_model *model, int32_t K, int32_t n_leaves);

/* sample_scenarios (Sec. III-A): K start states drawn from the belief into
 * `out` (device), scenario k using counter (k, 0, block, 1).  Errors:
 * HDX_E_SHAPE for K <= 0 or K > 2^24. */
hdx_status hdx_sample_scenarios(hdx_ctx *ctx, const hdx_model *model, const hdx_belief *belief,
                                int32_t K, uint32_t seed, uint32_t step, hdx_states out,
                                hdx_stream stream);

/* expand_leaf (Sec. III-D, Eq. 10-13): expand n_leaves leaves (host array
 * of descriptors pointing at device buffers) in one launch; leaves may use
 * different models, sizes and rollout settings.  Results are written as
 * described for hdx_leaf and do not depend on how leaves are batched or on
 * the launch schedule.  Errors: HDX_E_SHAPE if a leaf has more than
 * HDX_MAX_LEAF_SCENARIOS scenarios (HDX_MAX_NAV_LEAF_SCENARIOS for
 * navigation) or a rollout longer than
 * HDX_MAX_HORIZON, HDX_E_CAPACITY if cap is too small, HDX_E_INVALID for a
 * missing required pointer; nothing is launched on error. */
hdx_status hdx_expand_leaf(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves,
                           hdx_stream stream);

/* ---- Expansion that allocates nothing ---------------------------------- */

/* For callers that cannot allocate device or host memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * hdx_expand_leaf_noalloc expands leaves exactly as hdx_expand_leaf does
 * (same arguments, outputs, validation and errors; results bit-identical),
 * but the call's own device buffers -- the leaf descriptors, the (leaf,
 * action) tile list and the tile-queue heads -- live in a fixed array of
 * the library, HDX_NOALLOC_SCRATCH_BYTES on each GPU it runs on, held until
 * the process ends, and the host staging it copies them from is set up by
 * hdx_init.  The call itself allocates nothing: no hipMalloc, hipFree or
 * other allocating routine, host or device.
 * Limits: at most HDX_NOALLOC_MAX_LEAVES leaves and HDX_NOALLOC_MAX_TILES
 * tiles (the sum of the leaves' action counts) per call; beyond them the
 * call returns HDX_E_CAPACITY and launches nothing.
 * Sharing: every call on a GPU uses that GPU's one array, which keeps the
 * last call's contents (the queue heads are rewritten by every call).  Calls
 * on one stream are ordered; calls that overlap on one GPU -- on other
 * streams, from other threads or other contexts -- race and must not be
 * made.  Up to four leaves of one kernel travel in the kernel arguments, as
 * in hdx_expand_leaf, and leave the array untouched. */
#define HDX_NOALLOC_MAX_LEAVES 512
#define HDX_NOALLOC_MAX_TILES 65536
#define HDX_NOALLOC_SCRATCH_BYTES (1 << 20)
hdx_status hdx_expand_leaf_noalloc(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, hdx_stream stream);

/* ---- Batched form: many leaves, many instances, one launch ------------- */

/* A reusable batch of leaves (node-level parallelism of Sec. III-D, leaves
 * from many search threads and many planner instances in one launch).  The
 * descriptors live in device memory owned by the batch, so a launch does no
 * host work and can be captured in a HIP graph and replayed; in persistent
 * mode the kernel drains a tile queue with a fixed grid, so one captured
 * graph serves every batch of the same kernel variant.  The library owns
 * *out (release with hdx_batch_destroy).  A batch is used on one stream at
 * a time. */
typedef struct hdx_batch hdx_batch;
hdx_status hdx_batch_create(hdx_ctx *ctx, int32_t max_leaves, int64_t max_tiles, hdx_batch **out);
hdx_status hdx_batch_destroy(hdx_ctx *ctx, hdx_batch *batch);
/* Validate and stage n_leaves leaves (same rules and errors as
 * hdx_expand_leaf, plus HDX_E_CAPACITY beyond the batch's capacity); the
 * copy to device memory is enqueued on `stream`. */
hdx_status hdx_batch_set_leaves(hdx_ctx *ctx, hdx_batch *batch, const hdx_leaf *leaves, int32_t n_leaves,
                                hdx_stream stream);
/* Launch plan and schedule.  Tiles launch in groups of one model variant
 * (0 RockSample; 1, 2, 3 driving with up to 8, 16, 32 pedestrians; 4
 * multi-agent RockSample; 5 navigation), each
 * group one dispatch with an LDS carve-up and workgroup size for its
 * largest leaf, tiles ordered largest leaf first.  Unsplit (the default):
 * one group per variant, filed under the size class of its largest leaf.
 * Split: one group per variant and size class of leaf (class c holds leaves
 * of 64*2^(c-1) < n <= 64*2^c scenarios, c = 0..5), the groups launched side
 * by side.  Group = variant * HDX_SIZE_CLASSES + class.  set_split re-plans
 * the staged leaves (and later ones).  A group's schedule: workgroup size
 * (multiple of 64; capped at 512 for both RockSample models and 256 for
 * driving, and at
 * what the group's leaves need), persistent workgroups per CU (0 = one
 * workgroup per tile), and the XCD-contiguous tile mapping.  set_schedule applies to every group, set_class_schedule to the
 * groups of one size class; get_group_schedule reports one group (and its
 * tile count), get_class_schedule the class's group with the most tiles,
 * get_schedule the group with the most tiles.  Results are bit-identical
 * under every schedule. */
#define HDX_SIZE_CLASSES 6
#define HDX_LAUNCH_GROUPS 36
hdx_status hdx_batch_set_split(hdx_ctx *ctx, hdx_batch *batch, int32_t split);
hdx_status hdx_batch_get_split(const hdx_batch *batch, int32_t *split);
hdx_status hdx_batch_set_schedule(hdx_ctx *ctx, hdx_batch *batch, int32_t threads, int32_t persistent,
                                  int32_t xcd_remap);
hdx_status hdx_batch_set_class_schedule(hdx_ctx *ctx, hdx_batch *batch, int32_t size_class, int32_t threads,
                                        int32_t persistent, int32_t xcd_remap);
/* tiles may be NULL. */
hdx_status hdx_batch_get_class_schedule(const hdx_batch *batch, int32_t size_class, int32_t *threads,
                                        int32_t *persistent, int32_t *xcd_remap, int64_t *tiles);
hdx_status hdx_batch_get_group_schedule(const hdx_batch *batch, int32_t group, int32_t *threads, int32_t *persistent,
                                        int32_t *xcd_remap, int64_t *tiles);
hdx_status hdx_batch_get_schedule(const hdx_batch *batch, int32_t *threads, int32_t *persistent,
                                  int32_t *xcd_remap);
/* Launch through a captured HIP graph (captured on first use and again
 * when the kernel variant or schedule changes). */
hdx_status hdx_batch_use_graph(hdx_ctx *ctx, hdx_batch *batch, int32_t enable);
/* Expand every staged leaf: one kernel launch (or graph replay), no copies. */
hdx_status hdx_batch_launch(hdx_ctx *ctx, hdx_batch *batch, hdx_stream stream);
/* Autotuner (an internal stream; blocks until done), for the unsplit and
 * the split plan in turn: per launch group, time each candidate schedule
 * `reps` times on that group's staged tiles alone; then, as the groups run
 * side by side, refine each group's schedule once more against the whole
 * launch.  The faster plan and its schedules are kept.  *best_ms is the mean
 * time of the chosen whole launch (of the single group when there is one).
 * Outputs are rewritten with identical values. */
hdx_status hdx_batch_autotune(hdx_ctx *ctx, hdx_batch *batch, int32_t reps, float *best_ms);

/* rollout_bounds (Eq. 12, 13 per scenario): for each of n states (device),
 * U = upper-bound heuristic and L = discounted default-policy rollout from
 * depths[k]; steps[k] = model steps taken.  ids/depths/U/L/steps are
 * device arrays of n elements. */
hdx_status hdx_rollout_bounds(hdx_ctx *ctx, const hdx_model *model, const hdx_rollout_cfg *cfg,
                              uint32_t seed, uint32_t step, hdx_states states,
                              const uint32_t *ids, const int32_t *depths, int64_t n, float *U,
                              float *L, int32_t *steps, hdx_stream stream);

/* The raw Philox4x32-10 block function on device, for checking the random
 * stream: out[i][0..3] = philox(ctr[i][0..3], key (k0, k1)). */
hdx_status hdx_philox(hdx_ctx *ctx, const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1,
                      uint32_t *out, hdx_stream stream);

/* Rounding self-test of the FP32 operations the driving model's state
 * update relies on being IEEE-754 exact on the device (device arrays of n):
 * out[0][i] = sqrt(|a_i|), out[1][i] = a_i / b_i, out[2][i] = a_i*b_i + c_i
 * (two roundings, no fused multiply-add), out[3][i] = floor(a_i). */
hdx_status hdx_fp32_selftest(hdx_ctx *ctx, const float *a, const float *b, const float *c, int64_t n,
                             float *out, hdx_stream stream);

/* ---- Host side of the method: DESPOT tree and backup (Sec. III-A) ------ */

/* A tree whose root holds n_root scenarios with bounds (u0, l0).  Node 0 is
 * the root.  The library owns *out; release with hdx_tree_destroy. */
hdx_status hdx_tree_create(int32_t n_actions, double gamma, int32_t n_root, double u0, double l0,
                           hdx_tree **out);
hdx_status hdx_tree_destroy(hdx_tree *tree);
/* Attach the action and observation branches of an expanded node from a
 * host copy of its hdx_leaf outputs (Eq. 11): for action a, children
 * c < n_children[a] with (child_z, child_n, child_u0, child_l0)[a*cap+c];
 * r_mean[a].  Child node ids are assigned in (a, c) order starting at
 * *first_child.  Errors: HDX_E_INVALID if the node already has children or
 * the child counts do not sum to the node's scenario count. */
hdx_status hdx_tree_add_children(hdx_tree *tree, int64_t node, const int32_t *n_children,
                                 const uint64_t *child_z, const int32_t *child_n,
                                 const float *child_u0, const float *child_l0,
                                 const float *r_mean, int32_t cap, int64_t *first_child);
/* backup (Eq. 4): recompute u and l of `node` and of every ancestor up to
 * the root, V(b) = max_a { R(b,a) + gamma sum_z |Phi_b'|/|Phi_b| V(b') }. */
hdx_status hdx_backup(hdx_tree *tree, int64_t node);
hdx_status hdx_tree_bounds(const hdx_tree *tree, int64_t node, double *u, double *l);
int64_t hdx_tree_size(const hdx_tree *tree);

/* Belief update of the online loop (Sec. III-A, Eq. 3) for RockSample,
 * host only: the belief after `action` and observation z from belief b (the
 * robot cell x, y and p_good[n_rocks] of the description).  The robot's
 * moves are deterministic, so the new cell is the action's; sampling makes
 * the rock under the robot bad (p = 0); a reading z (1 good, 2 bad) of rock
 * i at Euclidean distance d, correct with probability 0.5 + 0.5 2^(-d/20),
 * updates p_i by Bayes' rule.  *out is b with the new cell and p_good =
 * p_out (caller-owned, n_rocks entries); *terminal is 1 when the action
 * leaves the grid eastwards.  HDX_E_UNSUPPORTED for other models,
 * HDX_E_INVALID for a cell outside the grid, an unknown action, or a
 * reading that is neither 1 nor 2. */
hdx_status hdx_belief_update(const hdx_model_desc *desc, const hdx_belief *b, int32_t action, uint64_t z,
                             hdx_belief *out, double *p_out, int32_t *terminal);

/* ---- Rollout-value surrogate ------------------------------------------- */

/* A small MLP that estimates the default-policy rollout value of a state
 * (the lower-bound term of Eq. 13) from 64 state features:
 * 64 -> 256 -> 256 -> 256 -> 1 with ReLU, BF16 weights and activations on
 * MFMA with FP32 accumulation, FP32 master weights trained with Adam on the
 * mean squared error.  Parameters are one packed FP32 vector:
 * W1[64][256], b1[256], W2[256][256], b2[256], W3[256][256], b3[256],
 * w4[256], b4[1] (W[in][out], row-major).  Feature matrices are BF16
 * [n][64] in device memory.  Forward, backward and the optimizer are the
 * library's own kernels.  The library owns the handle; the first call with
 * a larger batch allocates scratch. */
#define HDX_MLP_IN 64
#define HDX_MLP_HIDDEN 256
#define HDX_MLP_PARAMS 148481
typedef struct hdx_mlp hdx_mlp;
/* He-uniform initialisation from `seed`. */
hdx_status hdx_mlp_create(hdx_ctx *ctx, uint32_t seed, hdx_mlp **out);
hdx_status hdx_mlp_destroy(hdx_ctx *ctx, hdx_mlp *mlp);
/* Copy the FP32 parameters to / from host memory (set resets Adam). */
hdx_status hdx_mlp_get_params(hdx_ctx *ctx, const hdx_mlp *mlp, float *host_params);
hdx_status hdx_mlp_set_params(hdx_ctx *ctx, hdx_mlp *mlp, const float *host_params);
/* Checkpoint: save writes the FP32 parameters, the Adam moments and step to
 * a file (after the device is idle); load restores them (E_SHAPE for a file
 * that is not such a checkpoint, E_INVALID if it cannot be opened). */
hdx_status hdx_mlp_save(hdx_ctx *ctx, hdx_mlp *mlp, const char *path);
hdx_status hdx_mlp_load(hdx_ctx *ctx, hdx_mlp *mlp, const char *path);
/* y[i] = MLP(X[i]) for n rows (device arrays). */
hdx_status hdx_mlp_forward(hdx_ctx *ctx, hdx_mlp *mlp, const uint16_t *X, int64_t n, float *y, hdx_stream stream);
/* Gradients of mean((MLP(X) - t)^2) over a batch (a multiple of 64, at
 * most 65536 rows) into grads (device, HDX_MLP_PARAMS floats); loss
 * (device float) may be NULL.  No update. */
hdx_status hdx_mlp_gradients(hdx_ctx *ctx, hdx_mlp *mlp, const uint16_t *X, const float *t, int32_t batch,
                             float *grads, float *loss, hdx_stream stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on one batch. */
hdx_status hdx_mlp_train_step(hdx_ctx *ctx, hdx_mlp *mlp, const uint16_t *X, const float *t, int32_t batch,
                              float lr, float *loss, hdx_stream stream);
/* Surrogate input features of n states (device): RockSample x/n, y/n,
 * terminal, (horizon - depth)/100, rock qualities, rock offsets dx/n and
 * dy/n; driving s/L, speed level, terminal, (horizon - depth)/100, then per
 * pedestrian (px - s)/10, py/10, goal/n_goals; zero padding to 64.
 * HDX_E_UNSUPPORTED for the multi-agent and navigation models (no features defined). */
hdx_status hdx_features(hdx_ctx *ctx, const hdx_model *model, hdx_states states, const int32_t *depths, int64_t n,
                        int32_t horizon, uint16_t *X, hdx_stream stream);

/* expand_leaf with the surrogate in place of the default-policy rollouts:
 * the same outputs as hdx_expand_leaf, except that child_l0 is the mean of
 * MLP(features(s')) over the child's scenarios (features at depth+1 with
 * the given horizon), steps[a][1] is 0, and L (if given) receives the
 * surrogate value per (action, scenario).  Scratch for the stepped states,
 * features and values belongs to the MLP handle (grown on demand); calls
 * on one handle are serialised.  HDX_E_UNSUPPORTED for a multi-agent or navigation leaf. */
hdx_status hdx_expand_leaf_surrogate(hdx_ctx *ctx, const hdx_leaf *leaves, int32_t n_leaves, hdx_mlp *mlp,
                                     int32_t horizon, hdx_stream stream);

/* ---- Parallel DESPOT search (Sec. III-A, III-C) over the GPU expansion -- */

/* One planning step of DESPOT run by n_threads CPU threads on one shared
 * tree.  Each trial descends from the root choosing the action by the
 * scenario-based PO-UCT bound (Eq. 8; Eq. 5 when c_a = 0) and the
 * observation branch by the weighted excess uncertainty with virtual loss
 * (Eq. 6-7, 9), stopping where the excess uncertainty is not positive; a
 * leaf it reaches above max_depth is expanded on the GPU (hdx_expand_leaf:
 * Eq. 10-13), its children attached (Eq. 11) and the path backed up (Eq. 4).
 * The threads share the tree without a tree-wide lock: descents read the
 * bounds as they stand, a leaf is claimed by an atomic state change, and
 * each backup step locks one node.  Leaves are expanded either on one HIP
 * stream per thread (batch_leaves <= 1) or by batcher threads (one per
 * batch_leaves threads, at most eight) that each take up to batch_leaves
 * pending leaves of all threads and launch them in packs of up to 11
 * (descriptors in the kernel arguments).  The search stops at the time budget, after
 * max_trials trials (if > 0), or when the root gap u - l falls below
 * gap_epsilon; it returns the action with the largest lower bound.  Device
 * memory for the tree comes from an arena of arena_bytes; when it is full
 * the search stops early (reported in the result).  A failing expansion
 * stops the search and its error is returned (text via hdx_last_error). */
typedef struct {
    int32_t K;             /* scenarios sampled at the root (up to HDX_MAX_LEAF_SCENARIOS,
                              HDX_MAX_NAV_LEAF_SCENARIOS for navigation) */
    int32_t n_threads;     /* concurrent search threads (1..64) */
    int32_t max_depth;     /* search horizon D: leaves at this depth are not expanded */
    int32_t batch_leaves;  /* <= 1: one stream per thread; > 1: batchers taking up to this many leaves */
    double time_budget_s;  /* planning time */
    int64_t max_trials;    /* 0 = no limit */
    double xi;             /* target uncertainty of Eq. 7 */
    double c_a, c_o;       /* exploration constants of Eq. 8 and Eq. 9, as multiples of the
                              root gap u(b0) - l(b0) (c_a: initial gap, c_o: current gap) */
    double gap_epsilon;    /* stop when u(b0) - l(b0) <= gap_epsilon */
    int64_t arena_bytes;   /* device memory for node data */
    uint32_t seed, step;   /* random-stream key of this planning step */
    hdx_rollout_cfg rollout;
    hdx_mlp *surrogate;    /* non-NULL: leaves are expanded with hdx_expand_leaf_surrogate (the
                              root's initial bounds still come from rollouts) */
    int32_t surrogate_horizon; /* horizon of the surrogate's remaining-depth feature */
    int32_t surrogate_judge_every; /* > 0: every j-th surrogate expansion is done with rollouts
                                      (kept in the tree) and also with the surrogate, to
                                      measure the surrogate's child-l0 error */
    double surrogate_max_rel_err;  /* > 0: once 8 leaves are judged, fall back to rollouts for
                                      the rest of the search if sum|l0_sur - l0| / sum|l0|
                                      exceeds this */
    int32_t surrogate_bias_correct; /* 1: once 8 leaves are judged, add the judged children's
                                       mean of (l0_rollout - l0_sur) to every later surrogate
                                       child l0 (at most the child's u0) */
} hdx_search_cfg;

typedef struct {
    int32_t best_action;            /* argmax_a of the root's action lower bounds */
    double u_root, l_root;          /* root bounds after the search */
    double u0_root, l0_root;        /* root bounds before the first expansion */
    int64_t trials;                 /* completed trials (expansion or stop, then backup) */
    int64_t idle_trials;            /* trials that ended without expanding a leaf */
    int64_t expansions;             /* leaves expanded on the GPU */
    int64_t nodes;                  /* tree size */
    int64_t scenario_steps;         /* model steps in expansions and rollouts */
    int64_t launches;               /* expansion kernel launches */
    int32_t max_depth_reached;
    int32_t arena_full;             /* 1 if the device arena ran out */
    double elapsed_s;
    double action_l[HDX_MAX_ACTIONS]; /* per-action lower bounds at the root (first n_actions) */
    double action_u[HDX_MAX_ACTIONS];
    int64_t judged_leaves, judged_children; /* surrogate judge: leaves and children compared */
    double judge_mae;                       /* mean |l0_sur - l0_rollout| per judged child */
    double judge_rel_err;                   /* sum |l0_sur - l0_rollout| / sum |l0_rollout| */
    double judge_bias;                      /* mean (l0_rollout - l0_sur) per judged child */
    int32_t surrogate_off;                  /* 1 if the search fell back to rollouts */
    /* where the threads' time went, summed over threads (seconds): descents
       (Eq. 7-9), expansions (launch and wait, or the batcher's round trip),
       attaching children and backups (Eq. 4) */
    double time_select_s, time_expand_s, time_backup_s;
} hdx_search_result;

hdx_status hdx_search(hdx_ctx *ctx, const hdx_model *model, const hdx_belief *belief,
                      const hdx_search_cfg *cfg, hdx_search_result *out);

#ifdef __cplusplus
}
#endif
#endif /* HDX_H */
