/*
 * Sequential CPU oracle for DESPOT leaf-node expansion as HyP-DESPOT uses it
 * (Cai, Luo, Hsu, Lee, "HyP-DESPOT", arXiv:1802.06215).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg call this file; the GPU library never links,
 * includes or calls it, and it shares no code with the GPU library.
 *
 * What it computes, written as plain loops in the paper's order:
 *   - scenarios phi = (s0, random numbers) (Sec. III-A, DESPOT);
 *   - leaf expansion: gather + update, then s',z = g(s,a,phi) for every
 *     action and scenario (Eq. 10, Sec. III-D);
 *   - grouping of scenarios by observation into children (Eq. 11);
 *   - per-child mean of the upper-bound heuristic (Eq. 12) and of the
 *     discounted default-policy rollout return (Eq. 13);
 *   - the per-action mean step reward, the first term of Eq. 4.
 * Values are accumulated in FP64.  The crowd-driving model's state update is
 * FP32 by definition (its positions are FP32 numbers), so it is evaluated in
 * FP32 here too, with contraction disabled at compile time.
 *
 * Readings of points the paper leaves open (random-number indexing, the two
 * model definitions, bound heuristics, child order) follow the project's
 * model specification; each is named where it is used.
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Ten rounds; the key is bumped by the Weyl       */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static void philox_block(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t count)
{
    for (int64_t i = 0; i < count; i++)
        philox_block(ctr + 4 * i, key, out + 4 * i);
}

/* The scenario's random numbers (Sec. III-A): one counter-based stream per
 * scenario id, addressed by absolute tree depth, so every action at a depth
 * sees the same numbers.  Key = (episode seed, planning step); counter =
 * (scenario id, depth, block, purpose tag). */
enum { TAG_STEP = 0, TAG_INIT = 1, TAG_POLICY = 2 };

static void draw_block(uint32_t seed, uint32_t step, uint32_t id, uint32_t depth,
                       uint32_t block, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {id, depth, block, tag};
    uint32_t key[2] = {seed, step};
    philox_block(ctr, key, out);
}

/* Bernoulli(p) from a 32-bit uniform word: success iff word < floor(p 2^32). */
static uint64_t prob_threshold(double p)
{
    if (p <= 0.0) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------ */
/* Models                                                                    */
/* ------------------------------------------------------------------------ */
#define OR_MAX_ROCKS 20
#define OR_MAX_PEDS 32
#define OR_MAX_GOALS 8

typedef struct {
    int32_t kind; /* 0: RockSample, 1: crowd driving, 2: multi-agent RockSample, 3: navigation */
    int32_t n_actions;
    double gamma;
    /* RockSample */
    int32_t n, m;
    int32_t rock_x[OR_MAX_ROCKS], rock_y[OR_MAX_ROCKS];
    /* crowd driving */
    int32_t n_peds, n_goals, n_levels, pad_;
    float goal_x[OR_MAX_GOALS], goal_y[OR_MAX_GOALS];
    float path_len, dt, ped_speed, sigma_h, coll_radius;
    float r_collision, r_step, r_goal;
    double p_fail;
    /* navigation (also uses n, gamma, p_fail) */
    int32_t nav_goal_x, nav_wall, nav_gate_x[2];
    int16_t nav_cell[256]; /* [y * n + x]: -1 known free, -2 known wall, >= 0 unknown cell index */
    double p_err;          /* per-neighbour sensor error */
} or_model;

typedef struct {
    int32_t policy;       /* 0: model default, 1: constant action, 2: uniform random */
    int32_t const_action; /* used by policy 1 */
    int32_t max_steps;    /* rollout length cap R */
    int32_t max_depth;    /* search horizon D; negative = unbounded */
} or_rollout_cfg;

/* One scenario's state, in a form the plain loops can copy freely. */
typedef struct {
    int32_t w;  /* RockSample: packed word; multi-agent: the robots' row */
    int32_t w2; /* multi-agent RockSample: the rocks' row */
    int32_t nw[4]; /* navigation: unknown cells' occupancy, cell i in bit i%32 of nw[i/32] */
    float s;   /* crowd driving: car position along the path */
    int32_t level;
    int32_t term;
    float px[OR_MAX_PEDS], py[OR_MAX_PEDS];
    uint8_t goal[OR_MAX_PEDS];
} or_state;

/* Struct-of-arrays views, in the library's documented state layout. */
typedef struct {
    int32_t *w;     /* RockSample word per scenario; multi-agent: [2][stride] */
    float *s;       /* car position */
    int32_t *car;   /* speed level in bits 0-7, terminal in bit 8 */
    float *px, *py; /* [ped][scenario] */
    uint8_t *goal;  /* [ped][scenario] */
    int64_t stride; /* scenarios per row of the [ped][scenario] arrays */
} or_soa;

static void load_state(const or_model *M, const or_soa *A, int64_t k, or_state *st)
{
    memset(st, 0, sizeof(*st));
    if (M->kind == 0) {
        st->w = A->w[k];
        st->term = (st->w >> 30) & 1;
    } else if (M->kind == 2) {
        st->w = A->w[k];
        st->w2 = A->w[A->stride + k];
        st->term = (st->w >> 30) & 1;
    } else if (M->kind == 3) {
        st->w = A->w[k];
        for (int j = 0; j < 4; j++) st->nw[j] = A->w[(1 + j) * A->stride + k];
        st->term = (st->w >> 30) & 1;
    } else {
        st->s = A->s[k];
        st->level = A->car[k] & 0xff;
        st->term = (A->car[k] >> 8) & 1;
        for (int j = 0; j < M->n_peds; j++) {
            st->px[j] = A->px[j * A->stride + k];
            st->py[j] = A->py[j * A->stride + k];
            st->goal[j] = A->goal[j * A->stride + k];
        }
    }
}

static void store_state(const or_model *M, const or_soa *A, int64_t k, const or_state *st)
{
    if (M->kind == 0) {
        A->w[k] = st->w;
    } else if (M->kind == 2) {
        A->w[k] = st->w;
        A->w[A->stride + k] = st->w2;
    } else if (M->kind == 3) {
        A->w[k] = st->w;
        for (int j = 0; j < 4; j++) A->w[(1 + j) * A->stride + k] = st->nw[j];
    } else {
        A->s[k] = st->s;
        A->car[k] = (st->level & 0xff) | (st->term ? 0x100 : 0);
        for (int j = 0; j < M->n_peds; j++) {
            A->px[j * A->stride + k] = st->px[j];
            A->py[j * A->stride + k] = st->py[j];
            A->goal[j * A->stride + k] = st->goal[j];
        }
    }
}

/* --- RockSample (Sec. IV-A, one robot): state word = x in bits 0-4,
 *     y in bits 5-9, quality of rock i in bit 10+i, terminal in bit 30.
 *     Actions 0..3 = north (y+1), south, east (x+1), west; 4 = sample;
 *     5+i = sense rock i.  Observations 0 = none, 1 = good, 2 = bad. */
enum { RS_NORTH = 0, RS_SOUTH = 1, RS_EAST = 2, RS_WEST = 3, RS_SAMPLE = 4, RS_SENSE0 = 5 };
enum { OBS_NONE = 0, OBS_GOOD = 1, OBS_BAD = 2 };

static int rs_x(int32_t w) { return w & 31; }
static int rs_y(int32_t w) { return (w >> 5) & 31; }
static int rs_good(int32_t w, int i) { return (w >> (10 + i)) & 1; }

/* Sensor accuracy decays exponentially with distance: 0.5 + 0.5 2^(-d/20),
 * d the Euclidean distance between robot cell and rock cell. */
static uint64_t rs_sense_threshold(int d2)
{
    double acc = 0.5 + 0.5 * pow(2.0, -sqrt((double)d2) / 20.0);
    return prob_threshold(acc);
}

static void rs_step(const or_model *M, or_state *st, int a, uint32_t seed, uint32_t step,
                    uint32_t id, uint32_t depth, float *r, uint64_t *z)
{
    int32_t w = st->w;
    *r = 0.0f;
    *z = OBS_NONE;
    if (st->term) return; /* terminal states are absorbing */
    int x = rs_x(w), y = rs_y(w), n = M->n;
    if (a == RS_NORTH) {
        if (y + 1 < n) y = y + 1; /* a move into a wall is a no-op */
    } else if (a == RS_SOUTH) {
        if (y > 0) y = y - 1;
    } else if (a == RS_WEST) {
        if (x > 0) x = x - 1;
    } else if (a == RS_EAST) {
        if (x + 1 == n) { /* leaving through the east border ends the episode */
            *r = 10.0f;
            st->term = 1;
        } else {
            x = x + 1;
        }
    } else if (a == RS_SAMPLE) {
        for (int i = 0; i < M->m; i++) {
            if (M->rock_x[i] == x && M->rock_y[i] == y) {
                if (rs_good(w, i)) {
                    *r = 10.0f;
                    w &= ~(1 << (10 + i)); /* a sampled rock turns bad */
                } else {
                    *r = -10.0f;
                }
            }
        }
    } else {
        int i = a - RS_SENSE0;
        int dx = x - M->rock_x[i], dy = y - M->rock_y[i];
        uint32_t u[4];
        draw_block(seed, step, id, depth, 0, TAG_STEP, u);
        int correct = (uint64_t)u[0] < rs_sense_threshold(dx * dx + dy * dy);
        int truth = rs_good(w, i);
        int reading = correct ? truth : !truth;
        *z = reading ? OBS_GOOD : OBS_BAD;
    }
    w = (w & ~0x3ff) | x | (y << 5);
    if (st->term) w |= 1 << 30;
    st->w = w;
}

/* Optimistic value: every good rock sampled on arrival at the shortest path
 * length, plus the exit reward at the shortest exit time. */
static double rs_upper(const or_model *M, const or_state *st)
{
    if (st->term) return 0.0;
    int x = rs_x(st->w), y = rs_y(st->w);
    double u = 0.0;
    for (int i = 0; i < M->m; i++)
        if (rs_good(st->w, i))
            u += 10.0 * pow(M->gamma, abs(x - M->rock_x[i]) + abs(y - M->rock_y[i]));
    u += 10.0 * pow(M->gamma, M->n - 1 - x);
    return u;
}

/* --- Multi-agent RockSample (Sec. IV-A): two robots on one n x n grid
 *     share the m rocks; each robot moves to a neighbouring cell, senses a
 *     rock or samples the rock it stands on, and earns +10 when it leaves
 *     through the east border; the world ends when both have left.
 *     State, two rows: robots' row = robot 1's cell (x bits 0-4, y bits
 *     5-9), robot 2's cell (x bits 10-14, y bits 15-19), robot j gone in bit
 *     20+j, terminal (both gone) in bit 30; rocks' row = quality of rock i in
 *     bit i.  Joint action a = a1 (5+m) + a2, each robot's own action
 *     numbered as in RockSample.  Readings: robot 1 acts first and robot 2
 *     then acts on the rocks robot 1 left (a rock both sample in one step
 *     pays +10 then -10); a robot that has left does nothing; robot j's
 *     sensor reads word j of the step block; the joint observation is
 *     3 z1 + z2. */
#define MARS_GONE0 20
#define MARS_TERM 30

static void mars_robot(const or_model *M, or_state *st, int j, int b, uint32_t word, float *r, int *zj)
{
    int32_t w = st->w;
    *r = 0.0f;
    *zj = OBS_NONE;
    if ((w >> (MARS_GONE0 + j)) & 1) return; /* this robot has left the map */
    int sh = 10 * j, n = M->n;
    int x = (w >> sh) & 31, y = (w >> (sh + 5)) & 31;
    if (b == RS_NORTH) {
        if (y + 1 < n) y = y + 1;
    } else if (b == RS_SOUTH) {
        if (y > 0) y = y - 1;
    } else if (b == RS_WEST) {
        if (x > 0) x = x - 1;
    } else if (b == RS_EAST) {
        if (x + 1 == n) {
            *r = 10.0f;
            w |= 1 << (MARS_GONE0 + j);
        } else {
            x = x + 1;
        }
    } else if (b == RS_SAMPLE) {
        for (int i = 0; i < M->m; i++) {
            if (M->rock_x[i] == x && M->rock_y[i] == y) {
                if ((st->w2 >> i) & 1) {
                    *r = 10.0f;
                    st->w2 &= ~(1 << i);
                } else {
                    *r = -10.0f;
                }
            }
        }
    } else {
        int i = b - RS_SENSE0;
        int dx = x - M->rock_x[i], dy = y - M->rock_y[i];
        int correct = (uint64_t)word < rs_sense_threshold(dx * dx + dy * dy);
        int truth = (st->w2 >> i) & 1;
        int reading = correct ? truth : !truth;
        *zj = reading ? OBS_GOOD : OBS_BAD;
    }
    w = (w & ~(0x3ff << sh)) | ((x | (y << 5)) << sh);
    st->w = w;
}

static void mars_step(const or_model *M, or_state *st, int a, uint32_t seed, uint32_t step,
                      uint32_t id, uint32_t depth, float *r, uint64_t *z)
{
    *r = 0.0f;
    *z = OBS_NONE;
    if (st->term) return; /* terminal states are absorbing */
    int per = 5 + M->m;
    uint32_t u[4];
    draw_block(seed, step, id, depth, 0, TAG_STEP, u);
    float r1, r2;
    int z1, z2;
    mars_robot(M, st, 0, a / per, u[0], &r1, &z1);
    mars_robot(M, st, 1, a % per, u[1], &r2, &z2);
    *r = r1 + r2;
    *z = (uint64_t)(3 * z1 + z2);
    if (((st->w >> MARS_GONE0) & 3) == 3) {
        st->term = 1;
        st->w |= 1 << MARS_TERM;
    }
}

/* Optimistic value: every good rock sampled by the nearer robot still on
 * the map on arrival at the shortest path length, plus each such robot's
 * exit reward at its shortest exit time. */
static double mars_upper(const or_model *M, const or_state *st)
{
    if (st->term) return 0.0;
    double u = 0.0;
    for (int i = 0; i < M->m; i++) {
        if (!((st->w2 >> i) & 1)) continue;
        int best = -1;
        for (int j = 0; j < 2; j++) {
            if ((st->w >> (MARS_GONE0 + j)) & 1) continue;
            int x = (st->w >> (10 * j)) & 31, y = (st->w >> (10 * j + 5)) & 31;
            int d = abs(x - M->rock_x[i]) + abs(y - M->rock_y[i]);
            if (best < 0 || d < best) best = d;
        }
        u += 10.0 * pow(M->gamma, best);
    }
    for (int j = 0; j < 2; j++)
        if (!((st->w >> (MARS_GONE0 + j)) & 1))
            u += 10.0 * pow(M->gamma, M->n - 1 - ((st->w >> (10 * j)) & 31));
    return u;
}

/* --- Navigation in a partially known map (Sec. IV-A): an n x n grid
 *     (13 x 13 in the paper), row 0 at the top.  Cells are known free,
 *     known walls, or unknown (occupied or not in each scenario; the two
 *     gates of the middle wall are unknown cells of which exactly one is
 *     open).  State: robot row word = x in bits 0-3, y in bits 4-7,
 *     terminal in bit 30; then four words of unknown-cell occupancy.
 *     Actions: 0 stay, 1-8 move to a neighbour N, NE, E, SE, S, SW, W, NW
 *     (y grows downwards).  Readings: a move fails (the robot stays) when
 *     word 0 of step block 0 is below the failure threshold, and still
 *     costs the motion cost; moving into a wall, an occupied cell or off
 *     the map is a crash (robot stays, -1); entering the goal pays +20
 *     instead of the motion cost and ends the episode; staying costs -0.2;
 *     every other move -0.1.  Observation: one bit per neighbour (in action
 *     order) after the step, 1 = occupied (off the map reads occupied),
 *     neighbour j's bit flipped when word j%4 of step block 1 + j/4 is below
 *     the sensor-error threshold; a terminal state observes 256. */
#define NAV_TERM 30
#define NAV_OBS_TERMINAL 256u
static const int NAV_DX[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const int NAV_DY[9] = {0, -1, -1, 0, 1, 1, 1, 0, -1};

/* Occupied in this scenario (off the map counts as occupied). */
static int nav_occupied(const or_model *M, const or_state *st, int x, int y)
{
    if (x < 0 || y < 0 || x >= M->n || y >= M->n) return 1;
    int c = M->nav_cell[y * M->n + x];
    if (c == -1) return 0;
    if (c == -2) return 1;
    return (st->nw[c / 32] >> (c % 32)) & 1;
}

static void nav_step(const or_model *M, or_state *st, int a, uint32_t seed, uint32_t step,
                     uint32_t id, uint32_t depth, float *r, uint64_t *z)
{
    *r = 0.0f;
    *z = NAV_OBS_TERMINAL;
    if (st->term) return; /* terminal states are absorbing */
    int x = st->w & 15, y = (st->w >> 4) & 15;
    uint32_t u[4];
    draw_block(seed, step, id, depth, 0, TAG_STEP, u);
    if (a == 0) {
        *r = -0.2f;
    } else if ((uint64_t)u[0] < prob_threshold(M->p_fail)) {
        *r = -0.1f; /* the move fails: the robot stays */
    } else {
        int tx = x + NAV_DX[a], ty = y + NAV_DY[a];
        if (nav_occupied(M, st, tx, ty)) {
            *r = -1.0f; /* crash: the robot stays */
        } else {
            x = tx;
            y = ty;
            if (x == M->nav_goal_x && y == M->n - 1) {
                *r = 20.0f;
                st->term = 1;
            } else {
                *r = -0.1f;
            }
        }
    }
    st->w = x | (y << 4) | (st->term ? 1 << NAV_TERM : 0);
    if (st->term) return; /* the world ends: no reading */
    uint32_t v[8];
    draw_block(seed, step, id, depth, 1, TAG_STEP, v);
    draw_block(seed, step, id, depth, 2, TAG_STEP, v + 4);
    uint64_t obs = 0;
    for (int j = 0; j < 8; j++) {
        int bit = nav_occupied(M, st, x + NAV_DX[j + 1], y + NAV_DY[j + 1]);
        if ((uint64_t)v[j] < prob_threshold(M->p_err)) bit = !bit;
        obs |= (uint64_t)bit << j;
    }
    *z = obs;
}

/* Optimistic value: the goal reward on the shortest path (Chebyshev
 * distance d in 8-connected moves, reward on the d-th move, at step d-1),
 * no costs. */
static double nav_upper(const or_model *M, const or_state *st)
{
    if (st->term) return 0.0;
    int x = st->w & 15, y = (st->w >> 4) & 15;
    int dx = abs(x - M->nav_goal_x), dy = abs(y - (M->n - 1));
    int d = dx > dy ? dx : dy;
    /* +20 is paid on entering the goal: from the goal cell itself (a state no
     * step produces, since entering is terminal) the soonest is to leave and
     * re-enter, two moves, so the bound is 20 gamma there */
    return 20.0 * pow(M->gamma, d > 0 ? d - 1 : 1);
}

/* Default policy: head for the open gate while above the wall, then for the
 * goal; take the diagonal step towards the target, else its vertical, else
 * its horizontal part, whichever lands on a free cell; else stay. */
static int nav_default_action(const or_model *M, const or_state *st)
{
    int x = st->w & 15, y = (st->w >> 4) & 15;
    int tx = M->nav_goal_x, ty = M->n - 1;
    if (y < M->nav_wall) {
        int g = ((st->nw[0] >> 0) & 1) == 0 ? 0 : (((st->nw[0] >> 1) & 1) == 0 ? 1 : -1);
        if (g >= 0) {
            tx = M->nav_gate_x[g];
            ty = M->nav_wall;
        }
    }
    int sx = tx > x ? 1 : (tx < x ? -1 : 0), sy = ty > y ? 1 : (ty < y ? -1 : 0);
    int cand[3][2] = {{sx, sy}, {0, sy}, {sx, 0}};
    for (int c = 0; c < 3; c++) {
        int dx = cand[c][0], dy = cand[c][1];
        if (dx == 0 && dy == 0) continue;
        if (nav_occupied(M, st, x + dx, y + dy)) continue;
        for (int a = 1; a < 9; a++)
            if (NAV_DX[a] == dx && NAV_DY[a] == dy) return a;
    }
    return 0;
}

/* --- Crowd driving: a car along a straight path among pedestrians walking
 *     to hidden goals with noisy headings; accelerate/decelerate fail with a
 *     small probability (Sec. IV-A).  Actions 0 accelerate, 1 maintain,
 *     2 decelerate.  Speed = 0.5 m/s per level. */
#define PED_OBS_TERMINAL 0xFFFFFFFFFFFFFFFFull

static uint64_t mix64(uint64_t x) /* splitmix64 output function (Steele, Lea, Flood 2014) */
{
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t hash_field(uint64_t h, int32_t f)
{
    return mix64((h ^ (uint64_t)(uint32_t)f) + 0x9E3779B97F4A7C15ull);
}

/* Observation: speed level and every pedestrian's position floored to whole
 * metres, hashed field by field; the hash value is the observation. */
static uint64_t ped_observe(const or_model *M, const or_state *st)
{
    if (st->term) return PED_OBS_TERMINAL;
    uint64_t h = 0x243F6A8885A308D3ull;
    h = hash_field(h, st->level);
    for (int j = 0; j < M->n_peds; j++) {
        h = hash_field(h, (int32_t)floorf(st->px[j]));
        h = hash_field(h, (int32_t)floorf(st->py[j]));
    }
    if (h == PED_OBS_TERMINAL) h = PED_OBS_TERMINAL - 1;
    return h;
}

/* Gaussian draw as the Irwin-Hall sum of four 24-bit uniforms, standardised. */
static float ped_gauss(const uint32_t u[4])
{
    int32_t sum = (int32_t)((u[0] >> 8) + (u[1] >> 8) + (u[2] >> 8) + (u[3] >> 8));
    float scale = (float)(sqrt(3.0) / 16777216.0);
    return (float)(sum - 33554430) * scale;
}

static void ped_step(const or_model *M, or_state *st, int a, uint32_t seed, uint32_t step,
                     uint32_t id, uint32_t depth, float *r, uint64_t *z)
{
    if (st->term) {
        *r = 0.0f;
        *z = PED_OBS_TERMINAL;
        return;
    }
    uint32_t u[4];
    draw_block(seed, step, id, depth, 0, TAG_STEP, u);
    int failed = (uint64_t)u[0] < prob_threshold(M->p_fail);
    int level = st->level;
    if (a == 0 && !failed && level < M->n_levels - 1) level = level + 1;
    if (a == 2 && !failed && level > 0) level = level - 1;
    float v = 0.5f * (float)level;
    float s_next = st->s + v * M->dt;

    float step_len = M->ped_speed * M->dt;
    float half_sigma = 0.5f * M->sigma_h;
    for (int j = 0; j < M->n_peds; j++) {
        draw_block(seed, step, id, depth, (uint32_t)(j + 1), TAG_STEP, u);
        float noise = ped_gauss(u);
        float gx = M->goal_x[st->goal[j]], gy = M->goal_y[st->goal[j]];
        float dx = gx - st->px[j];
        float dy = gy - st->py[j];
        float dist = sqrtf(dx * dx + dy * dy);
        if (dist <= step_len) {
            st->px[j] = gx; /* arrives at its goal and stays there */
            st->py[j] = gy;
        } else {
            float ux = dx / dist, uy = dy / dist;
            /* heading noise as a rotation written with the tangent of the
             * half angle t: cos = (1-t^2)/(1+t^2), sin = 2t/(1+t^2) */
            float t = half_sigma * noise;
            float t2 = t * t;
            float den = 1.0f + t2;
            float c = (1.0f - t2) / den;
            float sn = (2.0f * t) / den;
            float rx = ux * c - uy * sn;
            float ry = ux * sn + uy * c;
            st->px[j] = st->px[j] + step_len * rx;
            st->py[j] = st->py[j] + step_len * ry;
        }
    }

    int collided = 0;
    if (level > 0) {
        float r2 = M->coll_radius * M->coll_radius;
        for (int j = 0; j < M->n_peds; j++) {
            float ddx = st->px[j] - s_next;
            float d2 = ddx * ddx + st->py[j] * st->py[j];
            if (d2 < r2) collided = 1;
        }
    }
    float reward = M->r_step;
    if (collided) {
        reward = M->r_step + M->r_collision;
        st->term = 1;
    } else if (s_next >= M->path_len) {
        reward = M->r_step + M->r_goal;
        st->term = 1;
    }
    st->s = s_next;
    st->level = level;
    *r = reward;
    *z = ped_observe(M, st);
}

/* Optimistic value: the goal reward at the earliest possible arrival time. */
static double ped_upper(const or_model *M, const or_state *st)
{
    if (st->term) return 0.0;
    float reach = (0.5f * (float)(M->n_levels - 1)) * M->dt;
    float T = ceilf((M->path_len - st->s) / reach);
    int Ti = (int)T;
    if (Ti < 1) Ti = 1;
    return (double)M->r_goal * pow(M->gamma, Ti - 1);
}

/* Default policy of the crowd-driving task: brake when a pedestrian is in a
 * short corridor ahead, otherwise speed up. */
static int ped_default_action(const or_model *M, const or_state *st)
{
    for (int j = 0; j < M->n_peds; j++) {
        float ahead = st->px[j] - st->s;
        if (ahead >= 0.0f && ahead <= 3.0f && fabsf(st->py[j]) < 1.5f) return 2;
    }
    return 0;
}

/* One step of the deterministic simulative model s', r, z = g(s, a, phi). */
static void model_step(const or_model *M, or_state *st, int a, uint32_t seed, uint32_t step,
                       uint32_t id, uint32_t depth, float *r, uint64_t *z)
{
    if (M->kind == 0)
        rs_step(M, st, a, seed, step, id, depth, r, z);
    else if (M->kind == 2)
        mars_step(M, st, a, seed, step, id, depth, r, z);
    else if (M->kind == 3)
        nav_step(M, st, a, seed, step, id, depth, r, z);
    else
        ped_step(M, st, a, seed, step, id, depth, r, z);
}

static double model_upper(const or_model *M, const or_state *st)
{
    if (M->kind == 2) return mars_upper(M, st);
    if (M->kind == 3) return nav_upper(M, st);
    return M->kind == 0 ? rs_upper(M, st) : ped_upper(M, st);
}

static int policy_action(const or_model *M, const or_rollout_cfg *C, const or_state *st,
                         uint32_t seed, uint32_t step, uint32_t id, uint32_t depth)
{
    if (C->policy == 1) return C->const_action;
    if (C->policy == 2) {
        uint32_t u[4];
        draw_block(seed, step, id, depth, 0, TAG_POLICY, u);
        return (int)(u[0] % (uint32_t)M->n_actions);
    }
    if (M->kind == 2) return RS_EAST * (5 + M->m) + RS_EAST; /* both robots move east */
    if (M->kind == 3) return nav_default_action(M, st);
    return M->kind == 0 ? RS_EAST : ped_default_action(M, st);
}

/* Default-policy rollout from depth d0 (Eq. 13): discounted from d0, stopped
 * at a terminal state or after min(R, D - d0) steps; the tail heuristic past
 * the horizon is 0. */
static double rollout(const or_model *M, const or_rollout_cfg *C, or_state st, uint32_t seed,
                      uint32_t step, uint32_t id, int d0, int64_t *steps, double *abs_sum)
{
    double mag = 0.0;
    int n_roll = C->max_steps;
    if (C->max_depth >= 0 && C->max_depth - d0 < n_roll) n_roll = C->max_depth - d0;
    double value = 0.0;
    for (int j = 0; j < n_roll; j++) {
        if (st.term) break;
        int a = policy_action(M, C, &st, seed, step, id, (uint32_t)(d0 + j));
        float r;
        uint64_t z;
        model_step(M, &st, a, seed, step, id, (uint32_t)(d0 + j), &r, &z);
        value += pow(M->gamma, j) * (double)r;
        mag += pow(M->gamma, j) * fabs((double)r);
        *steps += 1;
    }
    if (abs_sum) *abs_sum = mag;
    return value;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

/* Apply g to each state of an array with one action (for tests). */
void or_step_batch(const or_model *M, const or_soa *in, const uint32_t *ids, int64_t n,
                   int32_t action, int32_t depth, uint32_t seed, uint32_t step,
                   const or_soa *out, float *r, uint64_t *z)
{
    or_state st;
    for (int64_t k = 0; k < n; k++) {
        load_state(M, in, k, &st);
        model_step(M, &st, action, seed, step, ids[k], (uint32_t)depth, &r[k], &z[k]);
        store_state(M, out, k, &st);
    }
}

/* Draw K start states from the belief (Sec. III-A): scenario k uses counter
 * (k, 0, block, INIT).  RockSample: known cell, rock i good with
 * probability p[i] (word i%4 of block i/4).  Multi-agent RockSample: x0 is
 * the known robots' row, the rocks drawn as for RockSample.  Navigation:
 * draw k = word k%4 of block k/4; the robot on row 0 at column
 * floor(draw0 * n / 2^32); gate 0 open (unknown cell 0 free, cell 1
 * occupied) iff draw1 < 2^31, else the reverse; unknown cell i >= 2
 * occupied iff draw i is below the threshold of p[i].  Crowd driving: known car and
 * pedestrian positions, pedestrian j's goal drawn from goal_p[j][.]. */
void or_sample_scenarios(const or_model *M, int32_t K, uint32_t seed, uint32_t step,
                         int32_t x0, int32_t y0, const double *p_good,
                         float s0, int32_t level0, const float *px0, const float *py0,
                         const double *goal_p, const or_soa *out)
{
    for (int32_t k = 0; k < K; k++) {
        or_state st;
        memset(&st, 0, sizeof(st));
        if (M->kind == 0) {
            int32_t w = x0 | (y0 << 5);
            for (int i = 0; i < M->m; i++) {
                uint32_t u[4];
                draw_block(seed, step, (uint32_t)k, 0, (uint32_t)(i / 4), TAG_INIT, u);
                if ((uint64_t)u[i % 4] < prob_threshold(p_good[i])) w |= 1 << (10 + i);
            }
            st.w = w;
        } else if (M->kind == 3) {
            uint32_t u[4];
            int nu = 0;
            for (int c = 0; c < M->n * M->n; c++)
                if (M->nav_cell[c] >= 0) nu++;
            draw_block(seed, step, (uint32_t)k, 0, 0, TAG_INIT, u);
            int x = (int)(((uint64_t)u[0] * (uint64_t)M->n) >> 32);
            st.w = x;
            if (u[1] < 0x80000000u)
                st.nw[0] |= 2; /* gate 0 open, gate 1 closed */
            else
                st.nw[0] |= 1;
            for (int i = 2; i < nu; i++) {
                if (i % 4 == 0) draw_block(seed, step, (uint32_t)k, 0, (uint32_t)(i / 4), TAG_INIT, u);
                if ((uint64_t)u[i % 4] < prob_threshold(p_good[i])) st.nw[i / 32] |= 1 << (i % 32);
            }
        } else if (M->kind == 2) {
            st.w = x0;
            st.term = (x0 >> MARS_TERM) & 1;
            for (int i = 0; i < M->m; i++) {
                uint32_t u[4];
                draw_block(seed, step, (uint32_t)k, 0, (uint32_t)(i / 4), TAG_INIT, u);
                if ((uint64_t)u[i % 4] < prob_threshold(p_good[i])) st.w2 |= 1 << i;
            }
        } else {
            st.s = s0;
            st.level = level0;
            for (int j = 0; j < M->n_peds; j++) {
                uint32_t u[4];
                draw_block(seed, step, (uint32_t)k, 0, (uint32_t)(j / 4), TAG_INIT, u);
                int g = M->n_goals - 1;
                double cum = 0.0;
                for (int q = 0; q < M->n_goals - 1; q++) {
                    cum += goal_p[j * M->n_goals + q];
                    if ((uint64_t)u[j % 4] < prob_threshold(cum)) {
                        g = q;
                        break;
                    }
                }
                st.px[j] = px0[j];
                st.py[j] = py0[j];
                st.goal[j] = (uint8_t)g;
            }
        }
        store_state(M, out, k, &st);
    }
}

/* Upper bound and rollout lower bound for each state of an array. */
void or_rollout_bounds(const or_model *M, const or_rollout_cfg *C, uint32_t seed, uint32_t step,
                       const or_soa *in, const uint32_t *ids, const int32_t *depths, int64_t n,
                       double *U, double *L, int64_t *steps, double *Labs)
{
    for (int64_t k = 0; k < n; k++) {
        or_state st;
        load_state(M, in, k, &st);
        int64_t cnt = 0;
        U[k] = model_upper(M, &st);
        L[k] = rollout(M, C, st, seed, step, ids[k], depths[k], &cnt, Labs ? &Labs[k] : NULL);
        steps[k] = cnt;
    }
}

typedef struct {
    uint64_t z;
    int32_t k;
} zk_pair;

static int cmp_zk(const void *a, const void *b)
{
    const zk_pair *p = (const zk_pair *)a, *q = (const zk_pair *)b;
    if (p->z != q->z) return p->z < q->z ? -1 : 1;
    return p->k < q->k ? -1 : (p->k > q->k);
}

/* Outputs of one leaf expansion; NULL members are not written. */
typedef struct {
    or_soa states;      /* the leaf's own states after the update step */
    uint32_t *ids;      /* [n] scenario ids */
    or_soa sprime;      /* [A][n] stepped states (row stride A*n for peds) */
    float *r;           /* [A][n] step rewards */
    uint64_t *z;        /* [A][n] observations */
    double *U, *L;      /* [A][n] per-scenario bounds */
    double *Labs;       /* [A][n] sum of |discounted rollout terms| (tolerance scale) */
    int32_t *child_of;  /* [A][n] child index of each scenario */
    int32_t *perm;      /* [A][n] leaf positions grouped by child */
    int32_t *n_children;/* [A] */
    uint64_t *child_z;  /* [A][cap] */
    int32_t *child_n, *child_off; /* [A][cap] */
    double *child_u0, *child_l0;  /* [A][cap] */
    double *r_mean;     /* [A] */
    int64_t *expand_steps, *rollout_steps; /* scalars */
    int64_t *steps;     /* [A][2] per action: expansion steps, rollout steps */
} or_expand_out;

/* Leaf expansion (Sec. III-D): gather the leaf's scenarios from its parent by
 * position, update them with the last action at depth-1 (none at the root),
 * expand every action at the leaf's depth (Eq. 10), group by observation
 * (Eq. 11), and set each child's initial bounds (Eq. 12, 13).
 * Children of an action come in ascending observation order; a child's
 * scenarios in ascending leaf position.  Returns 0, or -1 if an action has
 * more children than cap. */
int or_expand_leaf(const or_model *M, const or_rollout_cfg *C, uint32_t seed, uint32_t step,
                   const or_soa *parent, const uint32_t *parent_ids, const int32_t *idx,
                   int32_t n, int32_t depth, int32_t last_action, int32_t cap,
                   const or_expand_out *out)
{
    int A = M->n_actions;
    or_state *leaf = (or_state *)malloc(sizeof(or_state) * (n > 0 ? n : 1));
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    zk_pair *pairs = (zk_pair *)malloc(sizeof(zk_pair) * (n > 0 ? n : 1));
    double *U = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *L = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    uint64_t *ch_z = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    int32_t *ch_off = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ch_n = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    double *ch_u = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *ch_l = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    int status = 0;
    int64_t exp_steps = 0, roll_steps = 0;

    for (int32_t k = 0; k < n; k++) {
        load_state(M, parent, idx[k], &leaf[k]);
        ids[k] = parent_ids[idx[k]];
        if (last_action >= 0) {
            float r;
            uint64_t z;
            model_step(M, &leaf[k], last_action, seed, step, ids[k], (uint32_t)(depth - 1), &r, &z);
        }
        if (out->states.w || out->states.s) store_state(M, &out->states, k, &leaf[k]);
        if (out->ids) out->ids[k] = ids[k];
    }

    for (int a = 0; a < A; a++) {
        double r_sum = 0.0;
        int64_t a_exp = 0, a_roll = 0;
        for (int32_t k = 0; k < n; k++) {
            or_state st = leaf[k];
            float r;
            uint64_t z;
            if (!leaf[k].term) a_exp += 1;
            model_step(M, &st, a, seed, step, ids[k], (uint32_t)depth, &r, &z);
            r_sum += (double)r;
            U[k] = model_upper(M, &st);
            double mag = 0.0;
            L[k] = rollout(M, C, st, seed, step, ids[k], depth + 1, &a_roll, &mag);
            pairs[k].z = z;
            pairs[k].k = k;
            int64_t pk = (int64_t)a * n + k;
            if (out->sprime.w || out->sprime.s) store_state(M, &out->sprime, pk, &st);
            if (out->r) out->r[pk] = r;
            if (out->z) out->z[pk] = z;
            if (out->U) out->U[pk] = U[k];
            if (out->L) out->L[pk] = L[k];
            if (out->Labs) out->Labs[pk] = mag;
        }
        if (out->r_mean) out->r_mean[a] = n > 0 ? r_sum / n : 0.0;
        /* step counts (model steps on non-terminal states) of this action */
        exp_steps += a_exp;
        roll_steps += a_roll;
        if (out->steps) {
            out->steps[2 * a] = a_exp;
            out->steps[2 * a + 1] = a_roll;
        }

        /* Eq. 11: one child per distinct observation; a stable sort keeps
         * each child's scenarios in ascending leaf position. */
        qsort(pairs, (size_t)n, sizeof(zk_pair), cmp_zk);
        int c = -1;
        for (int32_t i = 0; i < n; i++) {
            if (i == 0 || pairs[i].z != pairs[i - 1].z) {
                c += 1;
                ch_z[c] = pairs[i].z;
                ch_off[c] = i;
                ch_n[c] = 0;
                ch_u[c] = 0.0;
                ch_l[c] = 0.0;
            }
            int k = pairs[i].k;
            ch_n[c] += 1;
            ch_u[c] += U[k];
            ch_l[c] += L[k];
            if (out->perm) out->perm[(int64_t)a * n + i] = k;
            if (out->child_of) out->child_of[(int64_t)a * n + k] = c;
        }
        int n_ch = c + 1;
        if (out->n_children) out->n_children[a] = n_ch;
        if (n_ch > cap) status = -1;
        for (int q = 0; q < n_ch && q < cap; q++) {
            int64_t o = (int64_t)a * cap + q;
            if (out->child_z) out->child_z[o] = ch_z[q];
            if (out->child_off) out->child_off[o] = ch_off[q];
            if (out->child_n) out->child_n[o] = ch_n[q];
            /* Eq. 12 and 13: plain means over the child's scenarios */
            if (out->child_u0) out->child_u0[o] = ch_u[q] / ch_n[q];
            if (out->child_l0) out->child_l0[o] = ch_l[q] / ch_n[q];
        }
    }
    if (out->expand_steps) *out->expand_steps = exp_steps;
    if (out->rollout_steps) *out->rollout_steps = roll_steps;
    free(leaf);
    free(ids);
    free(pairs);
    free(U);
    free(L);
    free(ch_z);
    free(ch_off);
    free(ch_n);
    free(ch_u);
    free(ch_l);
    return status;
}

/* The observation hash's mixing function, exposed so the tests can check it
 * against the published splitmix64 generator. */
uint64_t or_mix64(uint64_t x) { return mix64(x); }

/* Sensor threshold table, exposed so the tests can check the accuracy law. */
uint64_t or_rs_sense_threshold(int32_t d2) { return rs_sense_threshold(d2); }

/* ------------------------------------------------------------------------ */
/* The DESPOT trial loop on one host thread (Sec. III-A), the baseline the  */
/* paper's speedups are quoted against, built on the expansion above: each   */
/* trial descends from the root taking the action of largest upper bound    */
/* (Eq. 5) and the observation child of largest weighted excess uncertainty */
/* E = (u - l) - (|Phi_c| / K) xi (u(b0) - l(b0)) (Eq. 6, 7), stops where E  */
/* is not positive, expands the leaf it reaches above the depth limit and   */
/* backs the path up (Eq. 4).  Ties go to the lowest action index and the   */
/* first child in observation order.  Values FP64.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t parent, action, n, depth;
    double u, l;
    int32_t src;           /* record whose states and ids this node's positions index */
    const int32_t *pos;    /* [n] positions in that record */
    int32_t act_begin;     /* first action branch; -1 until expanded */
} dn_node;

typedef struct {
    double r;
    int32_t child_begin, n_children;
} dn_act;

typedef struct {
    or_soa states;
    uint32_t *ids;
    int32_t *perm; /* [A][n] */
    void *buf;     /* the record's one allocation */
} dn_rec;

typedef struct {
    int64_t nodes, trials, expansions, scenario_steps;
    double u_root, l_root, elapsed_s;
    int32_t max_depth_reached;
    int32_t near_ties; /* choices whose runner-up was within 1e-6 (relative) but not equal */
} or_despot_result;

/* a choice decided by less than FP32 resolution of the values compared */
static int dn_near(double best, double second)
{
    if (!(second > -INFINITY) || best == second) return 0;
    return best - second <= 1e-6 * fmax(fabs(best), 1.0);
}

static double dn_now(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* A record of n scenarios: states in the library's layout, ids, grouped order. */
static int dn_rec_alloc(const or_model *M, int32_t n, dn_rec *r)
{
    const int64_t A = M->n_actions, nn = n > 0 ? n : 1;
    int64_t words = 0, fl = 0, bytes8 = 0;
    if (M->kind == 0) words = nn;
    else if (M->kind == 2) words = 2 * nn;
    else if (M->kind == 3) words = 5 * nn;
    else {
        words = nn;                      /* car */
        fl = nn * (1 + 2 * M->n_peds);   /* s, px, py */
        bytes8 = nn * M->n_peds;         /* goal */
    }
    size_t total = sizeof(int32_t) * (size_t)(words + nn + A * nn) + sizeof(float) * (size_t)fl + (size_t)bytes8 + 64;
    char *b = (char *)calloc(1, total);
    if (!b) return -1;
    memset(r, 0, sizeof(*r));
    r->buf = b;
    int32_t *wp = (int32_t *)b;
    r->ids = (uint32_t *)(wp + words);
    r->perm = (int32_t *)(r->ids + nn);
    float *fp = (float *)(r->perm + A * nn);
    if (M->kind == 1) {
        r->states.car = wp;
        r->states.s = fp;
        r->states.px = fp + nn;
        r->states.py = fp + nn + nn * M->n_peds;
        r->states.goal = (uint8_t *)(fp + fl);
    } else {
        r->states.w = wp;
    }
    r->states.stride = n;
    return 0;
}

#define DN_GROW(ptr, cnt, cap, type)                                              \
    do {                                                                           \
        if ((cnt) >= (cap)) {                                                      \
            int64_t nc_ = (cap) ? 2 * (cap) : 1024;                                \
            type *np_ = (type *)realloc((ptr), sizeof(type) * (size_t)nc_);        \
            if (!np_) { status = -1; goto done; }                                  \
            (ptr) = np_;                                                           \
            (cap) = nc_;                                                           \
        }                                                                          \
    } while (0)

/* Eq. 4 at one expanded node from its branches and children */
static void dn_bellman(const or_model *M, dn_node *nodes, const dn_act *acts, int32_t b)
{
    double bu = -INFINITY, bl = -INFINITY;
    for (int a = 0; a < M->n_actions; a++) {
        const dn_act *x = &acts[nodes[b].act_begin + a];
        double su = 0.0, sl = 0.0;
        for (int c = 0; c < x->n_children; c++) {
            const dn_node *k = &nodes[x->child_begin + c];
            const double w = (double)k->n / (double)nodes[b].n;
            su += w * k->u;
            sl += w * k->l;
        }
        if (x->r + M->gamma * su > bu) bu = x->r + M->gamma * su;
        if (x->r + M->gamma * sl > bl) bl = x->r + M->gamma * sl;
    }
    nodes[b].u = bu;
    nodes[b].l = bl;
}

/* One planning step from K root scenarios (states `root`, ids 0..K-1): trials
 * until `seconds` of wall time pass, max_trials trials (if > 0), or the
 * root's gap closes.  Returns 0, or -1 when memory runs out. */
int or_despot(const or_model *M, const or_rollout_cfg *C, uint32_t seed, uint32_t step, const or_soa *root,
              int32_t K, int32_t max_depth, double xi, double seconds, int64_t max_trials, or_despot_result *res)
{
    const int A = M->n_actions;
    int status = 0;
    dn_node *nodes = NULL;
    dn_act *acts = NULL;
    dn_rec *recs = NULL;
    int32_t *path = NULL, *iota = NULL;
    int64_t n_nodes = 0, cap_nodes = 0, n_acts = 0, cap_acts = 0, n_recs = 0, cap_recs = 0, cap_path = 0;
    double *U = NULL, *L = NULL, *cu = NULL, *cl = NULL, *rm = NULL;
    int64_t *st = NULL, *steps = NULL;
    int32_t *depths = NULL, *nch = NULL, *cn = NULL, *coff = NULL;
    uint64_t *cz = NULL;
    memset(res, 0, sizeof(*res));
    const double t0 = dn_now();

    /* the root record: the sampled states, ids 0..K-1 */
    DN_GROW(recs, n_recs, cap_recs, dn_rec);
    if (dn_rec_alloc(M, K, &recs[0]) != 0) { status = -1; goto done; }
    n_recs = 1;
    iota = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    U = (double *)malloc(sizeof(double) * (size_t)K);
    L = (double *)malloc(sizeof(double) * (size_t)K);
    st = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    depths = (int32_t *)calloc((size_t)K, sizeof(int32_t));
    if (!iota || !U || !L || !st || !depths) { status = -1; goto done; }
    for (int32_t k = 0; k < K; k++) {
        or_state s;
        load_state(M, root, k, &s);
        store_state(M, &recs[0].states, k, &s);
        recs[0].ids[k] = (uint32_t)k;
        iota[k] = k;
    }
    or_rollout_bounds(M, C, seed, step, &recs[0].states, recs[0].ids, depths, K, U, L, st, NULL);
    {
        double su = 0.0, sl = 0.0;
        for (int32_t k = 0; k < K; k++) {
            su += U[k];
            sl += L[k];
            res->scenario_steps += st[k];
        }
        DN_GROW(nodes, n_nodes, cap_nodes, dn_node);
        dn_node r0 = {-1, -1, K, 0, su / K, sl / K, 0, iota, -1};
        nodes[n_nodes++] = r0;
    }
    /* per-expansion outputs, sized for the root (the largest node) */
    {
        const int32_t cap = K;
        nch = (int32_t *)malloc(sizeof(int32_t) * A);
        rm = (double *)malloc(sizeof(double) * A);
        steps = (int64_t *)malloc(sizeof(int64_t) * 2 * A);
        cz = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)A * cap);
        cn = (int32_t *)malloc(sizeof(int32_t) * (size_t)A * cap);
        coff = (int32_t *)malloc(sizeof(int32_t) * (size_t)A * cap);
        cu = (double *)malloc(sizeof(double) * (size_t)A * cap);
        cl = (double *)malloc(sizeof(double) * (size_t)A * cap);
        if (!nch || !rm || !steps || !cz || !cn || !coff || !cu || !cl) { status = -1; goto done; }
    }

    for (;;) {
        if (dn_now() - t0 >= seconds) break;
        if (max_trials > 0 && res->trials >= max_trials) break;
        const double gap0 = nodes[0].u - nodes[0].l;
        if (gap0 <= 0.0) break;
        /* descend: Eq. 5 then Eq. 7 */
        int64_t depth_n = 0;
        int32_t b = 0;
        int ended = 0; /* the path ended at a node without a positive-E child */
        DN_GROW(path, depth_n, cap_path, int32_t);
        path[depth_n++] = 0;
        while (nodes[b].act_begin >= 0) {
            int best_a = 0;
            double best_v = -INFINITY, second_v = -INFINITY;
            for (int a = 0; a < A; a++) {
                const dn_act *x = &acts[nodes[b].act_begin + a];
                double s = 0.0;
                for (int c = 0; c < x->n_children; c++) {
                    const dn_node *k = &nodes[x->child_begin + c];
                    s += (double)k->n / (double)nodes[b].n * k->u;
                }
                const double v = x->r + M->gamma * s;
                if (v > best_v) {
                    second_v = best_v;
                    best_v = v;
                    best_a = a;
                } else if (v > second_v) {
                    second_v = v;
                }
            }
            res->near_ties += dn_near(best_v, second_v);
            const dn_act *x = &acts[nodes[b].act_begin + best_a];
            int32_t best = -1;
            double best_e = -INFINITY, second_e = -INFINITY;
            for (int c = 0; c < x->n_children; c++) {
                const dn_node *k = &nodes[x->child_begin + c];
                const double e = (k->u - k->l) - (double)k->n / (double)K * xi * gap0;
                if (e > best_e) {
                    second_e = best_e;
                    best_e = e;
                    best = x->child_begin + c;
                } else if (e > second_e) {
                    second_e = e;
                }
            }
            res->near_ties += dn_near(best_e, second_e) + dn_near(best_e, 0.0);
            if (best < 0 || best_e <= 0.0) {
                ended = 1;
                break;
            }
            b = best;
            DN_GROW(path, depth_n, cap_path, int32_t);
            path[depth_n++] = b;
        }
        res->trials += 1;
        if (ended) break; /* nothing below the root would change: the step is over */
        if (nodes[b].depth >= max_depth || nodes[b].n == 0) continue;
        /* expand the leaf (Sec. III-D) into a new record */
        DN_GROW(recs, n_recs, cap_recs, dn_rec);
        const int32_t rid = (int32_t)n_recs;
        dn_node leaf = nodes[b];
        if (dn_rec_alloc(M, leaf.n, &recs[rid]) != 0) { status = -1; goto done; }
        n_recs += 1;
        or_expand_out o;
        memset(&o, 0, sizeof(o));
        int64_t es = 0, rs = 0;
        o.states = recs[rid].states;
        o.ids = recs[rid].ids;
        o.perm = recs[rid].perm;
        o.n_children = nch;
        o.child_z = cz;
        o.child_n = cn;
        o.child_off = coff;
        o.child_u0 = cu;
        o.child_l0 = cl;
        o.r_mean = rm;
        o.expand_steps = &es;
        o.rollout_steps = &rs;
        o.steps = steps;
        const int32_t cap = leaf.n;
        if (or_expand_leaf(M, C, seed, step, &recs[leaf.src].states, recs[leaf.src].ids, leaf.pos, leaf.n,
                           leaf.depth, leaf.action, cap, &o) != 0) { status = -1; goto done; }
        res->expansions += 1;
        res->scenario_steps += es + rs;
        /* attach the branches (Eq. 11) */
        nodes[b].act_begin = (int32_t)n_acts;
        for (int a = 0; a < A; a++) {
            DN_GROW(acts, n_acts, cap_acts, dn_act);
            dn_act x = {rm[a], (int32_t)n_nodes, nch[a]};
            acts[n_acts++] = x;
            for (int c = 0; c < nch[a]; c++) {
                DN_GROW(nodes, n_nodes, cap_nodes, dn_node);
                const int64_t o2 = (int64_t)a * cap + c;
                dn_node k = {b, a, cn[o2], leaf.depth + 1, cu[o2], cl[o2], rid,
                             recs[rid].perm + (int64_t)a * leaf.n + coff[o2], -1};
                nodes[n_nodes++] = k;
            }
        }
        if (leaf.depth + 1 > res->max_depth_reached) res->max_depth_reached = leaf.depth + 1;
        /* Eq. 4 along the path, leaf first */
        for (int64_t i = depth_n; i-- > 0;) dn_bellman(M, nodes, acts, path[i]);
    }

done:
    res->nodes = n_nodes;
    if (n_nodes > 0) {
        res->u_root = nodes[0].u;
        res->l_root = nodes[0].l;
    }
    res->elapsed_s = dn_now() - t0;
    for (int64_t i = 0; i < n_recs; i++) free(recs[i].buf);
    free(recs);
    free(nodes);
    free(acts);
    free(path);
    free(iota);
    free(U);
    free(L);
    free(st);
    free(depths);
    free(nch);
    free(rm);
    free(steps);
    free(cz);
    free(cn);
    free(coff);
    free(cu);
    free(cl);
    return status;
}
