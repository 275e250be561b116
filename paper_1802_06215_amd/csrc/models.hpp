// Device-side step functions of the two models and the Philox4x32-10 stream.
//
// The step function is the deterministic simulative model g of DESPOT
// (Sec. III-A): s', r, z = g(s, a, phi), where the scenario phi supplies the
// random numbers through a counter-based generator indexed by (scenario id,
// depth, block, tag).  State arithmetic of the driving model is FP32,
// compiled without contraction and with correctly rounded division and
// square root (plain "/" and __builtin_sqrtf under
// -fhip-fp32-correctly-rounded-divide-sqrt; HIP's __fsqrt_rn/__fdiv_rn are
// native approximations unless OCML_BASIC_ROUNDED_OPERATIONS is set), so the
// results are bit-identical to any IEEE-754 FP32 evaluation in the same
// operation order.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace hdx {

// Constant address space on the device (the host pass parses the same
// declarations without it).
#if defined(__HIP_DEVICE_COMPILE__)
#define HDX_CONST __attribute__((address_space(4)))
#else
#define HDX_CONST
#endif

// A model as the kernels see it: the header and the device tables through
// the constant address space (never written by a kernel, so uniform
// addresses become scalar loads), and the first kGpowLds discount powers
// in LDS for per-lane lookups.
struct MView {
    const HDX_CONST ModelHdr *h;
    const HDX_CONST uint32_t *thr;
    const HDX_CONST float *gg;
    const float *gl;
    const int16_t *cl;  // navigation cell table, staged in LDS after the goal points
    const uint8_t *up;  // navigation: grid bit of each unknown cell, staged after the cell table
    __device__ float gpow_uniform(int j) const { return gg[j]; }
    __device__ float gpow_lane(int j) const { return j < kGpowLds ? gl[j] : gg[j]; }
    // goal point coordinates, staged in LDS after the discount powers
    __device__ float goal_x(int g) const { return gl[kGpowLds + g]; }
    __device__ float goal_y(int g) const { return gl[kGpowLds + kMaxGoals + g]; }
};

__device__ __forceinline__ MView make_view(const DevModel *gm, const float *gpow_lds) {
    MView v;
    v.h = (const HDX_CONST ModelHdr *)&gm->h;
    v.thr = (const HDX_CONST uint32_t *)gm->sense_thr_m1;
    v.gg = (const HDX_CONST float *)gm->gpow;
    v.gl = gpow_lds;
    v.cl = (const int16_t *)(gpow_lds + kGpowLds + 2 * kMaxGoals);
    v.up = (const uint8_t *)(v.cl + HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID);
    return v;
}

__device__ __forceinline__ StatesPtr load_states(const HDX_CONST StatesPtr *s) {
    StatesPtr r;
    r.w = s->w;
    r.s = s->s;
    r.car = s->car;
    r.px = s->px;
    r.py = s->py;
    r.goal = s->goal;
    r.stride = s->stride;
    return r;
}

// Stage the first kGpowLds discount powers and the goal points of a model
// into LDS, and for navigation its cell table and the unknown cells' grid
// bits after them (kModelLdsFloats floats in all; the caller synchronises
// afterwards).
constexpr int kNavCells = HDX_MAX_NAV_GRID * HDX_MAX_NAV_GRID;
constexpr int kModelLdsFloats = kGpowLds + 2 * kMaxGoals + kNavCells / 2 + HDX_MAX_NAV_UNKNOWN / 4;
__device__ __forceinline__ void stage_gpow(const DevModel *gm, float *gpow_lds) {
    const HDX_CONST float *g = (const HDX_CONST float *)gm->gpow;
    const HDX_CONST ModelHdr *h = (const HDX_CONST ModelHdr *)&gm->h;
    for (int j = threadIdx.x; j < kGpowLds + 2 * kMaxGoals; j += blockDim.x) {
        float v;
        if (j < kGpowLds) v = g[j];
        else if (j < kGpowLds + kMaxGoals) v = h->goal_x[j - kGpowLds];
        else v = h->goal_y[j - kGpowLds - kMaxGoals];
        gpow_lds[j] = v;
    }
}
// The navigation cell table, after the goal points (navigation kernels only).
__device__ __forceinline__ void stage_cells(const DevModel *gm, float *gpow_lds) {
    const HDX_CONST ModelHdr *h = (const HDX_CONST ModelHdr *)&gm->h;
    int16_t *cells = (int16_t *)(gpow_lds + kGpowLds + 2 * kMaxGoals);
    for (int c = threadIdx.x; c < kNavCells; c += blockDim.x) cells[c] = h->nav_cell[c];
    uint8_t *pos = (uint8_t *)(cells + kNavCells);
    for (int c = threadIdx.x; c < HDX_MAX_NAV_UNKNOWN; c += blockDim.x) pos[c] = h->nav_unknown_pos[c];
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies, the key advanced by the Weyl increments in between.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 product each (a single v_mad_u64_u32 instead of
        // separate high and low multiplies)
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

struct RolloutParams {
    uint32_t k0, k1;
    int32_t policy, const_action, max_steps, max_depth, n_actions;
};

// Eq. 12 bound of the rock models from tabulated group sums: entry 16 g + m
// of `tab0` (groups 0-3) or `tab1` (group 4) is the sum of group g's good
// rocks' terms when the four quality bits of rocks 4g .. 4g+3 read m.  The
// five lookups are issued together and added in group order; a group past
// the last rock tabulates +0 for every pattern, and the running sum of
// non-negative terms is never -0, so the result equals the sum over the
// rock groups alone, bit for bit.  `bits` holds rock i's quality in bit i.
// Called by all 64 lanes of a wavefront.
__device__ __forceinline__ float group_table_sum(uint32_t bits, float tab0, float tab1) {
    const float t0 = __shfl(tab0, (int)__builtin_amdgcn_ubfe(bits, 0, 4), 64);
    const float t1 = __shfl(tab0, 16 + (int)__builtin_amdgcn_ubfe(bits, 4, 4), 64);
    const float t2 = __shfl(tab0, 32 + (int)__builtin_amdgcn_ubfe(bits, 8, 4), 64);
    const float t3 = __shfl(tab0, 48 + (int)__builtin_amdgcn_ubfe(bits, 12, 4), 64);
    const float t4 = __shfl(tab1, (int)__builtin_amdgcn_ubfe(bits, 16, 4), 64);
    return (((((0.0f + t0) + t1) + t2) + t3) + t4);
}

// ---------------------------------------------------------------------------
// RockSample: one packed int32 word per scenario.
// ---------------------------------------------------------------------------
struct RsOps {
    struct State {
        int32_t w;
    };
    static constexpr bool kHashObs = false;
    static constexpr bool kSplitRollout = true;  // small step: one rollout loop per policy
    static constexpr bool kSmallObs = true;       // observations 0 (none), 1, 2 (sensor readings)
    static constexpr bool kLdsModel = false;      // expansion reads no per-lane table from LDS
    static constexpr bool kWaveUpper = true;      // upper bound evaluated by whole wavefronts
    static constexpr bool kGroupRollout = false;  // one lane per scenario in rollouts

    __device__ static void load(const MView &, const StatesPtr &S, int64_t p, State &st) { st.w = S.w[p]; }
    __device__ static void make_terminal(State &st) { st.w = 1 << 30; }
    __device__ static void store(const MView &, const StatesPtr &S, int64_t p, const State &st) { S.w[p] = st.w; }
    __device__ static bool terminal(const State &st) { return (st.w >> 30) & 1; }

    template <bool kObs>
    __device__ static void step(const MView &M, State &st, int a, uint32_t id, uint32_t depth, uint32_t k0,
                                uint32_t k1, float &r, uint64_t &z) {
        int32_t w = st.w;
        r = 0.0f;
        z = 0;
        if ((w >> 30) & 1) return;  // absorbing
        int x = w & 31, y = (w >> 5) & 31;
        const int n = M.h->grid;
        int32_t term = 0;
        if (a == 0) {
            if (y + 1 < n) ++y;
        } else if (a == 1) {
            if (y > 0) --y;
        } else if (a == 2) {
            if (x + 1 == n) {
                r = 10.0f;
                term = 1 << 30;
            } else {
                ++x;
            }
        } else if (a == 3) {
            if (x > 0) --x;
        } else if (a == 4) {
            int i = -1;
            for (int q = 0; q < M.h->n_rocks; ++q)
                if (M.h->rock_x[q] == x && M.h->rock_y[q] == y) i = q;
            if (i >= 0) {
                if ((w >> (10 + i)) & 1) {
                    r = 10.0f;
                    w &= ~(1 << (10 + i));
                } else {
                    r = -10.0f;
                }
            }
        } else if (kObs) {
            // a sense leaves the state unchanged; its random reading is only
            // drawn when the observation is wanted
            const int i = a - 5;
            const int dx = x - M.h->rock_x[i], dy = y - M.h->rock_y[i];
            const uint32_t u = philox(id, depth, 0, kTagStep, k0, k1).x;
            const int correct = u <= M.thr[(uint32_t)(dx * dx + dy * dy)];
            const int truth = (w >> (10 + i)) & 1;
            z = (correct ? truth : !truth) ? 1 : 2;
        }
        st.w = (w & ~0x3ff) | x | (y << 5) | term;
    }

    __device__ static float upper(const MView &M, const State &st) {
        if ((st.w >> 30) & 1) return 0.0f;
        const int x = st.w & 31, y = (st.w >> 5) & 31;
        float u = 0.0f;
        for (int i = 0; i < M.h->n_rocks; ++i)
            if ((st.w >> (10 + i)) & 1) u += 10.0f * M.gpow_lane(abs(x - M.h->rock_x[i]) + abs(y - M.h->rock_y[i]));
        return u + 10.0f * M.gpow_lane(M.h->grid - 1 - x);
    }

    // Partial sums of the last common cell, kept across the rounds of a
    // tile: entry 16 g + m (lane of tab0, or of tab1 past 63) is the sum of
    // the terms of the good rocks of group g (rocks 4g .. 4g+3) when their
    // qualities read m.
    struct WaveUpper {
        int x = -1, y = -1;
        float tab0 = 0.0f, tab1 = 0.0f, exit = 0.0f;
    };

    // The same value, bit for bit, whichever way it is computed: the good
    // rocks' terms 10 gamma^d are summed within groups of four rocks in
    // index order, the group sums added in group order, then the exit term.
    // Robot cells are deterministic, so the live scenarios of a tile usually
    // share one cell: then the wavefront tabulates every group's sum for all
    // 16 quality patterns (rebuilt only when the cell changes) and each lane
    // adds one table entry per group of four rocks (a bit-field extract, a
    // cross-lane read and an add).  Called by all 64 lanes of a wavefront.
    __device__ static float upper_wave(const MView &M, const State &st, WaveUpper &wu) {
        const bool live = !((st.w >> 30) & 1);
        const int x = st.w & 31, y = (st.w >> 5) & 31;
        const uint64_t lv = __ballot(live);
        if (lv == 0) return 0.0f;
        const int leader = __ffsll((unsigned long long)lv) - 1;
        const int xs = __builtin_amdgcn_readlane(x, leader), ys = __builtin_amdgcn_readlane(y, leader);
        const int nr = M.h->n_rocks;
        const int ng = (nr + 3) >> 2;
        if (__ballot(live && (x != xs || y != ys)) != 0) {
            // cells differ: per-lane terms, discount powers read from the model table
            if (!live) return 0.0f;
            float u = 0.0f;
            for (int g = 0; g < ng; ++g) {
                float p = 0.0f;
                for (int i = 4 * g; i < 4 * g + 4 && i < nr; ++i)
                    if ((st.w >> (10 + i)) & 1)
                        p = p + 10.0f * M.gg[abs(x - M.h->rock_x[i]) + abs(y - M.h->rock_y[i])];
                u = u + p;
            }
            return u + 10.0f * M.gg[M.h->grid - 1 - x];
        }
        if (xs != wu.x || ys != wu.y) {
            const int lane = (int)__lane_id();
            const float ci =
                lane < nr ? 10.0f * M.gg[(uint32_t)(abs(xs - M.h->rock_x[lane]) + abs(ys - M.h->rock_y[lane]))] : 0.0f;
            // entry e = 16 g + m: group g's good rocks under pattern m, in index order
            float t0 = 0.0f, t1 = 0.0f;
            const int g0 = lane >> 4, g1 = 4 + (lane >> 4), m = lane & 15;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float c0 = __shfl(ci, (4 * g0 + b) & 63, 64);
                const float c1 = __shfl(ci, (4 * g1 + b) & 63, 64);
                if (((m >> b) & 1) && 4 * g0 + b < nr) t0 = t0 + c0;
                if (((m >> b) & 1) && 4 * g1 + b < nr) t1 = t1 + c1;
            }
            wu.tab0 = t0;
            wu.tab1 = t1;
            wu.exit = 10.0f * M.gpow_uniform(M.h->grid - 1 - xs);
            wu.x = xs;
            wu.y = ys;
        }
        const float u = group_table_sum((uint32_t)st.w >> 10, wu.tab0, wu.tab1) + wu.exit;
        return live ? u : 0.0f;
    }

    __device__ static int default_action(const MView &, const State &) { return 2; }  // move east
};

// ---------------------------------------------------------------------------
// Multi-agent RockSample: two robots share the rocks.  Two int32 rows per
// scenario: the robots' row (robot 1's cell in bits 0-9, robot 2's in bits
// 10-19, x in the low five bits of each; robot j gone in bit 20+j; terminal
// in bit 30) and the rocks' row (rock i's quality in bit i), at w[k] and
// w[stride + k].  Joint action a = a1 (5+m) + a2; robot 1 acts first, then
// robot 2 on the rocks robot 1 left; robot j's sensor reads word j of the
// step block; the joint observation is 3 z1 + z2.
// ---------------------------------------------------------------------------
struct MarsOps {
    struct State {
        int32_t p, rk;
    };
    static constexpr bool kHashObs = false;
    static constexpr bool kSplitRollout = true;
    static constexpr bool kSmallObs = true;  // 9 joint observations
    static constexpr bool kLdsModel = false;
    static constexpr bool kWaveUpper = true;
    static constexpr bool kGroupRollout = false;
    static constexpr int kGone0 = 20, kTerm = 30;
    static constexpr int kFar = 62;  // beyond any Manhattan distance on a 31 x 31 grid

    __device__ static void load(const MView &, const StatesPtr &S, int64_t p, State &st) {
        st.p = S.w[p];
        st.rk = S.w[S.stride + p];
    }
    __device__ static void make_terminal(State &st) {
        st.p = (1 << kTerm) | (3 << kGone0);
        st.rk = 0;
    }
    __device__ static void store(const MView &, const StatesPtr &S, int64_t p, const State &st) {
        S.w[p] = st.p;
        S.w[S.stride + p] = st.rk;
    }
    __device__ static bool terminal(const State &st) { return (st.p >> kTerm) & 1; }

    // Robot J's own action b (numbered as in RockSample); returns its reward.
    template <int J, bool kObs>
    __device__ static float act(const MView &M, State &st, int b, uint32_t word, int &zj) {
        zj = 0;
        int32_t p = st.p;
        if ((p >> (kGone0 + J)) & 1) return 0.0f;  // this robot has left the map
        constexpr int sh = 10 * J;
        int x = (p >> sh) & 31, y = (p >> (sh + 5)) & 31;
        const int n = M.h->grid;
        float r = 0.0f;
        if (b == 0) {
            if (y + 1 < n) ++y;
        } else if (b == 1) {
            if (y > 0) --y;
        } else if (b == 2) {
            if (x + 1 == n) {
                r = 10.0f;
                p |= 1 << (kGone0 + J);
            } else {
                ++x;
            }
        } else if (b == 3) {
            if (x > 0) --x;
        } else if (b == 4) {
            int i = -1;
            for (int q = 0; q < M.h->n_rocks; ++q)
                if (M.h->rock_x[q] == x && M.h->rock_y[q] == y) i = q;
            if (i >= 0) {
                if ((st.rk >> i) & 1) {
                    r = 10.0f;
                    st.rk &= ~(1 << i);
                } else {
                    r = -10.0f;
                }
            }
        } else if (kObs) {
            const int i = b - 5;
            const int dx = x - M.h->rock_x[i], dy = y - M.h->rock_y[i];
            const int correct = word <= M.thr[(uint32_t)(dx * dx + dy * dy)];
            const int truth = (st.rk >> i) & 1;
            zj = (correct ? truth : !truth) ? 1 : 2;
        }
        st.p = (p & ~(0x3ff << sh)) | ((x | (y << 5)) << sh);
        return r;
    }

    template <bool kObs>
    __device__ static void step(const MView &M, State &st, int a, uint32_t id, uint32_t depth, uint32_t k0,
                                uint32_t k1, float &r, uint64_t &z) {
        r = 0.0f;
        z = 0;
        if ((st.p >> kTerm) & 1) return;  // absorbing
        const int per = 5 + M.h->n_rocks;
        const int a1 = (a * M.h->joint_inv) >> 16, a2 = a - a1 * per;  // a / per without a division
        uint32_t w0 = 0, w1 = 0;
        if (kObs && (a1 >= 5 || a2 >= 5)) {
            // a sense's reading is only drawn when the observation is wanted
            const uint4 u = philox(id, depth, 0, kTagStep, k0, k1);
            w0 = u.x;
            w1 = u.y;
        }
        int z1, z2;
        const float r1 = act<0, kObs>(M, st, a1, w0, z1);
        const float r2 = act<1, kObs>(M, st, a2, w1, z2);
        r = r1 + r2;
        z = (uint64_t)(3 * z1 + z2);
        if (((st.p >> kGone0) & 3) == 3) st.p |= 1 << kTerm;
    }

    // Distance from the nearer robot still on the map to cell (rx, ry).
    __device__ static int near(int32_t p, int rx, int ry) {
        const int d0 = ((p >> kGone0) & 1) ? kFar : abs((p & 31) - rx) + abs(((p >> 5) & 31) - ry);
        const int d1 = ((p >> (kGone0 + 1)) & 1) ? kFar : abs(((p >> 10) & 31) - rx) + abs(((p >> 15) & 31) - ry);
        return d0 < d1 ? d0 : d1;
    }

    // Every good rock sampled by the nearer robot on arrival, plus each
    // robot's exit reward at its shortest exit time (rocks summed within
    // groups of four in index order, the group sums in group order, then
    // robot 1's exit, then robot 2's).
    __device__ static float upper(const MView &M, const State &st) {
        if ((st.p >> kTerm) & 1) return 0.0f;
        float u = 0.0f;
        const int nr = M.h->n_rocks;
        for (int g = 0; g < (nr + 3) >> 2; ++g) {
            float p = 0.0f;
            for (int i = 4 * g; i < 4 * g + 4 && i < nr; ++i)
                if ((st.rk >> i) & 1) p = p + 10.0f * M.gg[near(st.p, M.h->rock_x[i], M.h->rock_y[i])];
            u = u + p;
        }
        const int n1 = M.h->grid - 1;
        if (!((st.p >> kGone0) & 1)) u += 10.0f * M.gg[n1 - (st.p & 31)];
        if (!((st.p >> (kGone0 + 1)) & 1)) u += 10.0f * M.gg[n1 - ((st.p >> 10) & 31)];
        return u;
    }

    struct WaveUpper {
        int32_t p = -1;
        float tab0 = 0.0f, tab1 = 0.0f, e0 = 0.0f, e1 = 0.0f;
    };

    // The same value, bit for bit.  Robot cells are deterministic, so the
    // live scenarios of a tile usually share the robots' row: then the
    // wavefront tabulates each group of four rocks' sum for all 16 quality
    // patterns, as RockSample's bound does, and each lane adds one entry per
    // group; a robot that has left adds +0 for its exit.  Called by all 64
    // lanes of a wavefront.
    __device__ static float upper_wave(const MView &M, const State &st, WaveUpper &wu) {
        const bool live = !((st.p >> kTerm) & 1);
        const uint64_t lv = __ballot(live);
        if (lv == 0) return 0.0f;
        const int leader = __ffsll((unsigned long long)lv) - 1;
        const int32_t ps = __builtin_amdgcn_readlane(st.p, leader);
        if (__ballot(live && st.p != ps) != 0) return upper(M, st);
        const int nr = M.h->n_rocks;
        if (ps != wu.p) {
            const int lane = (int)__lane_id();
            const float ci = lane < nr ? 10.0f * M.gg[(uint32_t)near(ps, M.h->rock_x[lane], M.h->rock_y[lane])] : 0.0f;
            float t0 = 0.0f, t1 = 0.0f;
            const int g0 = lane >> 4, g1 = 4 + (lane >> 4), m = lane & 15;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float c0 = __shfl(ci, (4 * g0 + b) & 63, 64);
                const float c1 = __shfl(ci, (4 * g1 + b) & 63, 64);
                if (((m >> b) & 1) && 4 * g0 + b < nr) t0 = t0 + c0;
                if (((m >> b) & 1) && 4 * g1 + b < nr) t1 = t1 + c1;
            }
            wu.tab0 = t0;
            wu.tab1 = t1;
            const int n1 = M.h->grid - 1;
            wu.e0 = ((ps >> kGone0) & 1) ? 0.0f : 10.0f * M.gpow_uniform(n1 - (ps & 31));
            wu.e1 = ((ps >> (kGone0 + 1)) & 1) ? 0.0f : 10.0f * M.gpow_uniform(n1 - ((ps >> 10) & 31));
            wu.p = ps;
        }
        float u = group_table_sum((uint32_t)st.rk, wu.tab0, wu.tab1);
        u = u + wu.e0;
        u = u + wu.e1;
        return live ? u : 0.0f;
    }

    __device__ static int default_action(const MView &M, const State &) {
        return 2 * (5 + M.h->n_rocks) + 2;  // both robots move east
    }
};

// ---------------------------------------------------------------------------
// Navigation in a partially known map.  Five int32 rows per scenario: the
// robot (x bits 0-3, y bits 4-7, terminal bit 30) at w[k], then the unknown
// cells' occupancy (cell i in bit i % 32 of row 1 + i / 32) at
// w[(1 + j) * stride + k].  Actions 0 stay, 1-8 move N, NE, E, SE, S, SW, W,
// NW (y grows downwards).  A move draws word 0 of step block 0 (failure);
// a reading draws step blocks 1 and 2 (one word per neighbour).
// ---------------------------------------------------------------------------
constexpr int nav_dx_of(int a) { return (a == 0 || a == 1 || a == 5) ? 0 : (a >= 2 && a <= 4) ? 1 : -1; }
constexpr int nav_dy_of(int a) { return (a == 0 || a == 3 || a == 7) ? 0 : (a == 1 || a == 2 || a == 8) ? -1 : 1; }
// dx + 1 and dy + 1 of each action in two bits; the action of each (dx, dy)
// in four bits at (dy + 1) * 3 + dx + 1
constexpr uint32_t nav_pack_dir(bool y) {
    uint32_t v = 0;
    for (int a = 0; a < 9; ++a) v |= (uint32_t)((y ? nav_dy_of(a) : nav_dx_of(a)) + 1) << (2 * a);
    return v;
}
constexpr uint64_t nav_action_table() {
    uint64_t t = 0;
    for (int a = 0; a < 9; ++a) t |= (uint64_t)a << (4 * ((nav_dy_of(a) + 1) * 3 + nav_dx_of(a) + 1));
    return t;
}

struct NavOps {
    struct State {
        int32_t p;
        uint32_t m0, m1, m2, m3;
    };
    static constexpr bool kHashObs = true;
    static constexpr bool kSplitRollout = true;
    static constexpr bool kSmallObs = false;  // 8 reading bits: 256 observations
    static constexpr bool kLdsModel = true;   // discount powers staged in LDS
    static constexpr bool kWaveUpper = false;
    static constexpr bool kGroupRollout = false;
    struct WaveUpper {};
    static constexpr uint32_t kDx = nav_pack_dir(false), kDy = nav_pack_dir(true);
    static constexpr uint64_t kAction = nav_action_table();
    static constexpr uint64_t kTerminalObs = 256;

    __device__ static int dx(int a) { return (int)((kDx >> (2 * a)) & 3u) - 1; }
    __device__ static int dy(int a) { return (int)((kDy >> (2 * a)) & 3u) - 1; }

    __device__ static void load(const MView &, const StatesPtr &S, int64_t p, State &st) {
        st.p = S.w[p];
        st.m0 = (uint32_t)S.w[S.stride + p];
        st.m1 = (uint32_t)S.w[2 * S.stride + p];
        st.m2 = (uint32_t)S.w[3 * S.stride + p];
        st.m3 = (uint32_t)S.w[4 * S.stride + p];
    }
    __device__ static void make_terminal(State &st) {
        st.p = 1 << 30;
        st.m0 = st.m1 = st.m2 = st.m3 = 0;
    }
    __device__ static void store(const MView &, const StatesPtr &S, int64_t p, const State &st) {
        S.w[p] = st.p;
        S.w[S.stride + p] = (int32_t)st.m0;
        S.w[2 * S.stride + p] = (int32_t)st.m1;
        S.w[3 * S.stride + p] = (int32_t)st.m2;
        S.w[4 * S.stride + p] = (int32_t)st.m3;
    }
    __device__ static bool terminal(const State &st) { return (st.p >> 30) & 1; }

    // The scenario's map as bits 16 y + x (a wall or an occupied unknown
    // cell), built once for a rollout: the walls from the model, then the
    // grid bit of each occupied unknown cell.
    struct Grid {
        uint64_t w0, w1, w2, w3;
    };
    __device__ static Grid grid_of(const MView &M, const State &st) {
        Grid g{M.h->nav_wall_bits[0], M.h->nav_wall_bits[1], M.h->nav_wall_bits[2], M.h->nav_wall_bits[3]};
        const uint32_t words[4] = {st.m0, st.m1, st.m2, st.m3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t w = words[q];
            while (w) {
                const int c = 32 * q + __builtin_ctz(w);
                w &= w - 1u;
                const int bit = M.up[c];
                const uint64_t b = 1ull << (bit & 63);
                const int h = bit >> 6;
                g.w0 |= h == 0 ? b : 0ull;
                g.w1 |= h == 1 ? b : 0ull;
                g.w2 |= h == 2 ? b : 0ull;
                g.w3 |= h == 3 ? b : 0ull;
            }
        }
        return g;
    }
    __device__ static int occupied_grid(const MView &M, const Grid &g, int x, int y) {
        const int n = M.h->grid;
        if (x < 0 || y < 0 || x >= n || y >= n) return 1;
        const int bit = 16 * y + x;
        const uint64_t lo = bit < 64 ? g.w0 : g.w1, hi = bit < 192 ? g.w2 : g.w3;
        return (int)(((bit < 128 ? lo : hi) >> (bit & 63)) & 1u);
    }

    // Occupied in this scenario; off the map counts as occupied.
    __device__ static int occupied(const MView &M, const State &st, int x, int y) {
        const int n = M.h->grid;
        if (x < 0 || y < 0 || x >= n || y >= n) return 1;
        const int c = M.cl[y * n + x];
        if (c < 0) return c == -2 ? 1 : 0;
        // two 64-bit halves and a select: a four-way select chain becomes a
        // private array indexed by c / 32 (scratch memory)
        const uint64_t lo = (uint64_t)st.m0 | ((uint64_t)st.m1 << 32);
        const uint64_t hi = (uint64_t)st.m2 | ((uint64_t)st.m3 << 32);
        const uint64_t half = c < 64 ? lo : hi;
        return (int)((half >> (c & 63)) & 1u);
    }

    // The motion of a step from a live state, with the failure word (word 0
    // of the step block) already drawn (a stay draws none) and the cells'
    // occupancy given by occ(x, y).
    template <class Occ>
    __device__ static void move(const MView &M, State &st, int a, uint32_t u_fail, float &r, const Occ &occ) {
        int x = st.p & 15, y = (st.p >> 4) & 15;
        int term = 0;
        if (a == 0) {
            r = -0.2f;
        } else if ((uint64_t)u_fail < M.h->fail_thr) {
            r = -0.1f;  // the move fails: the robot stays
        } else {
            const int tx = x + dx(a), ty = y + dy(a);
            if (occ(tx, ty)) {
                r = -1.0f;  // crash: the robot stays
            } else {
                x = tx;
                y = ty;
                if (x == M.h->nav_goal_x && y == M.h->grid - 1) {
                    r = 20.0f;
                    term = 1;
                } else {
                    r = -0.1f;
                }
            }
        }
        st.p = x | (y << 4) | (term << 30);
    }

    template <bool kObs>
    __device__ static void step(const MView &M, State &st, int a, uint32_t id, uint32_t depth, uint32_t k0,
                                uint32_t k1, float &r, uint64_t &z) {
        r = 0.0f;
        z = kTerminalObs;
        if ((st.p >> 30) & 1) return;  // absorbing
        const State s0 = st;
        move(M, st, a, a == 0 ? 0u : philox(id, depth, 0, kTagStep, k0, k1).x, r,
             [&](int cx, int cy) { return occupied(M, s0, cx, cy); });
        if (!kObs || ((st.p >> 30) & 1)) return;
        const int x = st.p & 15, y = (st.p >> 4) & 15;
        const uint4 b1 = philox(id, depth, 1, kTagStep, k0, k1);
        const uint4 b2 = philox(id, depth, 2, kTagStep, k0, k1);
        const uint32_t words[8] = {b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w};
        uint64_t obs = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int bit = occupied(M, st, x + dx(j + 1), y + dy(j + 1));
            if ((uint64_t)words[j] < M.h->err_thr) bit ^= 1;
            obs |= (uint64_t)bit << j;
        }
        z = obs;
    }

    // The goal reward on the shortest 8-connected path, no costs; it is paid
    // on entering the goal, so a robot standing on it must leave and re-enter
    // (two moves).
    __device__ static float upper(const MView &M, const State &st) {
        if ((st.p >> 30) & 1) return 0.0f;
        const int ax = abs((st.p & 15) - M.h->nav_goal_x), ay = abs(((st.p >> 4) & 15) - (M.h->grid - 1));
        const int d = ax > ay ? ax : ay;
        return 20.0f * M.gpow_lane(d > 0 ? d - 1 : 1);
    }
    __device__ static float upper_wave(const MView &M, const State &st, WaveUpper &) { return upper(M, st); }

    // Head for the open gate while above the wall, then for the goal: the
    // diagonal step towards the target, else its vertical part, else its
    // horizontal part, the first that lands on a free cell; else stay.
    template <class Occ>
    __device__ static int default_action_occ(const MView &M, const State &st, const Occ &occ) {
        const int x = st.p & 15, y = (st.p >> 4) & 15;
        int tx = M.h->nav_goal_x, ty = M.h->grid - 1;
        if (y < M.h->nav_wall) {
            const int g = !(st.m0 & 1u) ? 0 : (!(st.m0 & 2u) ? 1 : -1);
            if (g >= 0) {
                tx = M.h->nav_gate_x[g];
                ty = M.h->nav_wall;
            }
        }
        const int sx = tx > x ? 1 : (tx < x ? -1 : 0), sy = ty > y ? 1 : (ty < y ? -1 : 0);
        const int cx[3] = {sx, 0, sx}, cy[3] = {sy, sy, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (cx[c] == 0 && cy[c] == 0) continue;
            if (occ(x + cx[c], y + cy[c])) continue;
            return (int)((kAction >> (4 * ((cy[c] + 1) * 3 + cx[c] + 1))) & 15u);
        }
        return 0;
    }
    __device__ static int default_action(const MView &M, const State &st) {
        return default_action_occ(M, st, [&](int cx, int cy) { return occupied(M, st, cx, cy); });
    }

    // A rollout (rollout_loop's operations and order) with the map held as
    // bits in registers for its whole length: the occupancy tests of the
    // policy and of the moves read no table.  Shorter for the lone
    // wavefronts of small leaves; a batch of full tiles keeps the table
    // lookups, which need fewer registers.
    template <int POL>
    __device__ static float rollout_grid_p(const MView &M, const RolloutParams &P, State st, uint32_t id, int d0,
                                           int n_roll, int &nsteps) {
        float value = 0.0f;
        if (n_roll <= 0 || terminal(st)) return value;
        const Grid g = grid_of(M, st);
        const auto occ = [&](int cx, int cy) { return occupied_grid(M, g, cx, cy); };
        for (int j = 0; j < n_roll; ++j) {
            if (terminal(st)) break;
            const uint32_t depth = (uint32_t)(d0 + j);
            int a;
            if (POL == HDX_POLICY_CONST) {
                a = P.const_action;
            } else if (POL == HDX_POLICY_RANDOM) {
                a = (int)(philox(id, depth, 0, kTagPolicy, P.k0, P.k1).x % (uint32_t)P.n_actions);
            } else {
                a = default_action_occ(M, st, occ);
            }
            float r;
            move(M, st, a, a == 0 ? 0u : philox(id, depth, 0, kTagStep, P.k0, P.k1).x, r, occ);
            value += M.gpow_uniform(j) * r;
            ++nsteps;
        }
        return value;
    }
    __device__ static float rollout_grid(const MView &M, const RolloutParams &P, const State &st, uint32_t id,
                                         int d0, int &nsteps) {
        int n_roll = P.max_steps;
        if (P.max_depth >= 0 && P.max_depth - d0 < n_roll) n_roll = P.max_depth - d0;
        if (n_roll > kHorizon) n_roll = kHorizon;
        if (P.policy == HDX_POLICY_CONST) return rollout_grid_p<HDX_POLICY_CONST>(M, P, st, id, d0, n_roll, nsteps);
        if (P.policy == HDX_POLICY_RANDOM) return rollout_grid_p<HDX_POLICY_RANDOM>(M, P, st, id, d0, n_roll, nsteps);
        return rollout_grid_p<HDX_POLICY_DEFAULT>(M, P, st, id, d0, n_roll, nsteps);
    }

};

// ---------------------------------------------------------------------------
// Crowd driving: car (position, speed level, terminal) and up to PM
// pedestrians held in registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 output function
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ uint64_t hash_field(uint64_t h, int32_t f) {
    return mix64((h ^ (uint64_t)(uint32_t)f) + 0x9E3779B97F4A7C15ull);
}

template <int PM>
struct PedOps {
    struct State {
        float s;
        int32_t level, term;
        float px[PM], py[PM];
        int32_t goal[PM];
    };
    static constexpr bool kHashObs = true;
    static constexpr bool kSplitRollout = false;  // large step: one loop keeps the code small
    static constexpr bool kSmallObs = false;      // 64-bit hashed observations
    static constexpr bool kLdsModel = true;       // discount powers and goal points staged in LDS
    static constexpr bool kWaveUpper = false;     // per-lane upper bound
    static constexpr bool kGroupRollout = true;   // small leaves: one lane per pedestrian (group_expand)
    struct WaveUpper {};

    // One pedestrian's walk towards its goal with heading noise from the
    // four words of its block (shared by the one-lane step and the
    // element-level rollout, so both take the same operations).
    __device__ static void move_ped(const MView &M, const uint4 &u, int goal, float &px, float &py) {
        const int32_t sum = (int32_t)((u.x >> 8) + (u.y >> 8) + (u.z >> 8) + (u.w >> 8));
        const float noise = (float)(sum - 33554430) * M.h->ih_scale;
        const float gx = M.goal_x(goal), gy = M.goal_y(goal);
        const float dx = gx - px;
        const float dy = gy - py;
        const float dist = __builtin_sqrtf(dx * dx + dy * dy);
        const float step_len = M.h->step_len;
        if (dist <= step_len) {
            px = gx;
            py = gy;
        } else {
            const float ux = dx / dist, uy = dy / dist;
            const float t = M.h->half_sigma * noise;
            const float t2 = t * t;
            const float den = 1.0f + t2;
            const float c = (1.0f - t2) / den;
            const float sn = (2.0f * t) / den;
            const float rx = ux * c - uy * sn;
            const float ry = ux * sn + uy * c;
            px = px + step_len * rx;
            py = py + step_len * ry;
        }
    }

    __device__ static void load(const MView &M, const StatesPtr &S, int64_t p, State &st) {
        st.s = S.s[p];
        const int32_t car = S.car[p];
        st.level = car & 0xff;
        st.term = (car >> 8) & 1;
#pragma unroll
        for (int j = 0; j < PM; ++j) {
            if (j < M.h->n_peds) {
                st.px[j] = S.px[j * S.stride + p];
                st.py[j] = S.py[j * S.stride + p];
                st.goal[j] = S.goal[j * S.stride + p];
            } else {
                st.px[j] = 0.0f;
                st.py[j] = 0.0f;
                st.goal[j] = 0;
            }
        }
    }
    __device__ static void store(const MView &M, const StatesPtr &S, int64_t p, const State &st) {
        S.s[p] = st.s;
        S.car[p] = (st.level & 0xff) | (st.term ? 0x100 : 0);
#pragma unroll
        for (int j = 0; j < PM; ++j) {
            if (j < M.h->n_peds) {
                S.px[j * S.stride + p] = st.px[j];
                S.py[j * S.stride + p] = st.py[j];
                S.goal[j * S.stride + p] = (uint8_t)st.goal[j];
            }
        }
    }
    __device__ static bool terminal(const State &st) { return st.term != 0; }

    template <bool kObs>
    __device__ static void step(const MView &M, State &st, int a, uint32_t id, uint32_t depth, uint32_t k0,
                                uint32_t k1, float &r, uint64_t &z) {
        if (st.term) {
            r = 0.0f;
            z = kPedTerminalObs;
            return;
        }
        const uint4 u0 = philox(id, depth, 0, kTagStep, k0, k1);
        const bool failed = (uint64_t)u0.x < M.h->fail_thr;
        int level = st.level;
        if (a == 0 && !failed && level < M.h->n_levels - 1) level = level + 1;
        if (a == 2 && !failed && level > 0) level = level - 1;
        const float v = 0.5f * (float)level;
        const float s_next = st.s + v * M.h->dt;
#pragma unroll
        for (int j = 0; j < PM; ++j) {
            if (j < M.h->n_peds) {
                const uint4 u = philox(id, depth, (uint32_t)(j + 1), kTagStep, k0, k1);
                move_ped(M, u, st.goal[j], st.px[j], st.py[j]);
            }
        }
        bool collided = false;
        if (level > 0) {
            const float r2 = M.h->coll_r2;
#pragma unroll
            for (int j = 0; j < PM; ++j) {
                if (j < M.h->n_peds) {
                    const float ddx = st.px[j] - s_next;
                    const float d2 = ddx * ddx + st.py[j] * st.py[j];
                    collided = collided || (d2 < r2);
                }
            }
        }
        float reward = M.h->r_step;
        if (collided) {
            reward = M.h->r_step + M.h->r_collision;
            st.term = 1;
        } else if (s_next >= M.h->path_len) {
            reward = M.h->r_step + M.h->r_goal;
            st.term = 1;
        }
        st.s = s_next;
        st.level = level;
        r = reward;
        if (kObs) {
            if (st.term) {
                z = kPedTerminalObs;
            } else {
                uint64_t h = 0x243F6A8885A308D3ull;
                h = hash_field(h, level);
#pragma unroll
                for (int j = 0; j < PM; ++j) {
                    if (j < M.h->n_peds) {
                        h = hash_field(h, (int32_t)floorf(st.px[j]));
                        h = hash_field(h, (int32_t)floorf(st.py[j]));
                    }
                }
                z = (h == kPedTerminalObs) ? kPedTerminalObs - 1 : h;
            }
        } else {
            z = 0;
        }
    }

    __device__ static float upper(const MView &M, const State &st) {
        if (st.term) return 0.0f;
        const float T = ceilf((M.h->path_len - st.s) / M.h->reach);
        int Ti = (int)T;
        if (Ti < 1) Ti = 1;
        if (Ti > kHorizon) Ti = kHorizon;
        return M.h->r_goal * M.gpow_lane(Ti - 1);
    }

    __device__ static int default_action(const MView &M, const State &st) {
        bool brake = false;
#pragma unroll
        for (int j = 0; j < PM; ++j) {
            if (j < M.h->n_peds) {
                const float ahead = st.px[j] - st.s;
                brake = brake || (ahead >= 0.0f && ahead <= 3.0f && fabsf(st.py[j]) < 1.5f);
            }
        }
        return brake ? 2 : 0;
    }

    // Element-level work on a small leaf (Sec. III-D: the parallelism inside
    // one step of a scenario).  Scenario g of the wavefront's first n
    // scenarios runs on lanes [g*G, g*G + G), lane g*G + j holding
    // pedestrian j (G a power of two >= the pedestrian count, n * G <= 64);
    // every lane of a group carries the car, the reward and the value;
    // collisions and the braking rule are ORs of the group's ballot bits, and
    // the observation hash is chained over the group's lanes in pedestrian
    // order by shuffles.  The operations and their order are those of the
    // one-lane step and rollout, so the results are the same bits.
    struct Lanes {
        int g, j;        // scenario of the group, pedestrian of the lane
        bool active;     // g < n
        bool ped;        // active and j < n_peds
        uint64_t gmask;  // the group's lanes
    };
    __device__ static Lanes lanes(const MView &M, int n, int G) {
        Lanes L;
        const int lane = (int)__lane_id();
        L.g = lane / G;
        L.j = lane - L.g * G;
        L.active = L.g < n;
        L.ped = L.active && L.j < M.h->n_peds;
        L.gmask = (G >= 64 ? ~0ull : ((1ull << G) - 1ull)) << (L.g * G);
        return L;
    }

    // One step of one scenario spread over its group (PedOps::step).
    template <bool kObs>
    __device__ static void group_step(const MView &M, const Lanes &E, int G, int a, uint32_t id, uint32_t depth,
                                      uint32_t k0, uint32_t k1, float &s, int &level, int &term, float &px,
                                      float &py, int goal, float &r, uint64_t &z) {
        r = 0.0f;
        z = kObs ? kPedTerminalObs : 0;
        if (term) return;  // group-uniform
        const uint4 u0 = philox(id, depth, 0, kTagStep, k0, k1);
        const bool failed = (uint64_t)u0.x < M.h->fail_thr;
        if (a == 0 && !failed && level < M.h->n_levels - 1) level = level + 1;
        if (a == 2 && !failed && level > 0) level = level - 1;
        const float v = 0.5f * (float)level;
        const float s_next = s + v * M.h->dt;
        if (E.ped) {
            const uint4 u = philox(id, depth, (uint32_t)(E.j + 1), kTagStep, k0, k1);
            move_ped(M, u, goal, px, py);
        }
        bool hit = false;
        if (level > 0 && E.ped) {
            const float ddx = px - s_next;
            const float d2 = ddx * ddx + py * py;
            hit = d2 < M.h->coll_r2;
        }
        const bool collided = (__ballot(hit) & E.gmask) != 0;
        float reward = M.h->r_step;
        if (collided) {
            reward = M.h->r_step + M.h->r_collision;
            term = 1;
        } else if (s_next >= M.h->path_len) {
            reward = M.h->r_step + M.h->r_goal;
            term = 1;
        }
        s = s_next;
        r = reward;
        if (!kObs) return;
        // the chained hash, in pedestrian order: every lane of the group
        // walks the chain over its group's lanes
        const int fx = (int32_t)floorf(px), fy = (int32_t)floorf(py);
        uint64_t h = hash_field(0x243F6A8885A308D3ull, level);
        const int base = E.g * G;
        for (int q = 0; q < M.h->n_peds; ++q) {
            const int qx = __shfl(fx, base + q, 64);
            const int qy = __shfl(fy, base + q, 64);
            h = hash_field(h, qx);
            h = hash_field(h, qy);
        }
        if (!term) z = (h == kPedTerminalObs) ? kPedTerminalObs - 1 : h;
    }

    // The default-policy rollout of one scenario spread over its group,
    // from the lanes' element state (rollout_loop's operations).
    __device__ static float group_roll(const MView &M, const RolloutParams &P, const Lanes &E, float s, int level,
                                       int term, uint32_t sid, float px, float py, int goal, int d0, int &steps) {
        int n_roll = P.max_steps;
        if (P.max_depth >= 0 && P.max_depth - d0 < n_roll) n_roll = P.max_depth - d0;
        if (n_roll > kHorizon) n_roll = kHorizon;
        float value = 0.0f;
        steps = 0;
        for (int t = 0; t < n_roll; ++t) {
            if (term) break;
            const uint32_t depth = (uint32_t)(d0 + t);
            int a;
            if (P.policy == HDX_POLICY_CONST) {
                a = P.const_action;
            } else if (P.policy == HDX_POLICY_RANDOM) {
                a = (int)(philox(sid, depth, 0, kTagPolicy, P.k0, P.k1).x % (uint32_t)P.n_actions);
            } else {
                const float ahead = px - s;
                const bool b = E.ped && ahead >= 0.0f && ahead <= 3.0f && fabsf(py) < 1.5f;
                a = (__ballot(b) & E.gmask) ? 2 : 0;
            }
            const uint4 u0 = philox(sid, depth, 0, kTagStep, P.k0, P.k1);
            const bool failed = (uint64_t)u0.x < M.h->fail_thr;
            if (a == 0 && !failed && level < M.h->n_levels - 1) level = level + 1;
            if (a == 2 && !failed && level > 0) level = level - 1;
            const float v = 0.5f * (float)level;
            const float s_next = s + v * M.h->dt;
            if (E.ped) {
                const uint4 u = philox(sid, depth, (uint32_t)(E.j + 1), kTagStep, P.k0, P.k1);
                move_ped(M, u, goal, px, py);
            }
            bool hit = false;
            if (level > 0 && E.ped) {
                const float ddx = px - s_next;
                const float d2 = ddx * ddx + py * py;
                hit = d2 < M.h->coll_r2;
            }
            const bool collided = (__ballot(hit) & E.gmask) != 0;
            float reward = M.h->r_step;
            if (collided) {
                reward = M.h->r_step + M.h->r_collision;
                term = 1;
            } else if (s_next >= M.h->path_len) {
                reward = M.h->r_step + M.h->r_goal;
                term = 1;
            }
            s = s_next;
            value += M.gpow_uniform(t) * reward;
            ++steps;
        }
        return value;
    }

    // What one scenario of a small leaf yields in the element-level
    // expansion; lane k < n holds scenario k's.
    struct GroupOut {
        float r, U, L;
        uint64_t z;
        uint32_t id;
        int expanded, steps;
    };

    // Element-level expansion of a small leaf's tile: gather and update (the
    // parent's last action), the step of action a with its observation, the
    // upper bound and the rollout, all with one pedestrian per lane.  Leaf
    // states (write_leaf) and stepped states (sprime) are stored by the
    // owning lanes.  All 64 lanes of a wavefront call this.
    __device__ static GroupOut group_expand(const MView &M, const RolloutParams &P, const int16_t *idx,
                                            const uint32_t *parent_ids, const StatesPtr &parent,
                                            const StatesPtr &leaf_out, uint32_t *ids_out, const StatesPtr &sprime,
                                            bool write_leaf, bool pair_out, int a, int depth, int last_action, int n,
                                            int G) {
        const Lanes E = lanes(M, n, G);
        float s = 0.0f, px = 0.0f, py = 0.0f;
        int level = 0, term = 1, goal = 0;
        uint32_t id = 0;
        int p = 0;
        if (E.active) {
            p = idx[E.g];
            id = parent_ids[p];
            s = parent.s[p];
            const int32_t car = parent.car[p];
            level = car & 0xff;
            term = (car >> 8) & 1;
            if (E.ped) {
                px = parent.px[E.j * parent.stride + p];
                py = parent.py[E.j * parent.stride + p];
                goal = parent.goal[E.j * parent.stride + p];
            }
        }
        float r0;
        uint64_t z0;
        if (last_action >= 0)
            group_step<false>(M, E, G, last_action, id, (uint32_t)(depth - 1), P.k0, P.k1, s, level, term, px, py,
                              goal, r0, z0);
        const int k = E.g;
        if (write_leaf && E.active) {
            if (E.j == 0) {
                leaf_out.s[k] = s;
                leaf_out.car[k] = (level & 0xff) | (term ? 0x100 : 0);
                ids_out[k] = id;
            }
            if (E.ped) {
                leaf_out.px[E.j * leaf_out.stride + k] = px;
                leaf_out.py[E.j * leaf_out.stride + k] = py;
                leaf_out.goal[E.j * leaf_out.stride + k] = (uint8_t)goal;
            }
        }
        const int expanded = term ? 0 : 1;
        float r;
        uint64_t z;
        group_step<true>(M, E, G, a, id, (uint32_t)depth, P.k0, P.k1, s, level, term, px, py, goal, r, z);
        if (pair_out && E.active) {
            const int64_t q = (int64_t)a * n + k;
            if (E.j == 0) {
                sprime.s[q] = s;
                sprime.car[q] = (level & 0xff) | (term ? 0x100 : 0);
            }
            if (E.ped) {
                sprime.px[E.j * sprime.stride + q] = px;
                sprime.py[E.j * sprime.stride + q] = py;
                sprime.goal[E.j * sprime.stride + q] = (uint8_t)goal;
            }
        }
        State up;
        up.s = s;
        up.term = term;
        const float U = upper(M, up);
        int steps = 0;
        const float L = group_roll(M, P, E, s, level, term, id, px, py, goal, depth + 1, steps);
        // scenario k's results from its group's first lane to lane k
        const int from = ((int)__lane_id() < n ? (int)__lane_id() : 0) * G;
        GroupOut o;
        o.r = __shfl(r, from, 64);
        o.U = __shfl(U, from, 64);
        o.L = __shfl(L, from, 64);
        o.z = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(z >> 32), from, 64) << 32) |
              (uint32_t)__shfl((int)(uint32_t)z, from, 64);
        o.id = (uint32_t)__shfl((int)id, from, 64);
        o.expanded = __shfl(expanded, from, 64);
        o.steps = __shfl(steps, from, 64);
        return o;
    }
};

// Default-policy rollout from depth d0 (Eq. 13): discounted from d0, stops
// at a terminal state or after min(max_steps, max_depth - d0) steps; the
// tail value past the horizon is 0.  Accumulates in FP32 in step order.
// The loop is compiled once per policy, so the policy is not re-decided at
// every step and a model whose default action is a constant (RockSample's
// move east) steps through that action's code alone.
template <class Ops, int POL>
__device__ __forceinline__ float rollout_loop(const MView &M, const RolloutParams &P, typename Ops::State st,
                                              uint32_t id, int d0, int n_roll, int &nsteps) {
    float value = 0.0f;
    for (int j = 0; j < n_roll; ++j) {
        if (Ops::terminal(st)) break;
        const uint32_t depth = (uint32_t)(d0 + j);
        int a;
        if (POL == HDX_POLICY_CONST) {
            a = P.const_action;
        } else if (POL == HDX_POLICY_RANDOM) {
            a = (int)(philox(id, depth, 0, kTagPolicy, P.k0, P.k1).x % (uint32_t)P.n_actions);
        } else {
            a = Ops::default_action(M, st);
        }
        float r;
        uint64_t z;
        Ops::template step<false>(M, st, a, id, depth, P.k0, P.k1, r, z);
        value += M.gpow_uniform(j) * r;
        ++nsteps;
    }
    return value;
}

template <class Ops>
__device__ __forceinline__ float rollout(const MView &M, const RolloutParams &P, typename Ops::State st,
                                         uint32_t id, int d0, int &nsteps) {
    int n_roll = P.max_steps;
    if (P.max_depth >= 0 && P.max_depth - d0 < n_roll) n_roll = P.max_depth - d0;
    if (n_roll > kHorizon) n_roll = kHorizon;  // the discount table's length
    if (!Ops::kSplitRollout) {
        float value = 0.0f;
        for (int j = 0; j < n_roll; ++j) {
            if (Ops::terminal(st)) break;
            const uint32_t depth = (uint32_t)(d0 + j);
            int a;
            if (P.policy == HDX_POLICY_CONST) {
                a = P.const_action;
            } else if (P.policy == HDX_POLICY_RANDOM) {
                a = (int)(philox(id, depth, 0, kTagPolicy, P.k0, P.k1).x % (uint32_t)P.n_actions);
            } else {
                a = Ops::default_action(M, st);
            }
            float r;
            uint64_t z;
            Ops::template step<false>(M, st, a, id, depth, P.k0, P.k1, r, z);
            value += M.gpow_uniform(j) * r;
            ++nsteps;
        }
        return value;
    }
    if (P.policy == HDX_POLICY_CONST) return rollout_loop<Ops, HDX_POLICY_CONST>(M, P, st, id, d0, n_roll, nsteps);
    if (P.policy == HDX_POLICY_RANDOM) return rollout_loop<Ops, HDX_POLICY_RANDOM>(M, P, st, id, d0, n_roll, nsteps);
    return rollout_loop<Ops, HDX_POLICY_DEFAULT>(M, P, st, id, d0, n_roll, nsteps);
}

}  // namespace hdx
