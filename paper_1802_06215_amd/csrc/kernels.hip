// HIP kernels for gfx950: scenario sampling, fused leaf expansion (update,
// expand, group by observation, bounds, rollouts, reductions) and
// stand-alone rollout bounds.
//
// Leaf expansion (Sec. III-D, Eq. 10-13) runs one workgroup per tile, a tile
// being one (leaf, action) pair.  Inside a tile every lane owns scenarios
// k = tid, tid + T, ...: it gathers the parent state (struct-of-arrays,
// coalesced along k), applies the last action, steps the tile's action,
// evaluates the upper-bound heuristic and runs the default-policy rollout in
// registers.  Then the scenarios are grouped by observation, two ways:
//  - observation alphabets below 32 keys (RockSample): in registers, per
//    64-scenario chunk one ballot per key present gives counts and ranks
//    and DPP row reductions the key's U and L sums; one wavefront turns the
//    per-chunk tables into children (ascending key), offsets and means,
//    chunk partials added in chunk order;
//  - hashed observations (driving): an open-addressing LDS hash collects
//    the distinct observations, which are sorted (one wavefront bitonic
//    network, or an LDS bitonic network past 64 keys); scenario positions
//    inside each child come from wavefront ballots per 64-scenario chunk
//    and a prefix over chunks, and the per-child sums of U and L from
//    segmented wavefront scans over 64-aligned chunks of the grouped order,
//    chunk partials added in order.
// Either way the floating-point order depends only on the data, never on
// the workgroup size or the schedule.
#include <type_traits>

#include "models.hpp"

namespace hdx {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Sum of v over the 64 lanes (all active), in one fixed order: inclusive
// prefix sums inside each row of 16 lanes (row shifts by 1, 2, 4, 8), then
// the row totals carried by the row broadcasts of lanes 15 and 31; the total
// is lane 63's prefix.  Lanes without a source add +0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_src(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
__device__ __forceinline__ float wave_total(float v) {
    v = v + dpp_src<0x111, 0xf>(v);  // row_shr:1
    v = v + dpp_src<0x112, 0xf>(v);  // row_shr:2
    v = v + dpp_src<0x114, 0xf>(v);  // row_shr:4
    v = v + dpp_src<0x118, 0xf>(v);  // row_shr:8
    v = v + dpp_src<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = v + dpp_src<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// The same for integers (exact): the wavefront's sum, on every lane.
__device__ __forceinline__ int wave_total_i(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint64_t mix_key(uint64_t z) {
    return (z * 0x9E3779B97F4A7C15ull) >> 32;
}

// Lexicographic (key, val) compare-exchange used by both sorting networks.
__device__ __forceinline__ bool pair_less(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
    return ka < kb || (ka == kb && va < vb);
}

// Bitonic sort of up to 64 (key, val) pairs held one per lane of a wavefront.
__device__ void wave_sort_pairs(uint64_t *keys, uint32_t *vals, int count) {
    const int lane = lane_id();
    uint64_t k = lane < count ? keys[lane] : kEmptyKey;
    uint32_t v = lane < count ? vals[lane] : 0xFFFFFFFFu;
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint32_t klo = __shfl_xor((uint32_t)k, stride, 64);
            const uint32_t khi = __shfl_xor((uint32_t)(k >> 32), stride, 64);
            const uint32_t ov = __shfl_xor(v, stride, 64);
            const uint64_t ok = ((uint64_t)khi << 32) | klo;
            const bool ascending = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            const bool other_smaller = pair_less(ok, ov, k, v);
            // the lower lane of an ascending pair keeps the smaller element
            const bool take = (lower == ascending) ? other_smaller : !other_smaller;
            if (take) {
                k = ok;
                v = ov;
            }
        }
    }
    if (lane < count) {
        keys[lane] = k;
        vals[lane] = v;
    }
}

// Bitonic sort in LDS of p (a power of two) (key, val) pairs.
__device__ void block_sort_pairs(uint64_t *keys, uint32_t *vals, int p) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int size = 2; size <= p; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < p; i += nt) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool ascending = (i & size) == 0;
                    const bool swap = ascending ? pair_less(keys[j], vals[j], keys[i], vals[i])
                                                : pair_less(keys[i], vals[i], keys[j], vals[j]);
                    if (swap) {
                        const uint64_t tk = keys[i];
                        keys[i] = keys[j];
                        keys[j] = tk;
                        const uint32_t tv = vals[i];
                        vals[i] = vals[j];
                        vals[j] = tv;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Bitonic sort in LDS of p (a power of two) uint32 keys.
__device__ void block_sort_u32(uint32_t *keys, int p) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int size = 2; size <= p; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < p; i += nt) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool ascending = (i & size) == 0;
                    const uint32_t a = keys[i], b = keys[j];
                    if (ascending ? (b < a) : (a < b)) {
                        keys[i] = b;
                        keys[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Exclusive prefix sum of len ints, in place, by the whole workgroup.
// scratch holds one int per wavefront plus one.
__device__ void block_exclusive_scan(int32_t *a, int len, int32_t *scratch) {
    const int tid = threadIdx.x, nt = blockDim.x, lane = lane_id(), wid = tid >> 6, nw = nt >> 6;
    const int per = (len + nt - 1) / nt;
    const int lo = tid * per, hi = min(lo + per, len);
    int32_t local = 0;
    for (int i = lo; i < hi; ++i) local += a[i];
    int32_t incl = local;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) scratch[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int w = 0; w < nw; ++w) {
            const int32_t t = scratch[w];
            scratch[w] = run;
            run += t;
        }
    }
    __syncthreads();
    int32_t run = scratch[wid] + incl - local;
    for (int i = lo; i < hi; ++i) {
        const int32_t t = a[i];
        a[i] = run;
        run += t;
    }
    __syncthreads();
}

__device__ __forceinline__ bool has_states(const StatesPtr &S) { return S.w != nullptr || S.s != nullptr; }

// One (leaf, action) tile.
// kGroup: compile the element-level expansion of small leaves in (the
// kernel-argument launches of the search threads and batchers; the staged
// batched launch leaves it out, since its registers would cost the driving
// model a wavefront per SIMD).
template <class Ops, bool kGroup = false>
__device__ void run_tile(const HDX_CONST LeafTask *T, const int a, unsigned char *lds, const LdsLayout &Ly) {
    float *gpow_lds = (float *)(lds + Ly.gpow);
    const MView M = make_view(T->model, gpow_lds);
    const int n = T->n;
    const int cap = T->cap;
    const int tid = threadIdx.x, nt = blockDim.x, lane = lane_id(), wid = tid >> 6, nw = nt >> 6;
    uint64_t *zk = (uint64_t *)(lds + Ly.zkey);
    uint64_t *tab = (uint64_t *)(lds + Ly.tab);
    uint32_t *dslot = (uint32_t *)(lds + Ly.dslot);
    int32_t *nc = (int32_t *)(lds + Ly.dslot);  // after ranking
    int32_t *off = (int32_t *)(lds + Ly.off);
    float *ub = (float *)(lds + Ly.ubuf);
    float *lb = (float *)(lds + Ly.lbuf);
    int32_t *child = (int32_t *)(lds + Ly.child);
    int16_t *kchild = (int16_t *)(lds + Ly.child);  // small alphabets: key | rank << 5
    int32_t *permb = (int32_t *)(lds + Ly.perm);
    // per-chunk child counts: over zkey and tab (contiguous)
    int32_t *cnt = (int32_t *)(lds + Ly.zkey);
    int32_t *misc = (int32_t *)(lds + Ly.misc);                   // [0] distinct count, [1] sentinel seen
    unsigned long long *stepc = (unsigned long long *)(misc + 4);  // expansion, rollout steps
    float *chunk_r = (float *)(misc + 8);                          // per-chunk reward sums (<= 32)
    int32_t *scan_scratch = misc + 48;
    const int H = Ly.h;
    // small observation alphabet (keys below 32): per 64-scenario chunk t and
    // key v, the scenario count and the U and L sums (entry t * 32 + v, over
    // zkey), the chunk's key mask (over dslot), and per key the child offset
    // and child index (over off)
    const int kchunks = (Ly.np + 63) >> 6;
    int32_t *kc = (int32_t *)(lds + Ly.zkey);
    float *ku = (float *)(kc + 32 * kchunks);
    float *kl = ku + 32 * kchunks;
    uint32_t *kmask = (uint32_t *)(lds + Ly.dslot);
    int32_t *koff = (int32_t *)(lds + Ly.off);
    int32_t *kci = koff + 32;

    if constexpr (!Ops::kSmallObs)
        for (int h = tid; h < H; h += nt) tab[h] = kEmptyKey;
    if (tid == 0) {
        misc[0] = 0;
        misc[1] = 0;
        stepc[0] = 0;
        stepc[1] = 0;
    }
    if constexpr (Ops::kLdsModel) stage_gpow(T->model, gpow_lds);
    if constexpr (std::is_same<Ops, NavOps>::value) stage_cells(T->model, gpow_lds);
    __syncthreads();

    RolloutParams RP;
    RP.k0 = T->k0;
    RP.k1 = T->k1;
    RP.policy = T->policy;
    RP.const_action = T->const_action;
    RP.max_steps = T->max_steps;
    RP.max_depth = T->max_depth;
    RP.n_actions = T->n_actions;
    const int depth = T->depth, last_action = T->last_action;
    const StatesPtr parent = load_states(&T->parent);
    const StatesPtr leaf_out = load_states(&T->out);
    const StatesPtr sprime = load_states(&T->sprime);
    const bool write_leaf = (a == 0);
    const bool pair_out = has_states(sprime);
    // the optional per-pair outputs, tested once per tile rather than per round
    const bool pair_vals = T->r != nullptr || T->z != nullptr || T->U != nullptr || T->L != nullptr;
    // element-level expansion when the leaf is small enough for every
    // scenario to get a group of lanes of wavefront 0 (tile-uniform)
    int group_lanes = 0;
    if constexpr (Ops::kGroupRollout && kGroup) {
        const int G = pow2_at_least(M.h->n_peds > 0 ? M.h->n_peds : 1);
        if (n * G <= 64) group_lanes = G;
    }

    // -- gather + update + expand + bounds + rollouts (Eq. 10, 12, 13) ------
    // Every lane of a wavefront runs the same number of rounds, so a
    // 64-scenario chunk's reward (and, for small alphabets, its per-key
    // tables) are reduced by the whole wavefront right here.
    int my_exp = 0, my_roll = 0;
    typename Ops::WaveUpper wave_upper;
    for (int base = 0; base < n; base += nt) {
        const int k = base + tid;
        const bool valid = k < n;
        float r = 0.0f;
        uint64_t z = 0;
        uint32_t id = 0;
        typename Ops::State st;
        // gather + update + expansion step of one scenario
        auto expand_one = [&]() {
            // 32-bit unsigned offsets (positions are below 2^15, grouped-order
            // indices below 2^31) let the loads and stores take a scalar base
            const uint32_t p = (uint16_t)T->idx[(uint32_t)k];
            id = T->parent_ids[p];
            Ops::load(M, parent, p, st);
            if (last_action >= 0) {
                float r0;
                uint64_t z0;
                Ops::template step<false>(M, st, last_action, id, (uint32_t)(depth - 1), RP.k0, RP.k1, r0, z0);
            }
            if (write_leaf) {
                Ops::store(M, leaf_out, k, st);
                T->ids_out[k] = id;
            }
            my_exp += Ops::terminal(st) ? 0 : 1;
            Ops::template step<true>(M, st, a, id, (uint32_t)depth, RP.k0, RP.k1, r, z);
        };
        float U = 0.0f;
        float L = 0.0f;
        bool grouped = false;
        if constexpr (Ops::kGroupRollout && kGroup) {
            if (group_lanes > 0) {
                // n * G <= 64: one round; wavefront 0 expands the leaf with
                // one pedestrian per lane (leaf and stepped states stored
                // inside) and lane k receives scenario k's results
                grouped = true;
                if (wid == 0) {
                    const typename Ops::GroupOut o =
                        Ops::group_expand(M, RP, T->idx, T->parent_ids, parent, leaf_out, T->ids_out, sprime,
                                          write_leaf, pair_out, a, depth, last_action, n, group_lanes);
                    if (valid) {
                        r = o.r;
                        z = o.z;
                        U = o.U;
                        L = o.L;
                        id = o.id;
                        my_exp += o.expanded;
                        my_roll += o.steps;
                    }
                }
            }
        }
        if (!grouped) {
            if constexpr (Ops::kWaveUpper) {
                // every lane of the wavefront takes part in the bound (it
                // shares per-rock terms across lanes); lanes past n stay
                // terminal
                Ops::make_terminal(st);
                if (valid) expand_one();
                U = Ops::upper_wave(M, st, wave_upper);
            } else if (valid) {
                expand_one();
                U = Ops::upper(M, st);
            }
        }
        if (valid) {
            const int64_t pk = (int64_t)a * n + k;
            if (!grouped) {
                if (pair_out) Ops::store(M, sprime, pk, st);
                int ns = 0;
                L = rollout<Ops>(M, RP, st, id, depth + 1, ns);
                my_roll += ns;
            }
            if constexpr (!Ops::kSmallObs) {
                zk[k] = z;
                ub[k] = U;
                lb[k] = L;
            }
            if (pair_vals) {
                if (T->r) T->r[pk] = r;
                if (T->z) T->z[pk] = z;
                if (T->U) T->U[pk] = U;
                if (T->L) T->L[pk] = L;
            }
        }
        const bool chunk_live = base + wid * 64 < n;  // wavefront-uniform
        if constexpr (Ops::kSmallObs) {
            // this chunk's scenarios by key: counts, ranks, and the U and L
            // sums of each key present (keys in order of first appearance)
            if (chunk_live) {
                const int t = (base >> 6) + wid;
                const uint32_t key = valid ? (uint32_t)z : 0xFFFFFFFFu;
                uint64_t rem = __ballot(valid);
                uint32_t present = 0;
                int rank = 0;
                while (rem) {
                    const int leader = __ffsll((unsigned long long)rem) - 1;
                    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
                    const bool mine = key == v;
                    const uint64_t bv = __ballot(mine);
                    // lanes below this one with the same key
                    const int below = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(bv >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bv, 0u));
                    if (mine) rank = below;
                    const float su = wave_total(mine ? U : 0.0f);
                    const float sl = wave_total(mine ? L : 0.0f);
                    if (lane == 0) {
                        kc[t * 32 + v] = __popcll(bv);
                        ku[t * 32 + v] = su;
                        kl[t * 32 + v] = sl;
                    }
                    present |= 1u << v;
                    rem &= ~bv;
                }
                if (lane == 0) kmask[t] = present;
                if (valid) kchild[k] = (int16_t)(key | ((uint32_t)rank << 5));
            }
        }
        // mean step reward: sum of this 64-scenario chunk (lanes past n add 0;
        // a chunk without a reward sums to +0 without the reduction)
        const float r_chunk = __ballot(r != 0.0f) ? wave_total(r) : 0.0f;
        if (lane == 0 && chunk_live) chunk_r[(base >> 6) + wid] = r_chunk;
    }
    my_exp = wave_total_i(my_exp);
    my_roll = wave_total_i(my_roll);
    if (lane == 0) {
        atomicAdd(&stepc[0], (unsigned long long)my_exp);
        atomicAdd(&stepc[1], (unsigned long long)my_roll);
    }

    int D;
    if constexpr (Ops::kSmallObs) {
        // -- small observation alphabet: children from the per-chunk key tables --
        // Lane v of wavefront 0 owns key v: its scenario count (turning the
        // per-chunk counts into prefixes over chunks) and its U and L sums,
        // chunk partials added in chunk order.  A present key's child index
        // is the number of present keys below it (ascending observation).
        __syncthreads();
        const int nch = (n + 63) >> 6;
        if (wid == 0) {
            const uint32_t v = (uint32_t)lane;
            int run = 0;
            float tu = 0.0f, tl = 0.0f;
            // every chunk's entries are read (an absent key's entry is left
            // from an earlier tile and discarded), so the reads of several
            // chunks are in flight together; an entry is rewritten to the
            // key's count in earlier chunks
            const int e = (int)(v & 31u);
#pragma unroll 4
            for (int t = 0; t < nch; ++t) {
                const bool has = lane < 32 && ((kmask[t] >> e) & 1u);
                const int c = kc[t * 32 + e];
                const float fu = ku[t * 32 + e], fl = kl[t * 32 + e];
                if (has) {
                    kc[t * 32 + e] = run;
                    run += c;
                    tu = tu + fu;
                    tl = tl + fl;
                }
            }
            const bool present = run > 0;
            const uint32_t mask = (uint32_t)__ballot(present);
            D = __popc(mask);
            const int ci = lane < 32 ? __popc(mask & ((1u << v) - 1u)) : 0;
            // inclusive prefix over lanes 0-31: shifts inside rows of 16
            // lanes, then row 0's total broadcast into row 1 (lanes past 31
            // hold 0 counts and are not read)
            int incl = run;
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, true);  // row_shr:1
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, true);  // row_shr:2
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, true);  // row_shr:4
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, true);  // row_shr:8
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xa, 0xf, true);  // row_bcast:15
            const int off_v = incl - run;
            if (lane < 32) {
                koff[v] = off_v;
                kci[v] = ci;
            }
            if (present && ci < cap) {
                const int64_t o = (int64_t)a * cap + ci;
                T->child_z[o] = (uint64_t)v;
                T->child_n[o] = run;
                T->child_off[o] = off_v;
                T->child_u0[o] = tu / (float)run;
                T->child_l0[o] = tl / (float)run;
            }
            if (lane == 0) {
                T->n_children[a] = D;
                float tr = 0.0f;
                for (int t = 0; t < nch; ++t) tr = tr + chunk_r[t];
                T->r_mean[a] = n > 0 ? tr / (float)n : 0.0f;
                T->steps[2 * a + 0] = (int64_t)stepc[0];
                T->steps[2 * a + 1] = (int64_t)stepc[1];
            }
        }
        __syncthreads();
        // grouped order: a scenario's place is its child's offset, plus the
        // key's count in earlier chunks, plus its rank inside its chunk
        int32_t *const child_of = T->child_of;
        for (int k = tid; k < n; k += nt) {
            const int32_t cw = kchild[k];
            const int v = cw & 31;
            T->perm[(uint32_t)(a * n + koff[v] + kc[(k >> 6) * 32 + v] + (cw >> 5))] = (int16_t)k;
            if (child_of) child_of[(uint32_t)(a * n + k)] = kci[v];
        }
        __syncthreads();  // LDS is reused by the next tile
        return;
    } else {
        // -- LDS hash of the observations ----------------------------------------
        for (int k = tid; k < n; k += nt) {
            const uint64_t z = zk[k];
            int slot;
            if (z == kEmptyKey) {
                slot = H;
                misc[1] = 1;
            } else {
                int h = (int)(mix_key(z) & (uint64_t)(H - 1));
                for (;;) {
                    const unsigned long long old = atomicCAS((unsigned long long *)&tab[h], kEmptyKey, z);
                    if (old == kEmptyKey || old == z) break;
                    h = (h + 1) & (H - 1);
                }
                slot = h;
            }
            child[k] = slot;
        }
        __syncthreads();

        // -- distinct observations, sorted ascending -----------------------------
        uint64_t *dkey = zk;
        for (int h = tid; h <= H; h += nt) {
            const bool occupied = (h < H) ? (tab[h] != kEmptyKey) : (misc[1] != 0);
            if (occupied) {
                const int i = atomicAdd(&misc[0], 1);
                dkey[i] = (h < H) ? tab[h] : kEmptyKey;
                dslot[i] = (uint32_t)h;
            }
        }
        __syncthreads();
        D = misc[0];
        if (D <= 64) {
            if (wid == 0) wave_sort_pairs(dkey, dslot, D);
            __syncthreads();
        } else {
            const int p = pow2_at_least(D);
            for (int i = D + tid; i < p; i += nt) {
                dkey[i] = kEmptyKey;
                dslot[i] = 0xFFFFFFFFu;
            }
            __syncthreads();
            block_sort_pairs(dkey, dslot, p);
        }

        // -- child index of each scenario -----------------------------------------
        // rank_of_slot overlays the hash table; the distinct keys stay in zkey
        int32_t *rank_of_slot = (int32_t *)tab;
        for (int i = tid; i < D; i += nt) {
            rank_of_slot[dslot[i]] = i;
            if (i < cap) T->child_z[(int64_t)a * cap + i] = dkey[i];
        }
        if (tid == 0) T->n_children[a] = D;
        __syncthreads();
        for (int k = tid; k < n; k += nt) {
            const int c = rank_of_slot[child[k]];
            child[k] = c;
            if (T->child_of) T->child_of[(int64_t)a * n + k] = c;
        }
        __syncthreads();

    }

    // -- stable grouping: position of each scenario in perm --------------------
    const int nchunks = (n + 63) >> 6;
    if ((int64_t)nchunks * D <= Ly.table_cap) {
        for (int i = tid; i < nchunks * D; i += nt) cnt[i] = 0;
        __syncthreads();
        for (int t = wid; t < nchunks; t += nw) {
            const int k = t * 64 + lane;
            const bool valid = k < n;
            const int c = valid ? child[k] : -1;
            uint64_t rem = __ballot(valid);
            int myrank = 0;
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int cl = __shfl(c, leader, 64);
                const uint64_t m = __ballot(valid && c == cl);
                if (valid && c == cl) myrank = __popcll(m & __lanemask_lt());
                if (lane == leader) cnt[t * D + cl] = __popcll(m);
                rem &= ~m;
            }
            if (valid) child[k] = c | (myrank << 16);
        }
        __syncthreads();
        if (D <= 64) {
            // one wavefront: lane c turns child c's chunk counts into an
            // exclusive prefix, then the child offsets are a lane scan
            if (wid == 0) {
                int run = 0;
                if (lane < D)
                    for (int t = 0; t < nchunks; ++t) {
                        const int v = cnt[t * D + lane];
                        cnt[t * D + lane] = run;
                        run += v;
                    }
                int incl = run;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int o = __shfl_up(incl, d, 64);
                    if (lane >= d) incl += o;
                }
                if (lane < D) {
                    nc[lane] = run;
                    off[lane] = incl - run;
                }
            }
            __syncthreads();
        } else {
            for (int c = tid; c < D; c += nt) {
                int run = 0;
                for (int t = 0; t < nchunks; ++t) {
                    const int v = cnt[t * D + c];
                    cnt[t * D + c] = run;
                    run += v;
                }
                nc[c] = run;
                off[c] = run;
            }
            __syncthreads();
            block_exclusive_scan(off, D, scan_scratch);
        }
        for (int k = tid; k < n; k += nt) {
            const int cw = child[k];
            const int c = cw & 0xFFFF;
            permb[off[c] + cnt[(k >> 6) * D + c] + (cw >> 16)] = k;
            child[k] = c;
        }
        __syncthreads();
    } else {
        uint32_t *comp = (uint32_t *)permb;
        const int p = pow2_at_least(n);
        for (int i = tid; i < p; i += nt) comp[i] = (i < n) ? (((uint32_t)child[i] << 16) | (uint32_t)i) : 0xFFFFFFFFu;
        __syncthreads();
        block_sort_u32(comp, p);
        for (int i = tid; i < n; i += nt) {
            const uint32_t v = comp[i];
            const int c = (int)(v >> 16);
            if (i == 0 || (comp[i - 1] >> 16) != (uint32_t)c) off[c] = i;
        }
        __syncthreads();
        for (int c = tid; c < D; c += nt) nc[c] = ((c + 1 < D) ? off[c + 1] : n) - off[c];
        __syncthreads();
        for (int i = tid; i < n; i += nt) permb[i] = (int32_t)(comp[i] & 0xFFFFu);
        __syncthreads();
    }
    for (int i = tid; i < n; i += nt) T->perm[(int64_t)a * n + i] = (int16_t)permb[i];
    for (int c = tid; c < D && c < cap; c += nt) {
        T->child_n[(int64_t)a * cap + c] = nc[c];
        T->child_off[(int64_t)a * cap + c] = off[c];
    }

    // -- per-child sums: segmented wavefront scans over the grouped order ------
    float *su = (float *)(lds + Ly.zkey);  // keys, table and counts are done
    float *sl = su + Ly.p2;
    for (int t = wid; t < nchunks; t += nw) {
        const int i = t * 64 + lane;
        const bool valid = i < n;
        const int k = valid ? permb[i] : 0;
        float vu = valid ? ub[k] : 0.0f;
        float vl = valid ? lb[k] : 0.0f;
        const int c = valid ? child[k] : -1;
        const int c_prev = __shfl_up(c, 1, 64);
        bool head = (lane == 0) || (c_prev != c);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const float ou = __shfl_up(vu, d, 64);
            const float ol = __shfl_up(vl, d, 64);
            const int oh = __shfl_up((int)head, d, 64);
            if (lane >= d && !head) {
                vu = ou + vu;
                vl = ol + vl;
                head = oh != 0;
            }
        }
        if (valid) {
            su[i] = vu;
            sl[i] = vl;
        }
    }
    __syncthreads();
    for (int c = tid; c < D && c < cap; c += nt) {
        const int start = off[c], end = start + nc[c];
        float tu = 0.0f, tl = 0.0f;
        for (int t = start >> 6; t <= (end - 1) >> 6; ++t) {
            const int e = min(end, (t + 1) * 64) - 1;
            tu = tu + su[e];
            tl = tl + sl[e];
        }
        T->child_u0[(int64_t)a * cap + c] = tu / (float)nc[c];
        T->child_l0[(int64_t)a * cap + c] = tl / (float)nc[c];
    }
    if (tid == 0) {
        float tr = 0.0f;
        for (int t = 0; t < nchunks; ++t) tr = tr + chunk_r[t];
        T->r_mean[a] = n > 0 ? tr / (float)n : 0.0f;
        T->steps[2 * a + 0] = (int64_t)stepc[0];
        T->steps[2 * a + 1] = (int64_t)stepc[1];
    }
    __syncthreads();  // LDS is reused by the next tile
}

// One (leaf, action) tile of a model whose observation keys are all below
// kMedKeys (navigation: 8 reading bits, or the terminal key 256), for
// leaves of up to kMaxMedLeaf scenarios.  No hash table and no sort: every
// key is its own table index.
//  - ranks: the 64-scenario chunks are split into contiguous runs, one per
//    wavefront; a wavefront walks its run in order and keeps a running count
//    per key, so a scenario's rank is the count of its key in earlier chunks
//    of the run plus the lanes below it in its chunk with the same key;
//  - a key's count in earlier runs, its child offset (ascending key) and its
//    child index come from prefix sums over the runs and over the keys;
//  - the per-child U and L sums are the same segmented scans over 64-aligned
//    chunks of the grouped order as in the hashed path, chunk partials added
//    in chunk order, so both paths give identical results for a leaf either
//    can expand.
// kGroup: the kernel-argument launches (a search's small leaves) roll out
// with the map held as bits in registers (NavOps::rollout_grid).
template <class Ops, bool kGroup>
__device__ void run_tile_med(const HDX_CONST LeafTask *T, const int a, unsigned char *lds, const MedLayout &Ly) {
    static_assert(Ops::kTerminalObs < (uint64_t)kMedKeys, "observation keys exceed the medium alphabet");
    float *gpow_lds = (float *)(lds + Ly.gpow);
    const MView M = make_view(T->model, gpow_lds);
    const int n = T->n;
    const int cap = T->cap;
    const int tid = threadIdx.x, nt = blockDim.x, lane = lane_id(), wid = tid >> 6, nw = nt >> 6;
    uint16_t *keyb = (uint16_t *)(lds + Ly.key);
    uint16_t *rnk = (uint16_t *)(lds + Ly.rank);
    float *ub = (float *)(lds + Ly.ub);
    float *lb = (float *)(lds + Ly.lb);
    int16_t *permb = (int16_t *)(lds + Ly.perm);
    float *su = (float *)(lds + Ly.su);
    float *sl = (float *)(lds + Ly.sl);
    int32_t *wcnt = (int32_t *)(lds + Ly.wcnt);
    int32_t *kcnt = (int32_t *)(lds + Ly.kcnt);
    int32_t *koff = (int32_t *)(lds + Ly.koff);
    int32_t *kci = (int32_t *)(lds + Ly.kci);
    int32_t *cof = (int32_t *)(lds + Ly.cof);
    int32_t *cnc = (int32_t *)(lds + Ly.cnc);
    float *chunk_r = (float *)(lds + Ly.chunk_r);
    int32_t *misc = (int32_t *)(lds + Ly.misc);
    unsigned long long *stepc = (unsigned long long *)(misc + 4);  // expansion, rollout steps
    int32_t *scan_scratch = misc + 16;
    const int nch = (n + 63) >> 6;
    const int run_len = nch > 0 ? (nch + nw - 1) / nw : 1;  // chunks per wavefront run
    const int runs = (nch + run_len - 1) / run_len;        // <= min(nw, nch)

    for (int i = tid; i < runs * kMedKeys; i += nt) wcnt[i] = 0;
    if (tid == 0) {
        stepc[0] = 0;
        stepc[1] = 0;
    }
    stage_gpow(T->model, gpow_lds);
    stage_cells(T->model, gpow_lds);
    __syncthreads();

    RolloutParams RP;
    RP.k0 = T->k0;
    RP.k1 = T->k1;
    RP.policy = T->policy;
    RP.const_action = T->const_action;
    RP.max_steps = T->max_steps;
    RP.max_depth = T->max_depth;
    RP.n_actions = T->n_actions;
    const int depth = T->depth, last_action = T->last_action;
    const StatesPtr parent = load_states(&T->parent);
    const StatesPtr leaf_out = load_states(&T->out);
    const StatesPtr sprime = load_states(&T->sprime);
    const bool write_leaf = (a == 0);
    const bool pair_out = has_states(sprime);
    // the optional per-pair outputs, tested once per tile rather than per round
    const bool pair_vals = T->r != nullptr || T->z != nullptr || T->U != nullptr || T->L != nullptr;

    // -- gather + update + expand + bounds + rollouts (Eq. 10, 12, 13) ------
    int my_exp = 0, my_roll = 0;
    for (int base = 0; base < n; base += nt) {
        const int k = base + tid;
        const bool valid = k < n;
        float r = 0.0f;
        if (valid) {
            const int p = T->idx[k];
            const uint32_t id = T->parent_ids[p];
            typename Ops::State st;
            Ops::load(M, parent, p, st);
            if (last_action >= 0) {
                float r0;
                uint64_t z0;
                Ops::template step<false>(M, st, last_action, id, (uint32_t)(depth - 1), RP.k0, RP.k1, r0, z0);
            }
            if (write_leaf) {
                Ops::store(M, leaf_out, k, st);
                T->ids_out[k] = id;
            }
            my_exp += Ops::terminal(st) ? 0 : 1;
            uint64_t z;
            Ops::template step<true>(M, st, a, id, (uint32_t)depth, RP.k0, RP.k1, r, z);
            const float U = Ops::upper(M, st);
            const int64_t pk = (int64_t)a * n + k;
            if (pair_out) Ops::store(M, sprime, pk, st);
            int ns = 0;
            float L;
            if constexpr (kGroup)
                L = Ops::rollout_grid(M, RP, st, id, depth + 1, ns);
            else
                L = rollout<Ops>(M, RP, st, id, depth + 1, ns);
            my_roll += ns;
            keyb[k] = (uint16_t)z;
            ub[k] = U;
            lb[k] = L;
            if (pair_vals) {
                if (T->r) T->r[pk] = r;
                if (T->z) T->z[pk] = z;
                if (T->U) T->U[pk] = U;
                if (T->L) T->L[pk] = L;
            }
        }
        // mean step reward: sum of this 64-scenario chunk (lanes past n add 0;
        // a chunk without a reward sums to +0 without the reduction)
        const float r_chunk = __ballot(r != 0.0f) ? wave_total(r) : 0.0f;
        if (lane == 0 && base + wid * 64 < n) chunk_r[(base >> 6) + wid] = r_chunk;
    }
    my_exp = wave_total_i(my_exp);
    my_roll = wave_total_i(my_roll);
    if (lane == 0) {
        atomicAdd(&stepc[0], (unsigned long long)my_exp);
        atomicAdd(&stepc[1], (unsigned long long)my_roll);
    }
    __syncthreads();

    // -- ranks inside each wavefront's run of chunks ----------------------------
    if (wid < runs) {
        int32_t *cw = wcnt + wid * kMedKeys;
        const int t_end = min(nch, (wid + 1) * run_len);
        for (int t = wid * run_len; t < t_end; ++t) {
            const int k = t * 64 + lane;
            const bool valid = k < n;
            const uint32_t key = valid ? keyb[k] : 0xFFFFFFFFu;
            uint64_t rem = __ballot(valid);
            int rank = 0;
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
                const bool mine = key == v;
                const uint64_t bv = __ballot(mine);
                const int before = cw[v];  // one address: a broadcast read
                if (mine) rank = before + __popcll(bv & __lanemask_lt());
                if (lane == leader) cw[v] = before + __popcll(bv);
                rem &= ~bv;
            }
            if (valid) rnk[k] = (uint16_t)rank;
        }
    }
    __syncthreads();

    // -- per key: count in earlier runs, total, child offset and index ----------
    // koff packs the count (low 16 bits, at most kMaxMedLeaf) and presence
    // (high bits) so one exclusive scan gives both the offset and the index.
    for (int v = tid; v < kMedKeys; v += nt) {
        int run = 0;
        for (int w = 0; w < runs; ++w) {
            const int c = wcnt[w * kMedKeys + v];
            wcnt[w * kMedKeys + v] = run;
            run += c;
        }
        kcnt[v] = run;
        koff[v] = run + (run > 0 ? (1 << 16) : 0);
    }
    __syncthreads();
    block_exclusive_scan(koff, kMedKeys, scan_scratch);
    const int last = kMedKeys - 1;
    const int D = (koff[last] >> 16) + (kcnt[last] > 0 ? 1 : 0);
    for (int v = tid; v < kMedKeys; v += nt) {
        const int packed = koff[v];
        const int c = kcnt[v];
        const int o = packed & 0xFFFF, ci = packed >> 16;
        koff[v] = o;
        kci[v] = ci;
        if (c > 0) {
            cof[ci] = o;
            cnc[ci] = c;
            if (ci < cap) {
                const int64_t q = (int64_t)a * cap + ci;
                T->child_z[q] = (uint64_t)v;
                T->child_n[q] = c;
                T->child_off[q] = o;
            }
        }
    }
    if (tid == 0) T->n_children[a] = D;
    __syncthreads();

    // -- grouped order: child offset + count in earlier runs + rank -------------
    for (int k = tid; k < n; k += nt) {
        const int v = keyb[k];
        const int w = (k >> 6) / run_len;
        permb[koff[v] + wcnt[w * kMedKeys + v] + rnk[k]] = (int16_t)k;
        if (T->child_of) T->child_of[(int64_t)a * n + k] = kci[v];
    }
    __syncthreads();
    for (int i = tid; i < n; i += nt) T->perm[(int64_t)a * n + i] = permb[i];

    // -- per-child sums: segmented wavefront scans over the grouped order ------
    for (int t = wid; t < nch; t += nw) {
        const int i = t * 64 + lane;
        const bool valid = i < n;
        const int k = valid ? permb[i] : 0;
        float vu = valid ? ub[k] : 0.0f;
        float vl = valid ? lb[k] : 0.0f;
        const int c = valid ? (int)keyb[k] : -1;
        const int c_prev = __shfl_up(c, 1, 64);
        bool head = (lane == 0) || (c_prev != c);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const float ou = __shfl_up(vu, d, 64);
            const float ol = __shfl_up(vl, d, 64);
            const int oh = __shfl_up((int)head, d, 64);
            if (lane >= d && !head) {
                vu = ou + vu;
                vl = ol + vl;
                head = oh != 0;
            }
        }
        if (valid) {
            su[i] = vu;
            sl[i] = vl;
        }
    }
    __syncthreads();
    for (int c = tid; c < D && c < cap; c += nt) {
        const int start = cof[c], end = start + cnc[c];
        float tu = 0.0f, tl = 0.0f;
        for (int t = start >> 6; t <= (end - 1) >> 6; ++t) {
            const int e = min(end, (t + 1) * 64) - 1;
            tu = tu + su[e];
            tl = tl + sl[e];
        }
        T->child_u0[(int64_t)a * cap + c] = tu / (float)cnc[c];
        T->child_l0[(int64_t)a * cap + c] = tl / (float)cnc[c];
    }
    if (tid == 0) {
        float tr = 0.0f;
        for (int t = 0; t < nch; ++t) tr = tr + chunk_r[t];
        T->r_mean[a] = n > 0 ? tr / (float)n : 0.0f;
        T->steps[2 * a + 0] = (int64_t)stepc[0];
        T->steps[2 * a + 1] = (int64_t)stepc[1];
    }
    __syncthreads();  // LDS is reused by the next tile
}

template <int PM, bool kGroup>
__device__ __forceinline__ void run_ped(const HDX_CONST LeafTask *T, int a, unsigned char *lds, const LdsLayout &Ly) {
    run_tile<PedOps<PM>, kGroup>(T, a, lds, Ly);
}

__device__ __forceinline__ int remap_xcd(int b, int grid) {
    // workgroups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous run of tiles so the tiles of one leaf share an L2
    const int x = b & 7, slot = b >> 3, base = grid >> 3, extra = grid & 7;
    return x * base + min(x, extra) + slot;
}

// MODE 0: RockSample only; 1: crowd driving only; 2: both; 3: multi-agent
// RockSample only; 4: navigation only.  Workgroups of the driving model are
// capped at 256 lanes so its per-lane state can stay in registers;
// navigation (83 registers) takes up to 1024, because one large leaf's LDS
// carve-up leaves room for one workgroup per CU.
template <int MODE>
constexpr bool small_obs_mode() { return MODE == 0 || MODE == 3; }
template <int MODE>
constexpr int max_threads() { return small_obs_mode<MODE>() ? 512 : MODE == 4 ? 1024 : 256; }
// RockSample tiles: keep 7 wavefronts per SIMD resident (at most 72 VGPRs,
// no spills); the driving model's register state decides its own.
template <int MODE>
constexpr int min_waves() { return small_obs_mode<MODE>() ? 7 : 1; }

template <int MODE, int PM, bool kGroup = false>
__device__ __forceinline__ void run_mode(const HDX_CONST LeafTask *T, int a, unsigned char *lds, const LdsLayout &Ly) {
    if (MODE == 3) {
        run_tile<MarsOps>(T, a, lds, Ly);
    } else if (MODE == 4) {
        run_tile_med<NavOps, kGroup>(T, a, lds, make_med_layout(Ly.np));
    } else if (MODE == 0 || (MODE == 2 && T->kind == HDX_ROCKSAMPLE)) {
        run_tile<RsOps>(T, a, lds, Ly);
    } else {
        run_ped<PM, kGroup>(T, a, lds, Ly);
    }
}

template <int MODE, int PM, bool kGroup = false>
__global__ __launch_bounds__(max_threads<MODE>(), min_waves<MODE>()) void expand_tiles(const LeafTask *tasks,
                                                                                       const Tile *tiles,
                                                                                       TileQueue *queue,
                                                                                       int32_t n_max,
                                                                                       int32_t persistent,
                                                                                       int32_t xcd_remap) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int32_t s_tile;
    const LdsLayout Ly = make_layout(n_max, small_obs_mode<MODE>());
    const int32_t n_tiles = __builtin_amdgcn_readfirstlane(queue->n_tiles);
    int iter = 0;
    for (;;) {
        int t;
        if (persistent) {
            if (threadIdx.x == 0) s_tile = atomicAdd(&queue->next, 1);
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(s_tile);
            __syncthreads();
        } else {
            if (iter > 0) break;
            t = xcd_remap ? remap_xcd((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
        }
        ++iter;
        if (t >= n_tiles) break;
        const HDX_CONST Tile *tile = (const HDX_CONST Tile *)(tiles + t);
        const HDX_CONST LeafTask *T = (const HDX_CONST LeafTask *)(tasks + tile->leaf);
        run_mode<MODE, PM, kGroup>(T, tile->action, lds, Ly);
    }
    if (persistent && threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue->done, 1) == (int)gridDim.x - 1) {
            queue->next = 0;
            queue->done = 0;
            __threadfence();
        }
    }
}

// A few leaves carried in the kernel arguments: no descriptor staging, so
// the launch is ordered by its stream alone.  The pack is read in place in
// the kernarg segment (constant address space, scalar loads).
template <int MODE, int PM>
__global__ __launch_bounds__(max_threads<MODE>()) void expand_args(const ArgPack pack) {
    extern __shared__ __align__(16) unsigned char lds[];
#if defined(__HIP_DEVICE_COMPILE__)
    const HDX_CONST ArgPack *P = (const HDX_CONST ArgPack *)__builtin_amdgcn_kernarg_segment_ptr();
#else
    const ArgPack *P = &pack;
#endif
    const LdsLayout Ly = make_layout(P->n_max, small_obs_mode<MODE>());
    const int n_leaves = P->n_leaves;
    const int n_tiles = P->tile_begin[n_leaves];
    const int t = P->xcd_remap ? remap_xcd((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    if (t >= n_tiles) return;
    int i = 0;
    while (i + 1 < n_leaves && t >= P->tile_begin[i + 1]) ++i;
    const HDX_CONST LeafTask *T = &P->t[i];
    run_mode<MODE, PM, true>(T, t - P->tile_begin[i], lds, Ly);
}

// Dynamic LDS of one workgroup for leaves of up to n_max scenarios.
template <int MODE>
uint32_t lds_bytes(int32_t n_max) {
    return MODE == 4 ? make_med_layout(n_max).total : make_layout(n_max, small_obs_mode<MODE>()).total;
}

template <int MODE, int PM>
hipError_t configure_t() {
    hipError_t e = hipFuncSetAttribute((const void *)expand_tiles<MODE, PM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_dynamic_lds());
    if (e != hipSuccess) return e;
    if (MODE == 1) {
        e = hipFuncSetAttribute((const void *)expand_tiles<MODE, PM, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                max_dynamic_lds());
        if (e != hipSuccess) return e;
    }
    return hipFuncSetAttribute((const void *)expand_args<MODE, PM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               max_dynamic_lds());
}

template <int MODE, int PM>
hipError_t launch_args_t(const ArgPack &pack, const Schedule &sch, hipStream_t stream) {
    const int grid = pack.tile_begin[pack.n_leaves];
    if (grid < 1) return hipSuccess;
    const int threads = sch.threads > max_threads<MODE>() ? max_threads<MODE>() : sch.threads;
    hipLaunchKernelGGL((expand_args<MODE, PM>), dim3(grid), dim3(threads), lds_bytes<MODE>(pack.n_max), stream,
                       pack);
    return hipGetLastError();
}

template <int MODE, int PM, bool kGroup = false>
hipError_t launch_expand_t(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queue, int32_t n_tiles,
                           int32_t n_max, const Schedule &sch, int32_t n_cu, hipStream_t stream) {
    // persistent: a fixed grid that drains the tile queue, so a captured
    // graph stays valid for any tile count
    const int grid = sch.persistent > 0 ? n_cu * sch.persistent : n_tiles;
    if (grid < 1) return hipSuccess;
    const int threads = sch.threads > max_threads<MODE>() ? max_threads<MODE>() : sch.threads;
    hipLaunchKernelGGL((expand_tiles<MODE, PM, kGroup>), dim3(grid), dim3(threads), lds_bytes<MODE>(n_max), stream, d_tasks,
                       d_tiles, d_queue, n_max, sch.persistent > 0 ? 1 : 0, sch.xcd_remap);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sample_scenarios
// ---------------------------------------------------------------------------
// The arguments (belief thresholds, ~3.6 KB) are read from device memory.
__global__ void sample_kernel(const SampleArgs *args) {
    const HDX_CONST SampleArgs &A = *(const HDX_CONST SampleArgs *)args;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.K) return;
    const HDX_CONST ModelHdr *M = (const HDX_CONST ModelHdr *)&A.model->h;
    const StatesPtr &S = A.out;
    if (M->kind == HDX_ROCKSAMPLE) {
        int32_t w = A.x0 | (A.y0 << 5);
        uint4 u = make_uint4(0, 0, 0, 0);
        for (int i = 0; i < M->n_rocks; ++i) {
            if ((i & 3) == 0) u = philox((uint32_t)k, 0, (uint32_t)(i >> 2), kTagInit, A.k0, A.k1);
            const uint32_t word = (i & 3) == 0 ? u.x : (i & 3) == 1 ? u.y : (i & 3) == 2 ? u.z : u.w;
            if ((uint64_t)word < A.rock_thr[i]) w |= 1 << (10 + i);
        }
        S.w[k] = w;
    } else if (M->kind == HDX_MARS) {
        // the robots' row is known; rock i good as for RockSample
        int32_t rk = 0;
        uint4 u = make_uint4(0, 0, 0, 0);
        for (int i = 0; i < M->n_rocks; ++i) {
            if ((i & 3) == 0) u = philox((uint32_t)k, 0, (uint32_t)(i >> 2), kTagInit, A.k0, A.k1);
            const uint32_t word = (i & 3) == 0 ? u.x : (i & 3) == 1 ? u.y : (i & 3) == 2 ? u.z : u.w;
            if ((uint64_t)word < A.rock_thr[i]) rk |= 1 << i;
        }
        S.w[k] = A.x0;
        S.w[S.stride + k] = rk;
    } else if (M->kind == HDX_NAV) {
        // robot on row 0 at a uniform column; one gate open; other unknown
        // cells occupied at their prior (draw i = word i % 4 of block i / 4)
        uint4 u = philox((uint32_t)k, 0, 0, kTagInit, A.k0, A.k1);
        const int x = (int)(((uint64_t)u.x * (uint64_t)M->grid) >> 32);
        uint32_t m0 = u.y < 0x80000000u ? 2u : 1u, m1 = 0, m2 = 0, m3 = 0;
        for (int i = 2; i < A.n_unknown; ++i) {
            if ((i & 3) == 0) u = philox((uint32_t)k, 0, (uint32_t)(i >> 2), kTagInit, A.k0, A.k1);
            const uint32_t word = (i & 3) == 0 ? u.x : (i & 3) == 1 ? u.y : (i & 3) == 2 ? u.z : u.w;
            if ((uint64_t)word < A.cell_thr[i]) {
                const uint32_t bit = 1u << (i & 31);
                if (i < 32) m0 |= bit;
                else if (i < 64) m1 |= bit;
                else if (i < 96) m2 |= bit;
                else m3 |= bit;
            }
        }
        S.w[k] = x;
        S.w[S.stride + k] = (int32_t)m0;
        S.w[2 * S.stride + k] = (int32_t)m1;
        S.w[3 * S.stride + k] = (int32_t)m2;
        S.w[4 * S.stride + k] = (int32_t)m3;
    } else {
        S.s[k] = A.s0;
        S.car[k] = A.level0 & 0xff;
        uint4 u = make_uint4(0, 0, 0, 0);
        for (int j = 0; j < M->n_peds; ++j) {
            if ((j & 3) == 0) u = philox((uint32_t)k, 0, (uint32_t)(j >> 2), kTagInit, A.k0, A.k1);
            const uint32_t word = (j & 3) == 0 ? u.x : (j & 3) == 1 ? u.y : (j & 3) == 2 ? u.z : u.w;
            int g = M->n_goals - 1;
            for (int q = 0; q < M->n_goals - 1; ++q) {
                if ((uint64_t)word < A.goal_thr[j][q]) {
                    g = q;
                    break;
                }
            }
            S.px[j * S.stride + k] = A.px0[j];
            S.py[j * S.stride + k] = A.py0[j];
            S.goal[j * S.stride + k] = (uint8_t)g;
        }
    }
}

// ---------------------------------------------------------------------------
// rollout_bounds: one lane per state
// ---------------------------------------------------------------------------
template <class Ops>
__global__ __launch_bounds__(256) void bounds_kernel(const BoundsArgs A) {
    __shared__ float gpow_lds[kModelLdsFloats];
    stage_gpow(A.model, gpow_lds);
    if constexpr (std::is_same<Ops, NavOps>::value) stage_cells(A.model, gpow_lds);
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.n) return;
    const MView M = make_view(A.model, gpow_lds);
    typename Ops::State st;
    Ops::load(M, A.states, k, st);
    RolloutParams RP;
    RP.k0 = A.k0;
    RP.k1 = A.k1;
    RP.policy = A.policy;
    RP.const_action = A.const_action;
    RP.max_steps = A.max_steps;
    RP.max_depth = A.max_depth;
    RP.n_actions = M.h->n_actions;
    int ns = 0;
    A.U[k] = Ops::upper(M, st);
    A.L[k] = rollout<Ops>(M, RP, st, A.ids[k], A.depths[k], ns);
    if (A.steps) A.steps[k] = ns;
}

// FP32 rounding self-test: the operations the models' state updates use.
__global__ void fp32_selftest_kernel(const float *a, const float *b, const float *c, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = a[i], y = b[i], z = c[i];
    out[i] = __builtin_sqrtf(fabsf(x));
    out[n + i] = x / y;
    out[2 * n + i] = x * y + z;
    out[3 * n + i] = floorf(x);
}

__global__ void philox_kernel(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint4 c = reinterpret_cast<const uint4 *>(ctr)[i];
    reinterpret_cast<uint4 *>(out)[i] = philox(c.x, c.y, c.z, c.w, k0, k1);
}

}  // namespace

hipError_t launch_fp32_selftest(const float *a, const float *b, const float *c, int64_t n, float *out,
                                hipStream_t stream) {
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fp32_selftest_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, a, b, c, n, out);
    return hipGetLastError();
}

int32_t max_dynamic_lds() { return 160 * 1024 - 256; }

Variant pick_variant(int32_t has_rs, int32_t has_ped, int32_t ped_max, int32_t n_max, int32_t has_mars,
                     int32_t has_nav) {
    Variant v;
    v.mode = has_nav ? 4 : has_mars ? 3 : !has_ped ? 0 : (has_rs ? 2 : 1);
    v.pm = !has_ped ? 1 : ped_max <= 8 ? 8 : ped_max <= 16 ? 16 : 32;
    v.n_max = n_max < 1 ? 1 : n_max;
    return v;
}

int32_t variant_max_threads(const Variant &v) {
    return v.mode == 0 ? max_threads<0>() : v.mode == 3 ? max_threads<3>() : v.mode == 4 ? max_threads<4>()
                                                                            : max_threads<1>();
}

hipError_t configure_expand_kernels() {
    hipError_t e = configure_t<0, 1>();
    if (e == hipSuccess) e = configure_t<1, 8>();
    if (e == hipSuccess) e = configure_t<1, 16>();
    if (e == hipSuccess) e = configure_t<1, 32>();
    if (e == hipSuccess) e = configure_t<2, 8>();
    if (e == hipSuccess) e = configure_t<2, 16>();
    if (e == hipSuccess) e = configure_t<2, 32>();
    if (e == hipSuccess) e = configure_t<3, 1>();
    if (e == hipSuccess) e = configure_t<4, 1>();
    return e;
}

hipError_t launch_expand(const LeafTask *d_tasks, const Tile *d_tiles, TileQueue *d_queue, int32_t n_tiles,
                         const Variant &v, const Schedule &sch, int32_t n_cu, hipStream_t stream) {
#define HDX_LAUNCH(M, P) launch_expand_t<M, P>(d_tasks, d_tiles, d_queue, n_tiles, v.n_max, sch, n_cu, stream)
#define HDX_LAUNCH_G(P) launch_expand_t<1, P, true>(d_tasks, d_tiles, d_queue, n_tiles, v.n_max, sch, n_cu, stream)
    if (v.mode == 0) return HDX_LAUNCH(0, 1);
    if (v.mode == 3) return HDX_LAUNCH(3, 1);
    if (v.mode == 4) return HDX_LAUNCH(4, 1);
    if (v.mode == 1 && v.group)
        return v.pm == 8 ? HDX_LAUNCH_G(8) : v.pm == 16 ? HDX_LAUNCH_G(16) : HDX_LAUNCH_G(32);
    if (v.mode == 1) return v.pm == 8 ? HDX_LAUNCH(1, 8) : v.pm == 16 ? HDX_LAUNCH(1, 16) : HDX_LAUNCH(1, 32);
    return v.pm == 8 ? HDX_LAUNCH(2, 8) : v.pm == 16 ? HDX_LAUNCH(2, 16) : HDX_LAUNCH(2, 32);
#undef HDX_LAUNCH_G
#undef HDX_LAUNCH
}

hipError_t launch_expand_args(const ArgPack &pack, const Variant &v, const Schedule &sch, hipStream_t stream) {
#define HDX_LAUNCH(M, P) launch_args_t<M, P>(pack, sch, stream)
    if (v.mode == 0) return HDX_LAUNCH(0, 1);
    if (v.mode == 3) return HDX_LAUNCH(3, 1);
    if (v.mode == 4) return HDX_LAUNCH(4, 1);
    if (v.mode == 1) return v.pm == 8 ? HDX_LAUNCH(1, 8) : v.pm == 16 ? HDX_LAUNCH(1, 16) : HDX_LAUNCH(1, 32);
    return v.pm == 8 ? HDX_LAUNCH(2, 8) : v.pm == 16 ? HDX_LAUNCH(2, 16) : HDX_LAUNCH(2, 32);
#undef HDX_LAUNCH
}

hipError_t launch_sample(const SampleArgs *d_args, int32_t K, hipStream_t stream) {
    const int threads = 256;
    const int blocks = (K + threads - 1) / threads;
    if (blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks), dim3(threads), 0, stream, d_args);
    return hipGetLastError();
}

hipError_t launch_bounds(const BoundsArgs &args, int32_t kind, int32_t n_peds, hipStream_t stream) {
    const int threads = 256;
    const int64_t blocks = (args.n + threads - 1) / threads;
    if (blocks == 0) return hipSuccess;
    if (kind == HDX_ROCKSAMPLE) {
        hipLaunchKernelGGL(bounds_kernel<RsOps>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    } else if (kind == HDX_MARS) {
        hipLaunchKernelGGL(bounds_kernel<MarsOps>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    } else if (kind == HDX_NAV) {
        hipLaunchKernelGGL(bounds_kernel<NavOps>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    } else if (n_peds <= 8) {
        hipLaunchKernelGGL(bounds_kernel<PedOps<8>>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    } else if (n_peds <= 16) {
        hipLaunchKernelGGL(bounds_kernel<PedOps<16>>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    } else {
        hipLaunchKernelGGL(bounds_kernel<PedOps<32>>, dim3((unsigned)blocks), dim3(threads), 0, stream, args);
    }
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t *out,
                         hipStream_t stream) {
    const int threads = 256;
    const int64_t blocks = (count + threads - 1) / threads;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, ctr, count, k0, k1, out);
    return hipGetLastError();
}

}  // namespace hdx
