// Parallel DESPOT search on the CPU feeding leaf expansion to the GPU
// (HyP-DESPOT, Sec. III-A and III-C).  Several host threads share one tree
// without a tree-wide lock (descents read bounds as they stand, a leaf is
// claimed by an atomic state change, each backup step locks one node):
// each trial walks down by the scenario-based PO-UCT action bound (Eq. 8)
// and the weighted excess uncertainty with virtual loss (Eq. 7, 9), expands
// the leaf it reaches through hdx_expand_leaf (Eq. 10-13), attaches the
// children (Eq. 11) and backs the bounds up to the root (Eq. 4).  Node
// states stay on the device: a node's scenarios are a segment of its
// parent's grouped order, and its own states are materialised when it is
// expanded.
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <limits>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Offsets of one expansion record (device arena).  The head block holds
// what the host needs to build nodes and is copied back in one transfer.
struct RecLayout {
    size_t n_children, r_mean, steps, child_z, child_n, child_off, child_u0, child_l0, head;
    size_t w, s, car, px, py, goal, ids, perm, total;
};

RecLayout rec_layout(const hdx_model_desc &d, int n, int cap) {
    RecLayout L;
    const int A = d.n_actions;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align16(o + bytes);
        return at;
    };
    L.n_children = take(4ull * A);
    L.r_mean = take(4ull * A);
    L.steps = take(16ull * A);
    L.child_z = take(8ull * A * cap);
    L.child_n = take(4ull * A * cap);
    L.child_off = take(4ull * A * cap);
    L.child_u0 = take(4ull * A * cap);
    L.child_l0 = take(4ull * A * cap);
    L.head = o;
    L.w = L.s = L.car = L.px = L.py = L.goal = 0;
    if (d.kind == HDX_ROCKSAMPLE) {
        L.w = take(4ull * n);
    } else if (d.kind == HDX_MARS) {
        L.w = take(8ull * n);  // robots' row, then rocks' row
    } else if (d.kind == HDX_NAV) {
        L.w = take(20ull * n);  // robot row, then four rows of unknown cells
    } else {
        L.s = take(4ull * n);
        L.car = take(4ull * n);
        L.px = take(4ull * d.n_peds * n);
        L.py = take(4ull * d.n_peds * n);
        L.goal = take(1ull * d.n_peds * n);
    }
    L.ids = take(4ull * n);
    L.perm = take(2ull * A * n);
    L.total = o;
    return L;
}

struct Rec {
    char *dev = nullptr;
    RecLayout L;
    int n = 0;
};

// One belief node.  The fields above `u` are written once, before the node
// is published (its parent's state becomes 2 with a release store), and
// read freely afterwards.  u and l, and the sums of the node's actions, are
// recomputed under the node's own lock (`lock`) and read without it; a
// reader sees the old or the new value of each.
struct Node {
    int32_t parent = -1;
    int32_t action = -1;  // action from the parent
    int32_t n = 0;        // |Phi_b|
    int32_t depth = 0;
    int32_t parent_rec = -1;           // record holding the parent's states
    const int16_t *idx_dev = nullptr;  // positions in that record
    int32_t act_begin = -1;            // set by the expanding thread before state becomes 2
    int32_t rec = -1;                  // likewise
    std::atomic<double> u{0.0}, l{0.0};
    std::atomic<int32_t> state{0};  // 0 leaf, 1 being expanded, 2 expanded
    std::atomic<int32_t> visits{0}, vloss{0};
    std::atomic<int32_t> lock{0};
    Node(int32_t parent_, int32_t action_, int32_t n_, int32_t depth_, int32_t parent_rec_, const int16_t *idx_,
         double u_, double l_)
        : parent(parent_), action(action_), n(n_), depth(depth_), parent_rec(parent_rec_), idx_dev(idx_), u(u_),
          l(l_) {}
};

// Append-only store with concurrent appends: a fixed table of chunk
// pointers (2^16 elements a chunk), ranges reserved by an atomic counter,
// a chunk allocated by the first thread that reserves into it.  Growth
// never moves an element, and an index handed over through a release /
// acquire pair (a node's state) is safe to dereference on the other side.
// Chunks are raw memory (2 MB aligned, transparent huge pages asked for):
// the thread that reserves a range constructs its elements in place, so
// creating a node is one pass of stores (a large tree adds tens of
// millions of nodes a second).
template <class T>
struct ChunkStore {
    static_assert(std::is_trivially_destructible<T>::value, "elements are never destroyed");
    static constexpr size_t kAlign = size_t(2) << 20;
    static constexpr int kShift = 16;
    static constexpr size_t kMask = (size_t(1) << kShift) - 1;
    static constexpr size_t kMaxChunks = size_t(1) << 14;  // 2^30 elements
    static constexpr size_t kCapacity = kMaxChunks << kShift;
    std::unique_ptr<std::atomic<T *>[]> table;
    std::atomic<size_t> n{0};
    std::mutex grow;
    ChunkStore() : table(new std::atomic<T *>[kMaxChunks]) {
        for (size_t c = 0; c < kMaxChunks; ++c) table[c].store(nullptr, std::memory_order_relaxed);
    }
    ~ChunkStore() {
        for (size_t c = 0; c < kMaxChunks; ++c) free(table[c].load(std::memory_order_relaxed));
    }
    T &operator[](size_t i) { return table[i >> kShift].load(std::memory_order_relaxed)[i & kMask]; }
    const T &operator[](size_t i) const { return table[i >> kShift].load(std::memory_order_relaxed)[i & kMask]; }
    size_t size() const { return std::min(n.load(), kCapacity); }
    // `count` (> 0) consecutive unconstructed elements; the first index, or
    // kCapacity when the store is full or out of memory
    size_t reserve(size_t count) {
        const size_t at = n.fetch_add(count);
        if (at + count > kCapacity) return kCapacity;
        for (size_t c = at >> kShift; c <= (at + count - 1) >> kShift; ++c) {
            if (table[c].load(std::memory_order_acquire)) continue;
            std::lock_guard<std::mutex> g(grow);
            if (table[c].load(std::memory_order_relaxed)) continue;
            const size_t bytes = ((sizeof(T) << kShift) + kAlign - 1) / kAlign * kAlign;
            void *p = aligned_alloc(kAlign, bytes);
            if (!p) return kCapacity;
            madvise(p, bytes, MADV_HUGEPAGE);  // advice only: its failure changes nothing
            table[c].store((T *)p, std::memory_order_release);
        }
        return at;
    }
};

struct Act {
    double r = 0.0;
    int32_t child_begin = 0, n_children = 0;
    std::atomic<int32_t> visits{0};
    Act(double r_, int32_t child_begin_, int32_t n_children_)
        : r(r_), child_begin(child_begin_), n_children(n_children_) {}
    // sum over the children of n_child / n_parent times their u and l, in
    // child order; recomputed whenever a child's bounds change, so Eq. 4 and
    // Eq. 8 read one value per action instead of visiting every child
    std::atomic<double> su{0.0}, sl{0.0};
};

template <class T>
T ld(const std::atomic<T> &x) {
    return x.load(std::memory_order_relaxed);
}
template <class T>
void put(std::atomic<T> &x, T v) {
    x.store(v, std::memory_order_relaxed);
}

// Per-node spin lock, held for a few dozen operations at a time.
void node_lock(Node &b) {
    int spins = 0;
    while (b.lock.exchange(1, std::memory_order_acquire)) {
        while (b.lock.load(std::memory_order_relaxed)) {
            if (++spins > 256) {
                std::this_thread::yield();
                spins = 0;
            }
        }
    }
}
void node_unlock(Node &b) { b.lock.store(0, std::memory_order_release); }

// A leaf handed to the batchers; its thread sleeps on `cv` until a batcher
// sets `done` (under `m`, so the request outlives the notification).
struct Request {
    hdx_leaf leaf;
    std::mutex m;
    std::condition_variable cv;
    bool done = false;
    hdx_status status = HDX_OK;
};

hdx_states rec_states(const hdx_model_desc &d, const Rec &r) {
    hdx_states s;
    memset(&s, 0, sizeof(s));
    if (d.kind == HDX_ROCKSAMPLE || d.kind == HDX_MARS || d.kind == HDX_NAV) {
        s.w = (int32_t *)(r.dev + r.L.w);
    } else {
        s.s = (float *)(r.dev + r.L.s);
        s.car = (int32_t *)(r.dev + r.L.car);
        s.px = (float *)(r.dev + r.L.px);
        s.py = (float *)(r.dev + r.L.py);
        s.goal = (uint8_t *)(r.dev + r.L.goal);
    }
    s.stride = r.n;
    return s;
}

// A thread's head block in pinned host memory mapped into the device's
// address space: the expansion kernels write a leaf's child tables there
// directly, so the host reads them after the stream synchronises, with no
// copy call.  Sized for the largest record.
struct HeadBuf {
    char *host = nullptr;
    char *dev = nullptr;
    bool alloc(size_t bytes) {
        if (hipHostMalloc((void **)&host, bytes, hipHostMallocMapped) != hipSuccess) {
            host = nullptr;
            return false;
        }
        if (hipHostGetDevicePointer((void **)&dev, host, 0) != hipSuccess) {
            hipHostFree(host);
            host = dev = nullptr;
            return false;
        }
        return true;
    }
    void release() {
        if (host) hipHostFree(host);
        host = dev = nullptr;
    }
};

// Per-thread scratch of the surrogate judge: a record for the largest leaf
// and its head block.
struct Judge {
    Rec rec;
    HeadBuf head;
};

// Points a leaf's outputs at a record's arrays, its head block at `head`
// (a mapped host block laid out like the record's head).
void fill_outputs(const hdx_model_desc &d, hdx_leaf &L, const Rec &r, char *head) {
    L.states_out = rec_states(d, r);
    L.ids_out = (uint32_t *)(r.dev + r.L.ids);
    L.perm = (int16_t *)(r.dev + r.L.perm);
    L.n_children = (int32_t *)(head + r.L.n_children);
    L.child_z = (uint64_t *)(head + r.L.child_z);
    L.child_n = (int32_t *)(head + r.L.child_n);
    L.child_off = (int32_t *)(head + r.L.child_off);
    L.child_u0 = (float *)(head + r.L.child_u0);
    L.child_l0 = (float *)(head + r.L.child_l0);
    L.r_mean = (float *)(head + r.L.r_mean);
    L.steps = (int64_t *)(head + r.L.steps);
}


struct Search {
    hdx_ctx *ctx;
    const hdx_model *model;
    hdx_model_desc d;
    hdx_search_cfg cfg;
    int A;
    char *arena = nullptr;
    std::atomic<int64_t> arena_used{0};
    std::atomic<int> arena_full{0};
    ChunkStore<Node> nodes;
    ChunkStore<Act> acts;
    ChunkStore<Rec> recs;
    std::atomic<int64_t> trials{0}, expansions{0}, steps{0}, launches{0};
    std::atomic<int> max_depth{0};
    std::atomic<bool> stop{false};
    std::atomic<int64_t> idle_trials{0};
    // surrogate judge (rollouts on every j-th surrogate expansion) and fallback
    std::atomic<bool> surrogate_off{false};
    std::atomic<int64_t> judge_ctr{0};
    std::mutex jmu;
    double j_err = 0.0, j_ref = 0.0, j_diff = 0.0;
    std::atomic<double> l0_bias{0.0};  // added to surrogate child l0 once enough leaves are judged
    int64_t j_leaves = 0, j_children = 0;
    double c_a_abs = 0.0;  // c_a scaled by the initial root gap
    std::mutex emu;        // error state and the time breakdown
    hdx_status error = HDX_OK;
    std::string error_msg;
    double t_select = 0.0, t_expand = 0.0, t_backup = 0.0;  // thread-seconds
    Clock::time_point t0;

    void fail(hdx_status st, const char *where) {
        std::lock_guard<std::mutex> g(emu);
        if (error == HDX_OK) {
            error = st;
            error_msg = std::string(where) + ": " + hdx_last_error(ctx);
        }
        stop = true;
    }
    // batchers: pending leaves, taken by whichever batcher is free
    std::mutex qmu;
    std::condition_variable qcv;
    std::deque<Request *> queue;
    bool batcher_exit = false;

    int cap_for(int n) const { return std::max(1, hdx_model_max_children(model, n)); }

    bool alloc_rec(int n, Rec *out) {
        RecLayout L = rec_layout(d, n, cap_for(n));
        const int64_t at = arena_used.fetch_add((int64_t)L.total);
        if (at + (int64_t)L.total > cfg.arena_bytes) {
            arena_full = 1;
            return false;
        }
        out->dev = arena + at;
        out->L = L;
        out->n = n;
        return true;
    }

    double root_gap() { return std::max(ld(nodes[0].u) - ld(nodes[0].l), 0.0); }

    // The weighted child sums of one action (the inner sums of Eq. 4); the
    // caller holds the lock of the node the action belongs to.
    void refresh(Act &x, int32_t parent_n) {
        double su = 0.0, sl = 0.0;
        for (int c = 0; c < x.n_children; ++c) {
            const Node &k = nodes[x.child_begin + c];
            const double w = (double)k.n / (double)parent_n;
            su += w * ld(k.u);
            sl += w * ld(k.l);
        }
        put(x.su, su);
        put(x.sl, sl);
    }

    // Eq. 4 for one expanded node under its lock; then its new bounds go
    // into its parent action's sums under the parent's lock.  One lock at a
    // time: the thread that stores a node's last value refreshes the
    // parent after it, so once every backup has ended each node agrees with
    // its children.
    void bellman(Node &b) {
        node_lock(b);
        double bu = -std::numeric_limits<double>::infinity(), bl = bu;
        for (int a = 0; a < A; ++a) {
            const Act &x = acts[b.act_begin + a];
            bu = std::max(bu, x.r + d.gamma * ld(x.su));
            bl = std::max(bl, x.r + d.gamma * ld(x.sl));
        }
        put(b.u, bu);
        put(b.l, bl);
        node_unlock(b);
        if (b.parent >= 0) {
            Node &p = nodes[b.parent];
            node_lock(p);
            refresh(acts[p.act_begin + b.action], p.n);
            node_unlock(p);
        }
    }

    // Action bound of Eq. 8: u(b,a) plus the scenario-based exploration bonus
    int choose_action(const Node &b) {
        int best = 0;
        double best_v = -std::numeric_limits<double>::infinity();
        const double nb = (double)b.n * (double)std::max(ld(b.visits), 1);
        const double log_nb = c_a_abs > 0.0 ? log(nb) : 0.0;
        for (int a = 0; a < A; ++a) {
            const Act &x = acts[b.act_begin + a];
            double v = x.r + d.gamma * ld(x.su);
            if (c_a_abs > 0.0) {
                const int32_t xv = ld(x.visits);
                if (xv == 0) {
                    v = std::numeric_limits<double>::infinity();
                } else {
                    v += c_a_abs * sqrt(log_nb / ((double)b.n * (double)xv));
                }
            }
            if (v > best_v) {
                best_v = v;
                best = a;
            }
        }
        return best;
    }

    // sur_leaf: set when the leaf's child lower bounds came from the surrogate
    bool expand(int node_id, hipStream_t stream, const HeadBuf &hb, Judge *J, bool *sur_leaf);
    void judge_leaf(const hdx_leaf &L0, const Rec &r, const char *head_host, Judge &J, hipStream_t stream);
    bool use_surrogate() const { return cfg.surrogate != nullptr && !surrogate_off.load(); }

    // The children of an expanded node (Eq. 11) from its head block: the
    // node's actions and children are filled in new ranges of the stores,
    // then published by the release store of state 2.  False when a store
    // is full.
    bool attach(int node_id, const char *head, double l0_add) {
        Node &b = nodes[node_id];
        const Rec &r = recs[b.rec];
        const int cap = cap_for(b.n);
        const int32_t *nch = (const int32_t *)(head + r.L.n_children);
        const float *rm = (const float *)(head + r.L.r_mean);
        const int64_t *st = (const int64_t *)(head + r.L.steps);
        const int32_t *cn = (const int32_t *)(head + r.L.child_n);
        const int32_t *co = (const int32_t *)(head + r.L.child_off);
        const float *cu = (const float *)(head + r.L.child_u0);
        const float *cl = (const float *)(head + r.L.child_l0);
        int64_t s = 0, total = 0;
        for (int a = 0; a < A; ++a) {
            s += st[2 * a] + st[2 * a + 1];
            total += nch[a];
        }
        const size_t ab = acts.reserve((size_t)A);
        const size_t cb = total > 0 ? nodes.reserve((size_t)total) : nodes.size();
        if (ab >= acts.kCapacity || cb >= nodes.kCapacity) {
            arena_full = 1;
            return false;
        }
        steps += s;
        size_t c_at = cb;
        const int16_t *perm = (const int16_t *)(r.dev + r.L.perm);
        for (int a = 0; a < A; ++a) {
            Act &x = *new (&acts[ab + a]) Act((double)rm[a], (int32_t)c_at, nch[a]);
            for (int c = 0; c < nch[a]; ++c) {
                const int q = a * cap + c;
                const double u = (double)cu[q];
                double l = (double)cl[q];
                if (l0_add != 0.0) l = std::min(l + l0_add, u);
                new (&nodes[c_at++]) Node(node_id, a, cn[q], b.depth + 1, b.rec, perm + (size_t)a * b.n + co[q], u, l);
            }
            refresh(x, b.n);
        }
        b.act_begin = (int32_t)ab;
        b.state.store(2, std::memory_order_release);
        int md = b.depth + 1;
        int cur = max_depth.load();
        while (md > cur && !max_depth.compare_exchange_weak(cur, md)) {
        }
        return true;
    }
};

// The surrogate's children l0 against the rollouts' on the same leaf (same
// grouping, both expansions being deterministic); falls back to rollouts
// when the accumulated relative error exceeds the configured bound.
void Search::judge_leaf(const hdx_leaf &L0, const Rec &r, const char *head_host, Judge &J, hipStream_t stream) {
    hdx_leaf L = L0;
    // the judge's record has room for the largest leaf; its head block takes
    // this leaf's layout (the offsets of r)
    fill_outputs(d, L, J.rec, J.head.dev);
    L.n_children = (int32_t *)(J.head.dev + r.L.n_children);
    L.child_z = (uint64_t *)(J.head.dev + r.L.child_z);
    L.child_n = (int32_t *)(J.head.dev + r.L.child_n);
    L.child_off = (int32_t *)(J.head.dev + r.L.child_off);
    L.child_u0 = (float *)(J.head.dev + r.L.child_u0);
    L.child_l0 = (float *)(J.head.dev + r.L.child_l0);
    L.r_mean = (float *)(J.head.dev + r.L.r_mean);
    L.steps = (int64_t *)(J.head.dev + r.L.steps);
    hdx_status st = hdx_expand_leaf_surrogate(ctx, &L, 1, cfg.surrogate, cfg.surrogate_horizon, stream);
    if (st != HDX_OK) {
        fail(st, "judge expansion");
        return;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        fail(HDX_E_DEVICE, "judge expansion wait");
        return;
    }
    const int cap = L0.cap;
    const int32_t *nch = (const int32_t *)(head_host + r.L.n_children);
    const float *lf = (const float *)(head_host + r.L.child_l0);
    const float *ls = (const float *)(J.head.host + r.L.child_l0);
    double e = 0.0, ref = 0.0, diff = 0.0;
    int64_t nc = 0;
    for (int a = 0; a < A; ++a)
        for (int c = 0; c < nch[a] && c < cap; ++c) {
            e += std::fabs((double)ls[a * cap + c] - (double)lf[a * cap + c]);
            diff += (double)lf[a * cap + c] - (double)ls[a * cap + c];
            ref += std::fabs((double)lf[a * cap + c]);
            ++nc;
        }
    std::lock_guard<std::mutex> g(jmu);
    j_err += e;
    j_ref += ref;
    j_diff += diff;
    j_children += nc;
    j_leaves += 1;
    if (cfg.surrogate_bias_correct && j_leaves >= 8 && j_children > 0) put(l0_bias, j_diff / (double)j_children);
    if (cfg.surrogate_max_rel_err > 0.0 && j_leaves >= 8 && j_err > cfg.surrogate_max_rel_err * j_ref)
        surrogate_off = true;
}

bool Search::expand(int node_id, hipStream_t stream, const HeadBuf &hb, Judge *J, bool *sur_leaf) {
    char *head_host = hb.host;
    Node &b = nodes[node_id];
    Rec r;
    if (!alloc_rec(b.n, &r)) return false;
    const size_t ri = recs.reserve(1);
    if (ri >= recs.kCapacity) {
        arena_full = 1;
        return false;
    }
    new (&recs[ri]) Rec(r);
    b.rec = (int32_t)ri;
    const Rec &parent = recs[b.parent_rec];
    hdx_leaf L;
    memset(&L, 0, sizeof(L));
    L.model = model;
    L.seed = cfg.seed;
    L.step = cfg.step;
    L.rollout = cfg.rollout;
    L.parent = rec_states(d, parent);
    L.parent_ids = (const uint32_t *)(parent.dev + parent.L.ids);
    L.idx = b.idx_dev;
    L.n = b.n;
    L.depth = b.depth;
    L.last_action = b.action;
    L.cap = cap_for(b.n);
    fill_outputs(d, L, r, hb.dev);
    hdx_status st = HDX_OK;
    const bool sur = use_surrogate();
    const bool judge = sur && J != nullptr && cfg.surrogate_judge_every > 0 &&
                       judge_ctr.fetch_add(1) % cfg.surrogate_judge_every == 0;
    *sur_leaf = sur && !judge;
    if (cfg.batch_leaves > 1 && !judge) {
        Request q;
        q.leaf = L;
        {
            std::lock_guard<std::mutex> lk(qmu);
            queue.push_back(&q);
        }
        qcv.notify_one();
        {
            std::unique_lock<std::mutex> lk(q.m);
            q.cv.wait(lk, [&] { return q.done; });
        }
        st = q.status;
    } else {
        // a judged leaf keeps its rollout bounds in the tree
        st = (sur && !judge) ? hdx_expand_leaf_surrogate(ctx, &L, 1, cfg.surrogate, cfg.surrogate_horizon, stream)
                             : hdx_expand_leaf(ctx, &L, 1, stream);
        if (st != HDX_OK) {
            fail(st, "expand_leaf");
        } else {
            const hipError_t e = hipStreamSynchronize(stream);  // the head block is then on the host
            if (e != hipSuccess) {
                st = HDX_E_DEVICE;
                std::lock_guard<std::mutex> g(emu);
                if (error == HDX_OK) {
                    error = st;
                    error_msg = std::string("expansion wait: ") + hipGetErrorString(e);
                }
                stop = true;
            }
            if (st == HDX_OK && judge) judge_leaf(L, r, head_host, *J, stream);
        }
        launches++;
    }
    return st == HDX_OK;
}

// One batcher: takes up to batch_leaves pending leaves, launches them in
// packs of at most kArgLeaves (descriptors in the kernel arguments, no
// staging copies) on its own stream, waits once for all of them (their head
// blocks are mapped host memory) and wakes their threads.  Several batchers
// keep several batches in flight.
void batcher_loop(Search *S) {
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
        S->fail(HDX_E_DEVICE, "batcher stream");
        stream = nullptr;
    }
    std::vector<Request *> batch;
    std::vector<hdx_leaf> leaves;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->qmu);
            S->qcv.wait(lk, [&] { return S->batcher_exit || !S->queue.empty(); });
            if (S->queue.empty() && S->batcher_exit) break;
            batch.clear();
            while (!S->queue.empty() && (int)batch.size() < S->cfg.batch_leaves) {
                batch.push_back(S->queue.front());
                S->queue.pop_front();
            }
        }
        leaves.clear();
        for (Request *q : batch) leaves.push_back(q->leaf);
        hdx_status st = stream ? HDX_OK : HDX_E_DEVICE;
        for (size_t i = 0; i < leaves.size() && st == HDX_OK; i += hdx::kArgLeaves) {
            const int32_t nl = (int32_t)std::min(leaves.size() - i, (size_t)hdx::kArgLeaves);
            st = S->use_surrogate() ? hdx_expand_leaf_surrogate(S->ctx, leaves.data() + i, nl, S->cfg.surrogate,
                                                               S->cfg.surrogate_horizon, stream)
                                    : hdx_expand_leaf(S->ctx, leaves.data() + i, nl, stream);
            S->launches++;
        }
        if (st != HDX_OK) S->fail(st, "batched expand_leaf");
        if (st == HDX_OK && hipStreamSynchronize(stream) != hipSuccess) {
            st = HDX_E_DEVICE;
            S->fail(st, "batched expansion wait");
        }
        for (Request *q : batch) {
            std::lock_guard<std::mutex> lk(q->m);
            q->status = st;
            q->done = true;
            q->cv.notify_one();
        }
    }
    if (stream) hipStreamDestroy(stream);
}

void worker(Search *S, int tid, size_t head_bytes) {
    hipStream_t stream = nullptr;
    hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    HeadBuf hb;
    if (!hb.alloc(head_bytes)) {
        S->fail(HDX_E_NOMEM, "head block");
        hipStreamDestroy(stream);
        return;
    }
    Judge judge;
    Judge *J = nullptr;
    if (S->cfg.surrogate && S->cfg.surrogate_judge_every > 0 && S->alloc_rec(S->cfg.K, &judge.rec) &&
        judge.head.alloc(head_bytes))
        J = &judge;
    std::vector<int> path;
    const double K = (double)S->cfg.K;
    double t_sel = 0.0, t_exp = 0.0, t_back = 0.0;
    auto since = [](Clock::time_point t) { return std::chrono::duration<double>(Clock::now() - t).count(); };
    while (!S->stop.load()) {
        const Clock::time_point ts = Clock::now();
        const double elapsed = std::chrono::duration<double>(ts - S->t0).count();
        if (elapsed >= S->cfg.time_budget_s || S->arena_full.load()) break;
        if (S->cfg.max_trials > 0 && S->trials.load() >= S->cfg.max_trials) break;
        const double eps0 = S->root_gap();
        if (eps0 <= S->cfg.gap_epsilon) {
            S->stop = true;
            break;
        }
        // descend (Eq. 8 actions, Eq. 7 observation branches with the virtual
        // loss of Eq. 9); a leaf is claimed by moving its state from 0 to 1
        int leaf = -1;
        path.clear();
        int b = 0;
        path.push_back(0);
        for (;;) {
            Node &nb = S->nodes[b];
            nb.visits.fetch_add(1, std::memory_order_relaxed);
            const int32_t state = nb.state.load(std::memory_order_acquire);
            if (state != 2) {
                int32_t expect = 0;
                if (state == 0 && nb.depth < S->cfg.max_depth && nb.n > 0 &&
                    nb.state.compare_exchange_strong(expect, 1, std::memory_order_acq_rel))
                    leaf = b;
                break;
            }
            const int a = S->choose_action(nb);
            Act &x = S->acts[nb.act_begin + a];
            x.visits.fetch_add(1, std::memory_order_relaxed);
            int best = -1;
            double best_e = -std::numeric_limits<double>::infinity(), best_plain = 0.0;
            for (int c = 0; c < x.n_children; ++c) {
                const Node &k = S->nodes[x.child_begin + c];
                const double e = (ld(k.u) - ld(k.l)) - (double)k.n / K * S->cfg.xi * eps0;
                const double ep = e - (double)ld(k.vloss) * S->cfg.c_o * eps0;
                if (ep > best_e) {
                    best_e = ep;
                    best = x.child_begin + c;
                    best_plain = e;
                }
            }
            if (best < 0 || best_plain <= 0.0) break;  // the path ends where E is not positive
            S->nodes[best].vloss.fetch_add(1, std::memory_order_relaxed);
            b = best;
            path.push_back(b);
        }
        const Clock::time_point te = Clock::now();
        t_sel += std::chrono::duration<double>(te - ts).count();
        bool ok = true;
        if (leaf >= 0) {
            bool sur_leaf = false;
            ok = S->expand(leaf, stream, hb, J, &sur_leaf);
            t_exp += since(te);
            const Clock::time_point tb = Clock::now();
            if (ok) ok = S->attach(leaf, hb.host, sur_leaf ? ld(S->l0_bias) : 0.0);
            if (ok) {
                S->expansions++;
            } else {
                S->nodes[leaf].state.store(0, std::memory_order_release);
            }
            t_back += since(tb);
        }
        const Clock::time_point tb = Clock::now();
        for (size_t i = path.size(); i-- > 0;) {
            Node &nb = S->nodes[path[i]];
            if (nb.state.load(std::memory_order_acquire) == 2) S->bellman(nb);
            if (i > 0) nb.vloss.fetch_sub(1, std::memory_order_relaxed);
        }
        t_back += since(tb);
        if (!ok) break;
        S->trials++;
        if (leaf < 0) {
            // the path ended where the excess uncertainty is not positive, or
            // at a leaf another thread is expanding: nothing was expanded
            S->idle_trials++;
            std::this_thread::yield();
        }
    }
    {
        std::lock_guard<std::mutex> g(S->emu);
        S->t_select += t_sel;
        S->t_expand += t_exp;
        S->t_backup += t_back;
    }
    hb.release();
    judge.head.release();
    hipStreamDestroy(stream);
}

}  // namespace

extern "C" hdx_status hdx_search(hdx_ctx *ctx, const hdx_model *model, const hdx_belief *belief,
                                 const hdx_search_cfg *cfg, hdx_search_result *out) {
    if (!ctx || !model || !belief || !cfg || !out) return HDX_E_INVALID;
    const int A = hdx_model_actions(model);
    const int k_max = hdx_internal_desc(model)->kind == HDX_NAV ? HDX_MAX_NAV_LEAF_SCENARIOS : HDX_MAX_LEAF_SCENARIOS;
    if (cfg->K < 1 || cfg->K > k_max || cfg->n_threads < 1 || cfg->n_threads > 64 ||
        cfg->max_depth < 1 || cfg->arena_bytes < (1 << 20) || A > HDX_MAX_ACTIONS)
        return HDX_E_INVALID;
    Search S;
    S.ctx = ctx;
    S.model = model;
    S.d = *hdx_internal_desc(model);
    S.cfg = *cfg;
    S.A = A;
    memset(out, 0, sizeof(*out));
    if (hipMalloc((void **)&S.arena, (size_t)cfg->arena_bytes) != hipSuccess) return HDX_E_NOMEM;
    hipStream_t main_stream = nullptr;
    hipStreamCreateWithFlags(&main_stream, hipStreamNonBlocking);
    hdx_status st = HDX_OK;

    // root: sample K scenarios (Sec. III-A) and set the initial bounds
    Rec root_rec;
    int16_t *iota = nullptr;  // the root's positions 0..K-1 in its own record
    int32_t *depths = nullptr;
    float *U = nullptr, *L = nullptr;
    const size_t K = (size_t)cfg->K;
    if (!S.alloc_rec(cfg->K, &root_rec)) st = HDX_E_NOMEM;
    if (st == HDX_OK) {
        const int64_t bytes = (int64_t)align16(14 * K);
        const int64_t at = S.arena_used.fetch_add(bytes);
        if (at + bytes > cfg->arena_bytes) st = HDX_E_NOMEM;
        depths = (int32_t *)(S.arena + at);
        U = (float *)(depths + K);
        L = U + K;
        iota = (int16_t *)(L + K);
    }
    std::vector<int32_t> h_iota(K), h_zero(K, 0);
    std::vector<int16_t> h_iota16(K);
    std::vector<float> hU(K), hL(K);
    for (size_t k = 0; k < K; ++k) {
        h_iota[k] = (int32_t)k;
        h_iota16[k] = (int16_t)k;
    }
    if (st == HDX_OK)
        st = hdx_sample_scenarios(ctx, model, belief, cfg->K, cfg->seed, cfg->step, rec_states(S.d, root_rec),
                                  main_stream);
    if (st == HDX_OK && (hipMemcpyAsync(iota, h_iota16.data(), 2 * K, hipMemcpyHostToDevice, main_stream) != hipSuccess ||
                         hipMemcpyAsync(depths, h_zero.data(), 4 * K, hipMemcpyHostToDevice, main_stream) != hipSuccess ||
                         hipMemcpyAsync(root_rec.dev + root_rec.L.ids, h_iota.data(), 4 * K, hipMemcpyHostToDevice,
                                        main_stream) != hipSuccess))
        st = HDX_E_DEVICE;
    if (st == HDX_OK)
        st = hdx_rollout_bounds(ctx, model, &cfg->rollout, cfg->seed, cfg->step, rec_states(S.d, root_rec),
                                (const uint32_t *)(root_rec.dev + root_rec.L.ids), depths, cfg->K, U, L, nullptr,
                                main_stream);
    if (st == HDX_OK && (hipMemcpyAsync(hU.data(), U, 4 * K, hipMemcpyDeviceToHost, main_stream) != hipSuccess ||
                         hipMemcpyAsync(hL.data(), L, 4 * K, hipMemcpyDeviceToHost, main_stream) != hipSuccess ||
                         hipStreamSynchronize(main_stream) != hipSuccess))
        st = HDX_E_DEVICE;
    if (st != HDX_OK) {
        hipStreamDestroy(main_stream);
        hipFree(S.arena);
        return st;
    }
    double su = 0.0, sl = 0.0;
    for (size_t k = 0; k < K; ++k) {
        su += hU[k];
        sl += hL[k];
    }
    const size_t root_at = S.nodes.reserve(1), rec_at = S.recs.reserve(1);
    if (root_at != 0 || rec_at != 0) {
        hipStreamDestroy(main_stream);
        hipFree(S.arena);
        return HDX_E_NOMEM;
    }
    new (&S.recs[0]) Rec(root_rec);
    const Node &root = *new (&S.nodes[0]) Node(-1, -1, cfg->K, 0, 0, iota, su / (double)K, sl / (double)K);
    out->u0_root = ld(root.u);
    out->l0_root = ld(root.l);
    S.c_a_abs = cfg->c_a * std::max(out->u0_root - out->l0_root, 0.0);

    const RecLayout big = rec_layout(S.d, cfg->K, S.cap_for(cfg->K));
    S.t0 = Clock::now();
    // one batcher per batch_leaves threads, at most eight
    std::vector<std::thread> batchers;
    if (cfg->batch_leaves > 1) {
        const int nb = std::min(8, std::max(1, (cfg->n_threads + cfg->batch_leaves - 1) / cfg->batch_leaves));
        for (int i = 0; i < nb; ++i) batchers.emplace_back(batcher_loop, &S);
    }
    std::vector<std::thread> workers;
    for (int t = 0; t < cfg->n_threads; ++t) workers.emplace_back(worker, &S, t, big.head);
    for (auto &w : workers) w.join();
    if (!batchers.empty()) {
        {
            std::lock_guard<std::mutex> lk(S.qmu);
            S.batcher_exit = true;
        }
        S.qcv.notify_all();
        for (auto &b : batchers) b.join();
    }
    out->elapsed_s = std::chrono::duration<double>(Clock::now() - S.t0).count();
    const Node &r = S.nodes[0];
    out->u_root = ld(r.u);
    out->l_root = ld(r.l);
    out->trials = S.trials.load();
    out->idle_trials = S.idle_trials.load();
    out->expansions = S.expansions.load();
    out->nodes = (int64_t)S.nodes.size();
    out->scenario_steps = S.steps.load();
    out->launches = S.launches.load();
    out->max_depth_reached = S.max_depth.load();
    out->arena_full = S.arena_full.load();
    out->judged_leaves = S.j_leaves;
    out->judged_children = S.j_children;
    out->judge_mae = S.j_children > 0 ? S.j_err / (double)S.j_children : 0.0;
    out->judge_rel_err = S.j_ref > 0.0 ? S.j_err / S.j_ref : 0.0;
    out->judge_bias = S.j_children > 0 ? S.j_diff / (double)S.j_children : 0.0;
    out->surrogate_off = S.surrogate_off.load() ? 1 : 0;
    out->time_select_s = S.t_select;
    out->time_expand_s = S.t_expand;
    out->time_backup_s = S.t_backup;
    out->best_action = 0;
    if (ld(r.state) == 2) {
        double best = -std::numeric_limits<double>::infinity();
        for (int a = 0; a < A; ++a) {
            const Act &x = S.acts[r.act_begin + a];
            double sum_u = 0.0, sum_l = 0.0;
            for (int c = 0; c < x.n_children; ++c) {
                const Node &k = S.nodes[x.child_begin + c];
                sum_u += (double)k.n / (double)r.n * ld(k.u);
                sum_l += (double)k.n / (double)r.n * ld(k.l);
            }
            out->action_u[a] = x.r + S.d.gamma * sum_u;
            out->action_l[a] = x.r + S.d.gamma * sum_l;
            if (out->action_l[a] > best) {
                best = out->action_l[a];
                out->best_action = a;
            }
        }
    }
    hipStreamSynchronize(main_stream);
    hdx_internal_quiesce(ctx);
    hipStreamDestroy(main_stream);
    hipDeviceSynchronize();
    hipFree(S.arena);
    if (S.error != HDX_OK) {
        hdx_internal_set_error(ctx, S.error_msg.c_str());
        return S.error;
    }
    return HDX_OK;
}
