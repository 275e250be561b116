// Parallel DESPOT search on the CPU feeding leaf expansion to the GPU
// (HyP-DESPOT, Sec. III-A and III-C).  Several host threads share one tree:
// each trial walks down by the scenario-based PO-UCT action bound (Eq. 8)
// and the weighted excess uncertainty with virtual loss (Eq. 7, 9), expands
// the leaf it reaches through hdx_expand_leaf (Eq. 10-13), attaches the
// children (Eq. 11) and backs the bounds up to the root (Eq. 4).  Node
// states stay on the device: a node's scenarios are a segment of its
// parent's grouped order, and its own states are materialised when it is
// expanded.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
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

struct Node {
    int32_t parent = -1;
    int32_t action = -1;  // action from the parent
    int32_t n = 0;        // |Phi_b|
    int32_t depth = 0;
    double u = 0.0, l = 0.0;
    int32_t parent_rec = -1;          // record holding the parent's states
    const int16_t *idx_dev = nullptr;  // positions in that record
    int32_t state = 0;                // 0 leaf, 1 being expanded, 2 expanded
    int32_t visits = 0, vloss = 0;
    int32_t act_begin = -1;
    int32_t rec = -1;
};

// Append-only store in chunks of 2^16 elements: growth never moves an
// element (a 625-action tree adds ~20 M nodes a second, and a vector's
// doubling copies stalled every thread behind the tree lock), and an index
// costs one shift and one mask.  Guarded by the tree lock like the tree.
template <class T>
struct ChunkStore {
    static constexpr int kShift = 16;
    static constexpr size_t kMask = (size_t(1) << kShift) - 1;
    std::vector<std::unique_ptr<T[]>> chunks;
    size_t n = 0;
    T &operator[](size_t i) { return chunks[i >> kShift][i & kMask]; }
    const T &operator[](size_t i) const { return chunks[i >> kShift][i & kMask]; }
    size_t size() const { return n; }
    void push_back(const T &v) {
        if ((n >> kShift) == chunks.size()) chunks.emplace_back(new T[size_t(1) << kShift]);
        (*this)[n++] = v;
    }
};

struct Act {
    double r;
    int32_t child_begin, n_children, visits;
    // sum over the children of n_child / n_parent times their u and l, in
    // child order; recomputed whenever a child's bounds change, so Eq. 4 and
    // Eq. 8 read one value per action instead of visiting every child
    double su = 0.0, sl = 0.0;
};

struct Request {
    hdx_leaf leaf;
    const Rec *rec;
    char *head_host;
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
    std::mutex mu;  // tree
    ChunkStore<Node> nodes;
    ChunkStore<Act> acts;
    std::deque<Rec> recs;  // stable addresses
    std::atomic<int64_t> trials{0}, expansions{0}, steps{0}, launches{0};
    std::atomic<int> max_depth{0};
    std::atomic<bool> stop{false};
    std::atomic<int64_t> idle_trials{0};
    // surrogate judge (rollouts on every j-th surrogate expansion) and fallback
    std::atomic<bool> surrogate_off{false};
    std::atomic<int64_t> judge_ctr{0};
    std::mutex jmu;
    double j_err = 0.0, j_ref = 0.0;
    int64_t j_leaves = 0, j_children = 0;
    double c_a_abs = 0.0;  // c_a scaled by the initial root gap
    std::mutex emu;
    hdx_status error = HDX_OK;
    std::string error_msg;
    Clock::time_point t0;

    void fail(hdx_status st, const char *where) {
        std::lock_guard<std::mutex> g(emu);
        if (error == HDX_OK) {
            error = st;
            error_msg = std::string(where) + ": " + hdx_last_error(ctx);
        }
        stop = true;
    }
    // batcher
    std::mutex qmu;
    std::condition_variable qcv, dcv;
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

    double root_gap() const { return std::max(nodes[0].u - nodes[0].l, 0.0); }

    // The weighted child sums of one action (the inner sums of Eq. 4).
    void refresh(Act &x, int32_t parent_n) {
        double su = 0.0, sl = 0.0;
        for (int c = 0; c < x.n_children; ++c) {
            const Node &k = nodes[x.child_begin + c];
            const double w = (double)k.n / (double)parent_n;
            su += w * k.u;
            sl += w * k.l;
        }
        x.su = su;
        x.sl = sl;
    }

    // Eq. 4 for one expanded node; its new bounds go into its parent
    // action's sums
    void bellman(Node &b) {
        double bu = -std::numeric_limits<double>::infinity(), bl = bu;
        for (int a = 0; a < A; ++a) {
            const Act &x = acts[b.act_begin + a];
            bu = std::max(bu, x.r + d.gamma * x.su);
            bl = std::max(bl, x.r + d.gamma * x.sl);
        }
        b.u = bu;
        b.l = bl;
        if (b.parent >= 0) {
            const Node &p = nodes[b.parent];
            refresh(acts[p.act_begin + b.action], p.n);
        }
    }

    // Action bound of Eq. 8: u(b,a) plus the scenario-based exploration bonus
    int choose_action(const Node &b) const {
        int best = 0;
        double best_v = -std::numeric_limits<double>::infinity();
        const double nb = (double)b.n * (double)std::max(b.visits, 1);
        for (int a = 0; a < A; ++a) {
            const Act &x = acts[b.act_begin + a];
            double v = x.r + d.gamma * x.su;
            if (c_a_abs > 0.0) {
                if (x.visits == 0) {
                    v = std::numeric_limits<double>::infinity();
                } else {
                    v += c_a_abs * sqrt(log(nb) / ((double)b.n * (double)x.visits));
                }
            }
            if (v > best_v) {
                best_v = v;
                best = a;
            }
        }
        return best;
    }

    bool expand(int node_id, hipStream_t stream, const HeadBuf &hb, Judge *J);
    void judge_leaf(const hdx_leaf &L0, const Rec &r, const char *head_host, Judge &J, hipStream_t stream);
    bool use_surrogate() const { return cfg.surrogate != nullptr && !surrogate_off.load(); }

    void attach(int node_id, const Rec &r, const char *head) {
        Node &b = nodes[node_id];
        const int cap = cap_for(b.n);
        const int32_t *nch = (const int32_t *)(head + r.L.n_children);
        const float *rm = (const float *)(head + r.L.r_mean);
        const int64_t *st = (const int64_t *)(head + r.L.steps);
        const int32_t *cn = (const int32_t *)(head + r.L.child_n);
        const int32_t *co = (const int32_t *)(head + r.L.child_off);
        const float *cu = (const float *)(head + r.L.child_u0);
        const float *cl = (const float *)(head + r.L.child_l0);
        int64_t s = 0;
        for (int a = 0; a < A; ++a) s += st[2 * a] + st[2 * a + 1];
        steps += s;
        const int32_t rec_index = b.rec;
        const int parent_depth = b.depth;
        const int parent_n = b.n;
        nodes[node_id].act_begin = (int32_t)acts.size();
        for (int a = 0; a < A; ++a) {
            const size_t ai = acts.size();
            acts.push_back(Act{(double)rm[a], (int32_t)nodes.size(), nch[a], 0});
            for (int c = 0; c < nch[a]; ++c) {
                Node k;
                k.parent = node_id;
                k.action = a;
                k.n = cn[a * cap + c];
                k.depth = parent_depth + 1;
                k.u = cu[a * cap + c];
                k.l = cl[a * cap + c];
                k.parent_rec = rec_index;
                k.idx_dev = (const int16_t *)(r.dev + r.L.perm) + (size_t)a * parent_n + co[a * cap + c];
                nodes.push_back(k);
            }
            refresh(acts[ai], parent_n);
        }
        nodes[node_id].state = 2;
        int md = parent_depth + 1;
        int cur = max_depth.load();
        while (md > cur && !max_depth.compare_exchange_weak(cur, md)) {
        }
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
    double e = 0.0, ref = 0.0;
    int64_t nc = 0;
    for (int a = 0; a < A; ++a)
        for (int c = 0; c < nch[a] && c < cap; ++c) {
            e += std::fabs((double)ls[a * cap + c] - (double)lf[a * cap + c]);
            ref += std::fabs((double)lf[a * cap + c]);
            ++nc;
        }
    std::lock_guard<std::mutex> g(jmu);
    j_err += e;
    j_ref += ref;
    j_children += nc;
    j_leaves += 1;
    if (cfg.surrogate_max_rel_err > 0.0 && j_leaves >= 8 && j_err > cfg.surrogate_max_rel_err * j_ref)
        surrogate_off = true;
}

bool Search::expand(int node_id, hipStream_t stream, const HeadBuf &hb, Judge *J) {
    char *head_host = hb.host;
    // builds the leaf descriptor; the caller holds no lock
    Node b;
    {
        std::lock_guard<std::mutex> g(mu);
        b = nodes[node_id];
    }
    Rec r;
    if (!alloc_rec(b.n, &r)) return false;
    const Rec *parent = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        parent = &recs[b.parent_rec];
    }
    hdx_leaf L;
    memset(&L, 0, sizeof(L));
    L.model = model;
    L.seed = cfg.seed;
    L.step = cfg.step;
    L.rollout = cfg.rollout;
    L.parent = rec_states(d, *parent);
    L.parent_ids = (const uint32_t *)(parent->dev + parent->L.ids);
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
    if (cfg.batch_leaves > 1 && !judge) {
        Request q;
        q.leaf = L;
        q.rec = nullptr;
        q.head_host = head_host;
        Rec *rp = nullptr;
        {
            std::lock_guard<std::mutex> g(mu);
            recs.push_back(r);
            rp = &recs.back();
            nodes[node_id].rec = (int32_t)recs.size() - 1;
        }
        q.rec = rp;
        {
            std::unique_lock<std::mutex> lk(qmu);
            queue.push_back(&q);
            qcv.notify_one();
            dcv.wait(lk, [&] { return q.done; });
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
        std::lock_guard<std::mutex> g(mu);
        recs.push_back(r);
        nodes[node_id].rec = (int32_t)recs.size() - 1;
    }
    if (st != HDX_OK) return false;
    expansions++;
    std::lock_guard<std::mutex> g(mu);
    attach(node_id, recs[nodes[node_id].rec], head_host);
    return true;
}

void batcher_loop(Search *S, hipStream_t stream) {
    std::vector<Request *> batch;
    std::vector<hdx_leaf> leaves;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->qmu);
            S->qcv.wait(lk, [&] { return S->batcher_exit || !S->queue.empty(); });
            if (S->queue.empty() && S->batcher_exit) return;
            batch.clear();
            while (!S->queue.empty() && (int)batch.size() < S->cfg.batch_leaves) {
                batch.push_back(S->queue.front());
                S->queue.pop_front();
            }
        }
        leaves.clear();
        for (Request *q : batch) leaves.push_back(q->leaf);
        const int32_t nl = (int32_t)leaves.size();
        hdx_status st = S->use_surrogate() ? hdx_expand_leaf_surrogate(S->ctx, leaves.data(), nl, S->cfg.surrogate,
                                                                     S->cfg.surrogate_horizon, stream)
                                         : hdx_expand_leaf(S->ctx, leaves.data(), nl, stream);
        if (st != HDX_OK) S->fail(st, "batched expand_leaf");
        // every leaf's head block is mapped host memory: one wait delivers all
        if (st == HDX_OK && hipStreamSynchronize(stream) != hipSuccess) st = HDX_E_DEVICE;
        S->launches++;
        {
            std::lock_guard<std::mutex> lk(S->qmu);
            for (Request *q : batch) {
                q->status = st;
                q->done = true;
            }
        }
        S->dcv.notify_all();
    }
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
    while (!S->stop.load()) {
        const double elapsed = std::chrono::duration<double>(Clock::now() - S->t0).count();
        if (elapsed >= S->cfg.time_budget_s || S->arena_full.load()) break;
        if (S->cfg.max_trials > 0 && S->trials.load() >= S->cfg.max_trials) break;
        int leaf = -1;
        path.clear();
        {
            std::lock_guard<std::mutex> g(S->mu);
            if (S->root_gap() <= S->cfg.gap_epsilon) {
                S->stop = true;
                break;
            }
            const double eps0 = S->root_gap();
            int b = 0;
            path.push_back(0);
            for (;;) {
                Node &nb = S->nodes[b];
                nb.visits++;
                if (nb.state != 2) {
                    if (nb.state == 0 && nb.depth < S->cfg.max_depth && nb.n > 0) {
                        nb.state = 1;
                        leaf = b;
                    }
                    break;
                }
                const int a = S->choose_action(nb);
                Act &x = S->acts[nb.act_begin + a];
                x.visits++;
                // Eq. 7 with the virtual loss of Eq. 9
                int best = -1;
                double best_e = -std::numeric_limits<double>::infinity(), best_plain = 0.0;
                for (int c = 0; c < x.n_children; ++c) {
                    const Node &k = S->nodes[x.child_begin + c];
                    const double e = (k.u - k.l) - (double)k.n / K * S->cfg.xi * eps0;
                    const double ep = e - (double)k.vloss * S->cfg.c_o * eps0;
                    if (ep > best_e) {
                        best_e = ep;
                        best = x.child_begin + c;
                        best_plain = e;
                    }
                }
                if (best < 0 || best_plain <= 0.0) break;  // the path ends where E is not positive
                S->nodes[best].vloss++;
                b = best;
                path.push_back(b);
            }
        }
        bool ok = true;
        if (leaf >= 0) {
            ok = S->expand(leaf, stream, hb, J);
            if (!ok) {
                std::lock_guard<std::mutex> g(S->mu);
                S->nodes[leaf].state = 0;
            }
        }
        {
            std::lock_guard<std::mutex> g(S->mu);
            for (size_t i = path.size(); i-- > 0;) {
                Node &nb = S->nodes[path[i]];
                if (nb.state == 2) S->bellman(nb);
                if (i > 0) nb.vloss--;
            }
        }
        if (!ok) break;
        S->trials++;
        if (leaf < 0) {
            // the path ended where the excess uncertainty is not positive:
            // nothing was expanded; let the other threads take the lock
            S->idle_trials++;
            std::this_thread::yield();
        }
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
    S.recs.push_back(root_rec);
    Node root;
    root.n = cfg->K;
    root.u = su / (double)K;
    root.l = sl / (double)K;
    root.parent_rec = 0;
    root.idx_dev = iota;
    S.nodes.push_back(root);
    out->u0_root = root.u;
    out->l0_root = root.l;
    S.c_a_abs = cfg->c_a * std::max(root.u - root.l, 0.0);

    const RecLayout big = rec_layout(S.d, cfg->K, S.cap_for(cfg->K));
    S.t0 = Clock::now();
    std::thread batcher;
    if (cfg->batch_leaves > 1) batcher = std::thread(batcher_loop, &S, main_stream);
    std::vector<std::thread> workers;
    for (int t = 0; t < cfg->n_threads; ++t) workers.emplace_back(worker, &S, t, big.head);
    for (auto &w : workers) w.join();
    if (batcher.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S.qmu);
            S.batcher_exit = true;
        }
        S.qcv.notify_all();
        batcher.join();
    }
    out->elapsed_s = std::chrono::duration<double>(Clock::now() - S.t0).count();
    const Node &r = S.nodes[0];
    out->u_root = r.u;
    out->l_root = r.l;
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
    out->surrogate_off = S.surrogate_off.load() ? 1 : 0;
    out->best_action = 0;
    if (r.state == 2) {
        double best = -std::numeric_limits<double>::infinity();
        for (int a = 0; a < A; ++a) {
            const Act &x = S.acts[r.act_begin + a];
            double sum_u = 0.0, sum_l = 0.0;
            for (int c = 0; c < x.n_children; ++c) {
                const Node &k = S.nodes[x.child_begin + c];
                sum_u += (double)k.n / (double)r.n * k.u;
                sum_l += (double)k.n / (double)r.n * k.l;
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
