// DESPOT tree on the host and the Bellman backup of Eq. 4 (Sec. III-A).
// Nodes keep their scenario count and bounds; an expanded node keeps, per
// action, the mean step reward and the range of its observation children.
#include <math.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <vector>

#include "hdx.h"

namespace {

struct ActionBranch {
    double r_mean;
    int64_t child_begin;
    int32_t n_children;
};

struct Node {
    int64_t parent;
    int32_t n;
    double u, l;
    int64_t act_begin;  // index into actions, -1 until expanded
    uint64_t z;
};

}  // namespace

struct hdx_tree {
    int32_t n_actions;
    double gamma;
    std::vector<Node> nodes;
    std::vector<ActionBranch> actions;
    mutable std::mutex mu;
};

extern "C" {

hdx_status hdx_tree_create(int32_t n_actions, double gamma, int32_t n_root, double u0, double l0, hdx_tree **out) {
    if (!out || n_actions < 1 || n_root < 1 || !(gamma > 0.0 && gamma <= 1.0)) return HDX_E_INVALID;
    hdx_tree *t = new hdx_tree();
    t->n_actions = n_actions;
    t->gamma = gamma;
    t->nodes.push_back(Node{-1, n_root, u0, l0, -1, 0});
    *out = t;
    return HDX_OK;
}

hdx_status hdx_tree_destroy(hdx_tree *t) {
    if (!t) return HDX_E_INVALID;
    delete t;
    return HDX_OK;
}

int64_t hdx_tree_size(const hdx_tree *t) {
    if (!t) return -1;
    std::lock_guard<std::mutex> g(t->mu);
    return (int64_t)t->nodes.size();
}

hdx_status hdx_tree_add_children(hdx_tree *t, int64_t node, const int32_t *n_children, const uint64_t *child_z,
                                 const int32_t *child_n, const float *child_u0, const float *child_l0,
                                 const float *r_mean, int32_t cap, int64_t *first_child) {
    if (!t || !n_children || !child_z || !child_n || !child_u0 || !child_l0 || !r_mean || cap < 0)
        return HDX_E_INVALID;
    std::lock_guard<std::mutex> g(t->mu);
    if (node < 0 || node >= (int64_t)t->nodes.size() || t->nodes[node].act_begin >= 0) return HDX_E_INVALID;
    const int32_t nb = t->nodes[node].n;
    for (int a = 0; a < t->n_actions; ++a) {
        if (n_children[a] < 0 || n_children[a] > cap) return HDX_E_INVALID;
        int64_t sum = 0;
        for (int c = 0; c < n_children[a]; ++c) sum += child_n[(int64_t)a * cap + c];
        if (sum != nb) return HDX_E_INVALID;  // each scenario reaches exactly one child
    }
    const int64_t first = (int64_t)t->nodes.size();
    t->nodes[node].act_begin = (int64_t)t->actions.size();
    for (int a = 0; a < t->n_actions; ++a) {
        t->actions.push_back(ActionBranch{(double)r_mean[a], (int64_t)t->nodes.size(), n_children[a]});
        for (int c = 0; c < n_children[a]; ++c) {
            const int64_t o = (int64_t)a * cap + c;
            t->nodes.push_back(Node{node, child_n[o], (double)child_u0[o], (double)child_l0[o], -1, child_z[o]});
        }
    }
    if (first_child) *first_child = first;
    return HDX_OK;
}

hdx_status hdx_backup(hdx_tree *t, int64_t node) {
    if (!t) return HDX_E_INVALID;
    std::lock_guard<std::mutex> g(t->mu);
    if (node < 0 || node >= (int64_t)t->nodes.size()) return HDX_E_INVALID;
    for (int64_t b = node; b >= 0; b = t->nodes[b].parent) {
        Node &nb = t->nodes[b];
        if (nb.act_begin < 0) continue;
        double best_u = -std::numeric_limits<double>::infinity(), best_l = best_u;
        for (int a = 0; a < t->n_actions; ++a) {
            const ActionBranch &ab = t->actions[nb.act_begin + a];
            double su = 0.0, sl = 0.0;
            for (int c = 0; c < ab.n_children; ++c) {
                const Node &k = t->nodes[ab.child_begin + c];
                const double w = (double)k.n / (double)nb.n;
                su += w * k.u;
                sl += w * k.l;
            }
            best_u = std::max(best_u, ab.r_mean + t->gamma * su);
            best_l = std::max(best_l, ab.r_mean + t->gamma * sl);
        }
        nb.u = best_u;
        nb.l = best_l;
    }
    return HDX_OK;
}

hdx_status hdx_tree_bounds(const hdx_tree *t, int64_t node, double *u, double *l) {
    if (!t || !u || !l) return HDX_E_INVALID;
    std::lock_guard<std::mutex> g(t->mu);
    if (node < 0 || node >= (int64_t)t->nodes.size()) return HDX_E_INVALID;
    *u = t->nodes[node].u;
    *l = t->nodes[node].l;
    return HDX_OK;
}

}  // extern "C"

// ---- Belief update of the online loop (Sec. III-A, Eq. 3) ----------------
// RockSample's state is the robot cell, which moves deterministically, and
// the rock qualities, independent a priori and each touched by at most one
// action per step; the belief factors into the cell and one probability per
// rock, and Eq. 3 (Bayes' rule over the transition and the observation
// likelihood) reduces to: a move sets the cell, sampling makes the rock
// under the robot bad, and a reading z of rock i at Euclidean distance d is
// correct with probability acc(d) = 0.5 + 0.5 2^(-d/20), so
// P'(good) = P(good) L(z|good) / (P(good) L(z|good) + P(bad) L(z|bad)).
extern "C" hdx_status hdx_belief_update(const hdx_model_desc *d, const hdx_belief *b, int32_t action, uint64_t z,
                                        hdx_belief *out, double *p_out, int32_t *terminal) {
    if (!d || !b || !out || !terminal || (d->n_rocks > 0 && (!b->p_good || !p_out))) return HDX_E_INVALID;
    if (d->kind != HDX_ROCKSAMPLE) return HDX_E_UNSUPPORTED;
    const int n = d->grid, m = d->n_rocks;
    if (action < 0 || action >= 5 + m || b->x < 0 || b->x >= n || b->y < 0 || b->y >= n) return HDX_E_INVALID;
    if (action >= 5 && z != 1 && z != 2) return HDX_E_INVALID;  // a reading is good (1) or bad (2)
    for (int i = 0; i < m; ++i) p_out[i] = b->p_good[i];
    *out = *b;
    out->p_good = p_out;
    *terminal = 0;
    int x = b->x, y = b->y;
    if (action == 0 && y + 1 < n) y += 1;       // north
    else if (action == 1 && y > 0) y -= 1;      // south
    else if (action == 3 && x > 0) x -= 1;      // west
    else if (action == 2) {                     // east; leaving the grid ends the episode
        if (x + 1 >= n) *terminal = 1;
        else x += 1;
    } else if (action == 4) {
        for (int i = 0; i < m; ++i)
            if (d->rock_x[i] == b->x && d->rock_y[i] == b->y) p_out[i] = 0.0;
    } else if (action >= 5) {
        const int i = action - 5;
        const double dx = (double)(b->x - d->rock_x[i]), dy = (double)(b->y - d->rock_y[i]);
        const double acc = 0.5 + 0.5 * pow(2.0, -sqrt(dx * dx + dy * dy) / 20.0);
        const double lg = z == 1 ? acc : 1.0 - acc, lb = z == 1 ? 1.0 - acc : acc;
        const double den = b->p_good[i] * lg + (1.0 - b->p_good[i]) * lb;
        if (den > 0.0) p_out[i] = b->p_good[i] * lg / den;
    }
    out->x = x;
    out->y = y;
    return HDX_OK;
}
