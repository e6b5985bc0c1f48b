// Host logic of the branch and bound (Alg. 1, Sec. 2.2 and 2.4), independent of
// any device: the frontier (best-first by (inherited LB, id) or LIFO), batch
// selection with pruning of nodes whose inherited bound already reaches the
// incumbent, the per-node decisions in selection order, child creation, the
// trace, and reference counts of the warm-start slots that children share.
// The node relaxations themselves are supplied by the caller per batch.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <queue>
#include <vector>

#include "../../include/l0l2.h"

namespace l0l2 {

// What the device computed for one node of a batch.
struct NodeOutcome {
    double lb;            // rigorous bound of the relaxation
    double primal;        // P(beta) at the final iterate
    int32_t iters, status;
    double ub;            // F(S, beta) of the refined incumbent candidate
    int32_t support_size;
    int32_t branch_j;     // -1 when no coordinate is free
    int32_t z_up;         // z at branch_j >= 1/2
};

struct OpenNode {
    double lb;            // inherited bound
    int64_t id;           // creation order (root 0)
    int64_t slot;         // warm-start slot (-1: zero start)
    int32_t depth;
};

class BnbCore {
  public:
    enum : uint8_t { FIX0 = 1, FIX1 = 2 };

    explicit BnbCore(const l0l2_bnb_opts &o) : o_(o), dfs_(o.policy == L0L2_DFS) {
        arena_.push_back({-1, -1, 0});
        push({-INFINITY, 0, -1, 0});
    }

    bool frontier_empty() const { return dfs_ ? stack_.empty() : heap_.empty(); }
    double ub() const { return ub_; }
    bool have_incumbent() const { return have_inc_; }
    int64_t solved() const { return solved_; }
    int64_t pruned() const { return pruned_; }
    int64_t trace_len() const { return tl_; }
    int64_t slots_in_use() const { return used_; }
    int64_t slot_high_water() const { return (int64_t)refs_.size(); }
    // Smallest bound among the closed nodes (pruned or leaves): with the open
    // nodes' bounds it bounds the optimum from below (+inf when none closed).
    double closed_lb() const { return closed_lb_; }

    // An incumbent found before the tree (the root heuristic): its objective
    // becomes UB when it is smaller.  Returns whether it did.
    bool seed_incumbent(double ub) {
        if (!(ub < ub_)) return false;
        ub_ = ub;
        have_inc_ = true;
        return true;
    }

    // Smallest inherited bound over the open nodes (+inf when none).
    double frontier_lb() const {
        if (dfs_) {
            double m = INFINITY;
            for (const auto &u : stack_) m = std::min(m, u.lb);
            return m;
        }
        return heap_.empty() ? INFINITY : heap_.top().lb;
    }

    // Stop condition before selecting a batch: 0 continue, 2 gap_tol reached.
    int gap_reached() const {
        if (o_.gap_tol > 0.0 && have_inc_ && !frontier_empty())
            if (ub_ - frontier_lb() <= o_.gap_tol * std::fabs(ub_)) return 2;
        return 0;
    }

    // Pop up to K nodes; nodes whose inherited bound prunes them are closed
    // (decision 3) and release their warm-start slot.  The root is solved alone.
    void select(int K, std::vector<OpenNode> &batch) {
        batch.clear();
        while (!frontier_empty() && (int)batch.size() < K &&
               solved_ + (int64_t)batch.size() < o_.max_nodes) {
            OpenNode u = pop();
            if (have_inc_ && u.lb >= ub_ * (1.0 - o_.eps_prune)) {
                ++pruned_;
                l0l2_trace_rec r = rec(u);
                r.decision = 3;
                r.lb = u.lb;
                r.ub_global = ub_;
                closed_lb_ = std::min(closed_lb_, u.lb);
                put(r);
                release(u.slot);
                continue;
            }
            batch.push_back(u);
            if (u.id == 0) break;
        }
    }

    // Fixings of a node as j * 4 + code, walking its chain to the root.
    void fixings(int64_t id, std::vector<int32_t> &out) const {
        for (int64_t a = id; a > 0; a = arena_[(size_t)a].parent)
            out.push_back(arena_[(size_t)a].j * 4 + arena_[(size_t)a].fix);
    }

    // The batch's warm-start slots have been read by the device.
    void gathered(const std::vector<OpenNode> &batch) {
        for (const auto &u : batch) release(u.slot);
    }

    // Decisions for the batch in selection order.  For every branched node the
    // caller must save that node's final iterates into saves[i].second (a slot
    // index).  best_k = batch index of the new incumbent (-1 if none).
    void process(const std::vector<OpenNode> &batch, const NodeOutcome *res,
                 std::vector<std::pair<int, int64_t>> &saves, int &best_k) {
        saves.clear();
        best_k = -1;
        solved_ += (int64_t)batch.size();
        for (size_t k = 0; k < batch.size(); ++k) {
            const OpenNode &u = batch[k];
            const NodeOutcome &x = res[k];
            l0l2_trace_rec r = rec(u);
            r.iters = x.iters;
            r.admm_status = x.status;
            r.primal = x.primal;
            double lb_eff = std::max(x.lb, u.lb);
            r.lb = lb_eff;
            if (have_inc_ && lb_eff >= ub_ * (1.0 - o_.eps_prune)) {
                ++pruned_;
                r.decision = 1;
                r.ub_global = ub_;
                closed_lb_ = std::min(closed_lb_, lb_eff);
                put(r);
                continue;
            }
            r.ub_node = x.ub;
            r.support_size = x.support_size;
            if (x.ub < ub_) {
                ub_ = x.ub;
                have_inc_ = true;
                best_k = (int)k;
            }
            r.ub_global = ub_;
            if (x.branch_j < 0) {
                r.decision = 2;
                closed_lb_ = std::min(closed_lb_, lb_eff);
                put(r);
                continue;
            }
            r.decision = 0;
            r.branch_j = x.branch_j;
            put(r);
            int64_t slot = alloc();
            saves.push_back({(int)k, slot});
            int64_t id0 = (int64_t)arena_.size();
            arena_.push_back({u.id, x.branch_j, FIX0});
            int64_t id1 = (int64_t)arena_.size();
            arena_.push_back({u.id, x.branch_j, FIX1});
            OpenNode c0{lb_eff, id0, slot, u.depth + 1}, c1{lb_eff, id1, slot, u.depth + 1};
            if (x.z_up) { push(c0); push(c1); }
            else { push(c1); push(c0); }
        }
    }

  private:
    struct TreeNode {
        int64_t parent;
        int32_t j, fix;
    };
    struct HeapCmp {
        bool operator()(const OpenNode &a, const OpenNode &b) const {
            if (a.lb != b.lb) return a.lb > b.lb;
            return a.id > b.id;
        }
    };

    void push(const OpenNode &u) {
        if (dfs_) stack_.push_back(u);
        else heap_.push(u);
    }
    OpenNode pop() {
        OpenNode u;
        if (dfs_) { u = stack_.back(); stack_.pop_back(); }
        else { u = heap_.top(); heap_.pop(); }
        return u;
    }
    l0l2_trace_rec rec(const OpenNode &u) const {
        l0l2_trace_rec r{};
        r.id = u.id;
        r.parent = arena_[(size_t)u.id].parent;
        r.depth = u.depth;
        r.branch_j = -1;
        return r;
    }
    void put(const l0l2_trace_rec &r) {
        if (o_.trace && tl_ < o_.trace_cap) o_.trace[tl_] = r;
        ++tl_;
    }
    int64_t alloc() {
        int64_t s;
        if (!free_.empty()) { s = free_.back(); free_.pop_back(); }
        else { s = (int64_t)refs_.size(); refs_.push_back(0); }
        refs_[(size_t)s] = 2;
        ++used_;
        return s;
    }
    void release(int64_t s) {
        if (s < 0) return;
        if (--refs_[(size_t)s] == 0) {
            free_.push_back(s);
            --used_;
        }
    }

    l0l2_bnb_opts o_;
    bool dfs_;
    std::vector<TreeNode> arena_;
    std::priority_queue<OpenNode, std::vector<OpenNode>, HeapCmp> heap_;
    std::vector<OpenNode> stack_;
    double ub_ = INFINITY;
    double closed_lb_ = INFINITY;
    bool have_inc_ = false;
    int64_t solved_ = 0, pruned_ = 0, tl_ = 0, used_ = 0;
    std::vector<int32_t> refs_;
    std::vector<int64_t> free_;
};

}  // namespace l0l2
