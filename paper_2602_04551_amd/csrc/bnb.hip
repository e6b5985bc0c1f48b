// Branch and bound over node batches (Alg. 1, Sec. 2.4).
//
// The host keeps the frontier, the incumbent and the decisions; each batch of up
// to K nodes is solved on the GPU (relaxation, rounding, branching index,
// incumbent refinement) with the warm starts of Sec. 3.1.3 gathered from a
// device-resident pool of parent states.  Per batch the host sends the fixing
// lists and pool slots of the nodes and reads back K-sized result arrays.
//
// Decisions follow Alg. 1 in the order the batch was selected: prune when the
// node bound reaches UB (1 - eps_prune); else take its incumbent; else branch on
// the chosen index.  A child inherits max(LB_u, inherited bound) and is
// discarded at selection when that already prunes it; a node without free
// coordinates is closed after its incumbent is taken.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <vector>

#include "device_math.hpp"
#include "internal.hpp"

namespace l0l2 {

namespace {

// codes[k][j] = FREE for j < p (FIX0 on padding), then the node's fixings.
__global__ void k_build_codes(uint8_t *__restrict__ codes, int64_t pp, int64_t p, int64_t K, int64_t Kp,
                              const int32_t *__restrict__ off, const int32_t *__restrict__ fix) {
    const int64_t k = blockIdx.x;
    if (k >= Kp) return;
    uint8_t *row = codes + k * pp;
    for (int64_t j = threadIdx.x; j < pp; j += blockDim.x)
        row[j] = (k < K && j < p) ? (uint8_t)CODE_FREE : (uint8_t)CODE_FIX0;
    __syncthreads();
    if (k >= K) return;
    for (int32_t e = off[k] + threadIdx.x; e < off[k + 1]; e += blockDim.x) {
        int32_t v = fix[e];
        row[v >> 2] = (uint8_t)(v & 3);
    }
}

// rows k of beta / V <- pool slot slot[k] (zeros for slot -1).
template <class T>
__global__ void k_gather(T *__restrict__ beta, T *__restrict__ V, int64_t pp, const T *__restrict__ pool,
                         const int64_t *__restrict__ slot, int64_t Kp, int64_t K) {
    const int64_t k = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pp || k >= Kp) return;
    int64_t s = k < K ? slot[k] : -1;
    T b = 0, v = 0;
    if (s >= 0) {
        b = pool[(2 * s) * pp + j];
        v = pool[(2 * s + 1) * pp + j];
    }
    beta[k * pp + j] = b;
    V[k * pp + j] = v;
}

// pool slot slot[e] <- rows row[e] of beta / V.
template <class T>
__global__ void k_scatter(const T *__restrict__ beta, const T *__restrict__ V, int64_t pp, T *__restrict__ pool,
                          const int64_t *__restrict__ row, const int64_t *__restrict__ slot, int64_t cnt) {
    const int64_t e = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pp || e >= cnt) return;
    int64_t k = row[e], s = slot[e];
    pool[(2 * s) * pp + j] = beta[k * pp + j];
    pool[(2 * s + 1) * pp + j] = V[k * pp + j];
}

struct TreeNode {
    int64_t parent;   // arena index of the parent (-1 root)
    int32_t j;        // fixed coordinate (-1 root)
    int32_t fix;      // CODE_FIX0 / CODE_FIX1
};

struct OpenNode {
    double lb;        // inherited bound
    int64_t id;       // arena index = creation order
    int64_t slot;     // warm-start pool slot (-1: zero start)
    int32_t depth;
};

struct HeapCmp {
    bool operator()(const OpenNode &a, const OpenNode &b) const {
        if (a.lb != b.lb) return a.lb > b.lb;
        return a.id > b.id;
    }
};

// Device pool of (beta, V) rows, one slot per branched node until both
// children have been gathered.
struct StatePool {
    DevBuf buf;
    int64_t cap = 0, pp = 0;
    size_t sb = 8;
    std::vector<int64_t> free_list;
    std::vector<int32_t> refs;
    int64_t used = 0, high = 0;

    void init(int64_t pp_, size_t sb_) { pp = pp_; sb = sb_; }
    int64_t alloc(hipStream_t st) {
        if (free_list.empty()) {
            int64_t ncap = std::max<int64_t>(64, cap * 2);
            DevBuf nb;
            nb.ensure(sb * 2 * pp * (size_t)ncap);
            if (cap) HIPCHK(hipMemcpyAsync(nb.ptr, buf.ptr, sb * 2 * pp * (size_t)cap, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            std::swap(buf.ptr, nb.ptr);
            std::swap(buf.bytes, nb.bytes);
            for (int64_t s = ncap - 1; s >= cap; --s) free_list.push_back(s);
            refs.resize((size_t)ncap, 0);
            cap = ncap;
        }
        int64_t s = free_list.back();
        free_list.pop_back();
        refs[(size_t)s] = 2;
        ++used;
        high = std::max(high, used);
        return s;
    }
    void release(int64_t s) {
        if (s < 0) return;
        if (--refs[(size_t)s] == 0) {
            free_list.push_back(s);
            --used;
        }
    }
};

template <class T>
void bnb_t(l0l2_ctx *ctx, const l0l2_bnb_opts &o, l0l2_bnb_result *out) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t st = ctx->stream;
    const int64_t p = in.p, pp = in.pp;
    const int K = std::max(1, o.K);
    ensure_workspace(ctx, K);

    StatePool pool;
    pool.init(pp, state_bytes(in.prec));

    // per-batch device arrays
    DevBuf d_off, d_fix, d_slot, d_row, d_sslot, d_sup, d_ssize, d_bj, d_zup, d_nfree, d_fbeta, d_obj, d_fit;
    d_off.ensure(sizeof(int32_t) * (K + 1));
    d_slot.ensure(sizeof(int64_t) * K);
    d_row.ensure(sizeof(int64_t) * K);
    d_sslot.ensure(sizeof(int64_t) * K);
    d_sup.ensure((size_t)K * p);
    d_ssize.ensure(sizeof(int32_t) * K);
    d_bj.ensure(sizeof(int32_t) * K);
    d_zup.ensure(sizeof(int32_t) * K);
    d_nfree.ensure(sizeof(int32_t) * K);
    d_fbeta.ensure(sizeof(double) * (size_t)K * p);
    d_obj.ensure(sizeof(double) * K);
    d_fit.ensure(sizeof(int32_t) * K);

    std::vector<TreeNode> arena;
    arena.push_back({-1, -1, 0});
    std::priority_queue<OpenNode, std::vector<OpenNode>, HeapCmp> heap;
    std::vector<OpenNode> stack;
    const bool dfs = o.policy == L0L2_DFS;
    auto push = [&](const OpenNode &u) {
        if (dfs) stack.push_back(u);
        else heap.push(u);
    };
    auto empty = [&]() { return dfs ? stack.empty() : heap.empty(); };
    auto pop = [&]() {
        OpenNode u;
        if (dfs) { u = stack.back(); stack.pop_back(); }
        else { u = heap.top(); heap.pop(); }
        return u;
    };
    push({-INFINITY, 0, -1, 0});

    double UB = INFINITY;
    bool have_inc = false;
    std::vector<uint8_t> inc_mask((size_t)p, 0);
    std::vector<double> inc_beta((size_t)p, 0.0);
    int64_t solved = 0, pruned = 0, tl = 0, batches = 0;
    int status = 0;
    auto trace_put = [&](const l0l2_trace_rec &r) {
        if (o.trace && tl < o.trace_cap) o.trace[tl] = r;
        ++tl;
    };
    const double eps = o.eps_prune;

    std::vector<OpenNode> batch;
    std::vector<int32_t> h_off, h_fix;
    std::vector<int64_t> h_slot, h_row, h_sslot;
    std::vector<double> h_lb(K), h_primal(K), h_obj(K);
    std::vector<int32_t> h_iters(K), h_status(K), h_ssize(K), h_bj(K), h_zup(K), h_nfree(K);

    while (!empty()) {
        if (o.gap_tol > 0.0 && have_inc) {
            double lbg = INFINITY;
            if (dfs) { for (auto &u : stack) lbg = std::min(lbg, u.lb); }
            else lbg = heap.top().lb;
            if (UB - lbg <= o.gap_tol * std::fabs(UB)) { status = 2; break; }
        }
        if (o.time_limit_s > 0 &&
            std::chrono::duration<double>(clock::now() - t0).count() > o.time_limit_s) { status = 3; break; }
        if (solved >= o.max_nodes) { status = 1; break; }
        // select the batch, discarding nodes already pruned by their inherited bound
        batch.clear();
        while (!empty() && (int)batch.size() < K && solved + (int64_t)batch.size() < o.max_nodes) {
            OpenNode u = pop();
            if (have_inc && u.lb >= UB * (1.0 - eps)) {
                ++pruned;
                l0l2_trace_rec r{};
                r.id = u.id; r.parent = arena[(size_t)u.id].parent; r.depth = u.depth; r.branch_j = -1;
                r.decision = 3; r.lb = u.lb; r.ub_global = UB;
                trace_put(r);
                pool.release(u.slot);
                continue;
            }
            batch.push_back(u);
            if (u.id == 0) break;   // the root is solved alone with its own sweep budget
        }
        const int B = (int)batch.size();
        if (B == 0) continue;
        ++batches;
        // fixing lists (walk each node's chain to the root)
        h_off.assign((size_t)B + 1, 0);
        h_fix.clear();
        h_slot.assign((size_t)B, -1);
        for (int k = 0; k < B; ++k) {
            for (int64_t a = batch[k].id; a > 0; a = arena[(size_t)a].parent)
                h_fix.push_back(arena[(size_t)a].j * 4 + arena[(size_t)a].fix);
            h_off[(size_t)k + 1] = (int32_t)h_fix.size();
            h_slot[(size_t)k] = batch[k].slot;
        }
        d_fix.ensure(sizeof(int32_t) * std::max<size_t>(h_fix.size(), 1));
        HIPCHK(hipMemcpyAsync(d_off.ptr, h_off.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, st));
        if (!h_fix.empty())
            HIPCHK(hipMemcpyAsync(d_fix.ptr, h_fix.data(), sizeof(int32_t) * h_fix.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d_slot.ptr, h_slot.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, st));
        const int64_t Bp = round_up(B, kPadNodes);
        hipLaunchKernelGGL(k_build_codes, dim3((unsigned)Bp), dim3(256), 0, st, ws.codes.as<uint8_t>(), pp, p,
                           (int64_t)B, Bp, d_off.as<int32_t>(), d_fix.as<int32_t>());
        hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)((pp + 255) / 256), (unsigned)Bp), dim3(256), 0, st,
                           ws.beta.as<T>(), ws.V.as<T>(), pp, (const T *)pool.buf.ptr, d_slot.as<int64_t>(), Bp,
                           (int64_t)B);
        HIPCHK(hipGetLastError());
        for (int k = 0; k < B; ++k) pool.release(batch[k].slot);
        // node relaxations
        l0l2_admm_opts ao = o.admm;
        if (batch[0].id == 0) ao.max_iter = o.max_iter_root;
        run_solve(ctx, B, ao);
        // rounding, branching, refinement
        run_round_branch(ctx, B, ws.codes.as<uint8_t>(), pp, ws.beta.ptr, pp, d_sup.as<uint8_t>(),
                         d_ssize.as<int32_t>(), d_bj.as<int32_t>(), d_zup.as<int32_t>(), d_nfree.as<int32_t>());
        state_to_f64(ctx, B, ws.beta.ptr, pp, d_fbeta.as<double>(), p);
        run_fista(ctx, B, d_sup.as<uint8_t>(), p, d_fbeta.as<double>(), p, o.fista, d_obj.as<double>(),
                  d_fit.as<int32_t>());
        HIPCHK(hipMemcpyAsync(h_lb.data(), ws.lb.ptr, 8 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_primal.data(), ws.primal.ptr, 8 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_iters.data(), ws.iters.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_status.data(), ws.status.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_ssize.data(), d_ssize.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_bj.data(), d_bj.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_zup.data(), d_zup.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_nfree.data(), d_nfree.ptr, 4 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_obj.data(), d_obj.ptr, 8 * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        solved += B;
        // decisions in selection order
        h_row.clear();
        h_sslot.clear();
        int best_k = -1;
        double best_ub = UB;
        for (int k = 0; k < B; ++k) {
            const OpenNode &u = batch[k];
            l0l2_trace_rec r{};
            r.id = u.id; r.parent = arena[(size_t)u.id].parent; r.depth = u.depth; r.branch_j = -1;
            r.iters = h_iters[k]; r.admm_status = h_status[k]; r.primal = h_primal[k];
            if (!std::isfinite(h_obj[k])) fail(L0L2_E_UNSUPPORTED, "support larger than the refinement kernel allows");
            double lb_eff = std::max(h_lb[k], u.lb);
            r.lb = lb_eff;
            if (have_inc && lb_eff >= UB * (1.0 - eps)) {
                ++pruned;
                r.decision = 1; r.ub_global = UB;
                trace_put(r);
                continue;
            }
            r.ub_node = h_obj[k]; r.support_size = h_ssize[k];
            if (h_obj[k] < UB) {
                UB = h_obj[k];
                have_inc = true;
                best_k = k;
                best_ub = UB;
            }
            r.ub_global = UB;
            if (h_bj[k] < 0) {
                r.decision = 2;
                trace_put(r);
                continue;
            }
            r.decision = 0; r.branch_j = h_bj[k];
            trace_put(r);
            int64_t slot = pool.alloc(st);
            h_row.push_back(k);
            h_sslot.push_back(slot);
            int64_t id0 = (int64_t)arena.size();
            arena.push_back({u.id, h_bj[k], CODE_FIX0});
            int64_t id1 = (int64_t)arena.size();
            arena.push_back({u.id, h_bj[k], CODE_FIX1});
            OpenNode c0{lb_eff, id0, slot, u.depth + 1}, c1{lb_eff, id1, slot, u.depth + 1};
            if (h_zup[k]) { push(c0); push(c1); }
            else { push(c1); push(c0); }
        }
        (void)best_ub;
        if (best_k >= 0) {
            HIPCHK(hipMemcpyAsync(inc_mask.data(), d_sup.as<uint8_t>() + (size_t)best_k * p, (size_t)p,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(inc_beta.data(), d_fbeta.as<double>() + (size_t)best_k * p, 8 * (size_t)p,
                                  hipMemcpyDeviceToHost, st));
        }
        if (!h_row.empty()) {
            HIPCHK(hipMemcpyAsync(d_row.ptr, h_row.data(), 8 * h_row.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(d_sslot.ptr, h_sslot.data(), 8 * h_sslot.size(), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL((k_scatter<T>), dim3((unsigned)((pp + 255) / 256), (unsigned)h_row.size()), dim3(256),
                               0, st, ws.beta.as<T>(), ws.V.as<T>(), pp, (T *)pool.buf.ptr, d_row.as<int64_t>(),
                               d_sslot.as<int64_t>(), (int64_t)h_row.size());
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    double lbg = UB;
    if (status != 0) {
        if (dfs) { for (auto &u : stack) lbg = std::min(lbg, u.lb); }
        else if (!heap.empty()) lbg = std::min(lbg, heap.top().lb);
        for (auto &u : batch) (void)u;
    }
    out->ub = UB;
    out->lb = status == 0 ? UB : lbg;
    out->nodes_solved = solved;
    out->nodes_pruned = pruned;
    out->trace_len = tl;
    out->batches = batches;
    out->status = status;
    std::vector<double> bex((size_t)p, 0.0);
    out->certified = have_inc ? run_exact_objective(ctx, inc_mask.data(), bex.data()) : INFINITY;
    int64_t ns = 0;
    for (int64_t j = 0; j < p; ++j) ns += inc_mask[(size_t)j] != 0;
    out->support_len = ns;
    out->support = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(ns, 1));
    out->beta = (double *)std::malloc(sizeof(double) * (size_t)p);
    ns = 0;
    for (int64_t j = 0; j < p; ++j)
        if (inc_mask[(size_t)j]) out->support[ns++] = (int32_t)j;
    std::memcpy(out->beta, bex.data(), sizeof(double) * (size_t)p);
    out->seconds = std::chrono::duration<double>(clock::now() - t0).count();
}

}  // namespace

void bnb_solve(l0l2_ctx *ctx, const l0l2_bnb_opts &o, l0l2_bnb_result *out) {
    if (ctx->inst.prec == L0L2_FP64) bnb_t<double>(ctx, o, out);
    else if (ctx->inst.prec == L0L2_FP32) bnb_t<float>(ctx, o, out);
    else fail(L0L2_E_UNSUPPORTED, "BF16 branch and bound is not available in this build");
}

}  // namespace l0l2
