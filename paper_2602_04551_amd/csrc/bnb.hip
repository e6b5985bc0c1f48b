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

#include "bnb_core.hpp"
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

// Per-node results of a batch, gathered into one array for a single read-back.
struct NodeOut {
    double lb, primal, obj;
    int32_t iters, status, ssize, bj, zup, pad;
};

__global__ void k_pack_out(const double *__restrict__ lb, const double *__restrict__ primal,
                           const double *__restrict__ obj, const int32_t *__restrict__ iters,
                           const int32_t *__restrict__ status, const int32_t *__restrict__ ssize,
                           const int32_t *__restrict__ bj, const int32_t *__restrict__ zup, NodeOut *__restrict__ out,
                           int64_t K) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    out[k] = NodeOut{lb[k], primal[k], obj[k], iters[k], status[k], ssize[k], bj[k], zup[k], 0};
}

// Pinned host staging memory, grown on demand (only between synchronised batches).
struct PinnedBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void ensure(size_t n) {
        if (n <= bytes) return;
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        bytes = 0;
        HIPCHK(hipHostMalloc(&ptr, n, hipHostMallocDefault));
        bytes = n;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
    ~PinnedBuf() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

// Device pool of (beta, V) rows indexed by the core's warm-start slots.
struct DevicePool {
    DevBuf buf;
    int64_t cap = 0, pp = 0;
    size_t sb = 8;
    void ensure(int64_t slots, hipStream_t st) {
        if (slots <= cap) return;
        int64_t ncap = std::max<int64_t>({64, cap * 2, slots});
        DevBuf nb;
        nb.ensure(sb * 2 * pp * (size_t)ncap);
        if (cap) HIPCHK(hipMemcpyAsync(nb.ptr, buf.ptr, sb * 2 * pp * (size_t)cap, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        std::swap(buf.ptr, nb.ptr);
        std::swap(buf.bytes, nb.bytes);
        std::swap(buf.charged, nb.charged);
        cap = ncap;
    }
};

template <class T>
void bnb_t(l0l2_ctx *ctx, const l0l2_bnb_opts &o, l0l2_bnb_result *out) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t st = ctx->stream;
    // state and code rows (and the warm-start pool's rows) have stride ldp
    const int64_t p = in.p, pp = in.ldp;
    const int K = std::max(1, o.K);
    ensure_workspace(ctx, K);
    DevicePool pool;
    pool.pp = pp;
    pool.sb = state_bytes(in.prec);

    // per batch: one host-to-device copy of [slots | fixing offsets | fixings], one
    // device-to-host copy of the packed results, one copy of the scatter pairs
    DevBuf d_in, d_sc, d_out, d_sup, d_ssize, d_bj, d_zup, d_nfree, d_fbeta, d_obj, d_fit;
    PinnedBuf h_in, h_sc, h_out;
    d_sc.ensure(sizeof(int64_t) * 2 * K);
    d_out.ensure(sizeof(NodeOut) * K);
    h_sc.ensure(sizeof(int64_t) * 2 * K);
    h_out.ensure(sizeof(NodeOut) * K);
    d_sup.ensure((size_t)K * p);
    d_ssize.ensure(sizeof(int32_t) * K);
    d_bj.ensure(sizeof(int32_t) * K);
    d_zup.ensure(sizeof(int32_t) * K);
    d_nfree.ensure(sizeof(int32_t) * K);
    d_fbeta.ensure(sizeof(double) * (size_t)K * p);
    d_obj.ensure(sizeof(double) * K);
    d_fit.ensure(sizeof(int32_t) * K);

    BnbCore core(o);
    std::vector<uint8_t> inc_mask((size_t)p, 0);
    if (o.root_heuristic == 1) {
        // Sec. 3.5: the matching-pursuit support, solved exactly, is the first incumbent
        std::vector<uint8_t> mp_mask((size_t)p, 0);
        std::vector<double> mp_beta((size_t)p, 0.0);
        int32_t nm = 0;
        double mp_obj = 0.0;
        const int64_t mm = 4 * std::min(in.n, in.p);
        run_matching_pursuit(ctx, (int)std::min<int64_t>(mm, 1 << 30), mp_mask.data(), mp_beta.data(), nullptr, &nm,
                             &mp_obj);
        const double f = run_exact_objective(ctx, mp_mask.data(), mp_beta.data());
        if (std::isfinite(f) && core.seed_incumbent(f)) inc_mask = mp_mask;
    }
    if (o.init_support) {
        // a support given by the caller (e.g. the previous point of a lambda0
        // path), solved exactly at the current penalties
        std::vector<uint8_t> m0((size_t)p, 0);
        for (int64_t j = 0; j < p; ++j) m0[(size_t)j] = o.init_support[j] ? 1 : 0;
        std::vector<double> b0((size_t)p, 0.0);
        const double f = run_exact_objective(ctx, m0.data(), b0.data());
        if (std::isfinite(f) && core.seed_incumbent(f)) inc_mask = m0;
    }
    const size_t row_bytes = state_bytes(in.prec) * (size_t)pp;
    int64_t batches = 0;
    int status = 0;
    std::vector<OpenNode> batch;
    std::vector<int32_t> h_fix;
    std::vector<NodeOutcome> res(K);
    std::vector<std::pair<int, int64_t>> saves;

    while (!core.frontier_empty()) {
        check_cancel(ctx);
        if ((status = core.gap_reached()) != 0) break;
        if (o.time_limit_s > 0 && std::chrono::duration<double>(clock::now() - t0).count() > o.time_limit_s) {
            status = 3;
            break;
        }
        if (core.solved() >= o.max_nodes) { status = 1; break; }
        core.select(K, batch);
        const int B = (int)batch.size();
        if (B == 0) continue;
        ++batches;
        // input layout: B slots (int64), B + 1 fixing offsets (int32), the fixings (int32)
        h_fix.clear();
        std::vector<int32_t> offs((size_t)B + 1, 0);
        for (int k = 0; k < B; ++k) {
            core.fixings(batch[k].id, h_fix);
            offs[(size_t)k + 1] = (int32_t)h_fix.size();
        }
        const size_t in_bytes = sizeof(int64_t) * B + sizeof(int32_t) * ((size_t)B + 1 + h_fix.size());
        h_in.ensure(in_bytes);
        d_in.ensure(in_bytes);
        int64_t *hs = h_in.as<int64_t>();
        for (int k = 0; k < B; ++k) hs[k] = batch[k].slot;
        int32_t *ho = reinterpret_cast<int32_t *>(hs + B);
        std::memcpy(ho, offs.data(), sizeof(int32_t) * ((size_t)B + 1));
        if (!h_fix.empty()) std::memcpy(ho + B + 1, h_fix.data(), sizeof(int32_t) * h_fix.size());
        HIPCHK(hipMemcpyAsync(d_in.ptr, h_in.ptr, in_bytes, hipMemcpyHostToDevice, st));
        const int64_t *d_slot = d_in.as<int64_t>();
        const int32_t *d_off = reinterpret_cast<const int32_t *>(d_slot + B);
        const int32_t *d_fix = d_off + B + 1;
        const int64_t Bp = round_up(B, kPadNodes);
        hipLaunchKernelGGL(k_build_codes, dim3((unsigned)Bp), dim3(256), 0, st, ws.codes.as<uint8_t>(), pp, p,
                           (int64_t)B, Bp, d_off, d_fix);
        hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)((pp + 255) / 256), (unsigned)Bp), dim3(256), 0, st,
                           ws.beta.as<T>(), ws.V.as<T>(), pp, (const T *)pool.buf.ptr, d_slot, Bp, (int64_t)B);
        HIPCHK(hipGetLastError());
        core.gathered(batch);
        l0l2_admm_opts ao = o.admm;
        const bool root = batch[0].id == 0;
        if (root) ao.max_iter = o.max_iter_root;
        if (root && o.warm_root && ws.have_root && ws.root_beta.bytes >= row_bytes) {
            // Sec. 3.1.3 across solves: the root starts from the previous tree's root iterates
            HIPCHK(hipMemcpyAsync(ws.beta.ptr, ws.root_beta.ptr, row_bytes, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(ws.V.ptr, ws.root_v.ptr, row_bytes, hipMemcpyDeviceToDevice, st));
        }
        run_solve(ctx, B, ao);
        if (root) {
            ws.root_beta.ensure(row_bytes);
            ws.root_v.ensure(row_bytes);
            HIPCHK(hipMemcpyAsync(ws.root_beta.ptr, ws.beta.ptr, row_bytes, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(ws.root_v.ptr, ws.V.ptr, row_bytes, hipMemcpyDeviceToDevice, st));
            ws.have_root = true;
        }
        run_round_branch(ctx, B, ws.codes.as<uint8_t>(), pp, ws.beta.ptr, pp, d_sup.as<uint8_t>(),
                         d_ssize.as<int32_t>(), d_bj.as<int32_t>(), d_zup.as<int32_t>(), d_nfree.as<int32_t>());
        state_to_f64(ctx, B, ws.beta.ptr, pp, d_fbeta.as<double>(), p);
        run_fista(ctx, B, d_sup.as<uint8_t>(), p, d_fbeta.as<double>(), p, o.fista, d_obj.as<double>(),
                  d_fit.as<int32_t>());
        hipLaunchKernelGGL(k_pack_out, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, ws.lb.as<double>(),
                           ws.primal.as<double>(), d_obj.as<double>(), ws.iters.as<int32_t>(), ws.status.as<int32_t>(),
                           d_ssize.as<int32_t>(), d_bj.as<int32_t>(), d_zup.as<int32_t>(), d_out.as<NodeOut>(),
                           (int64_t)B);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h_out.ptr, d_out.ptr, sizeof(NodeOut) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const NodeOut *ho_res = h_out.as<NodeOut>();
        for (int k = 0; k < B; ++k) {
            const NodeOut &r = ho_res[k];
            if (!std::isfinite(r.obj)) fail(L0L2_E_UNSUPPORTED, "support larger than the refinement kernel allows");
            res[k] = NodeOutcome{r.lb, r.primal, r.iters, r.status, r.obj, r.ssize, r.bj, r.zup};
        }
        int best_k;
        core.process(batch, res.data(), saves, best_k);
        if (best_k >= 0)
            HIPCHK(hipMemcpyAsync(inc_mask.data(), d_sup.as<uint8_t>() + (size_t)best_k * p, (size_t)p,
                                  hipMemcpyDeviceToHost, st));
        if (!saves.empty()) {
            pool.ensure(core.slot_high_water(), st);
            const int64_t ns = (int64_t)saves.size();
            int64_t *hr = h_sc.as<int64_t>();
            for (int64_t e = 0; e < ns; ++e) {
                hr[e] = saves[(size_t)e].first;
                hr[ns + e] = saves[(size_t)e].second;
            }
            HIPCHK(hipMemcpyAsync(d_sc.ptr, h_sc.ptr, sizeof(int64_t) * 2 * ns, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL((k_scatter<T>), dim3((unsigned)((pp + 255) / 256), (unsigned)ns), dim3(256), 0, st,
                               ws.beta.as<T>(), ws.V.as<T>(), pp, (T *)pool.buf.ptr, d_sc.as<int64_t>(),
                               d_sc.as<int64_t>() + ns, ns);
            HIPCHK(hipGetLastError());
        }
        // no wait here: the next batch's copies and kernels follow in stream order,
        // and the staging buffers are rewritten only after its results are read
    }
    HIPCHK(hipStreamSynchronize(st));
    const double UB = core.ub();
    out->ub = UB;
    // every support lies in a closed node (pruned: its bound reached UB (1 - eps);
    // a leaf) or an open one, so the smallest of their bounds bounds the optimum
    out->lb = std::min(UB, std::min(core.closed_lb(), status == 0 ? INFINITY : core.frontier_lb()));
    out->nodes_solved = core.solved();
    out->nodes_pruned = core.pruned();
    out->trace_len = core.trace_len();
    out->batches = batches;
    out->status = status;
    std::vector<double> bex((size_t)p, 0.0);
    out->certified = core.have_incumbent() ? run_exact_objective(ctx, inc_mask.data(), bex.data()) : INFINITY;
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
    else bnb_t<float>(ctx, o, out);
}

}  // namespace l0l2
