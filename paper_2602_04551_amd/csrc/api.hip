// extern "C" entry points of libl0l2 (include/l0l2.h): argument validation,
// error capture and dispatch.  No exception crosses this boundary.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace l0l2 {

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory) ? L0L2_E_OOM : L0L2_E_DEVICE;
        fail(code, std::string(what) + ": " + hipGetErrorString(e));
    }
}

void drop_graphs(l0l2_ctx *ctx) {
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
}

MemCount &global_mem() {
    static MemCount m;
    return m;
}

MemCount *&thread_mem() {
    static thread_local MemCount *m = nullptr;
    return m;
}

void DevBuf::release() {
    if (ptr) {
        (void)hipFree(ptr);
        global_mem().sub(bytes);
        if (charged) charged->sub(bytes);
    }
    ptr = nullptr;
    bytes = 0;
    charged = nullptr;
}

void DevBuf::ensure(size_t b) {
    if (b <= bytes && ptr) return;
    release();
    if (b == 0) b = 1;
    hipError_t e = hipMalloc(&ptr, b);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        fail(L0L2_E_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
    global_mem().add(b);
    charged = thread_mem();
    if (charged) charged->add(b);
}

}  // namespace l0l2

using l0l2::Error;

namespace {

thread_local std::string g_create_err;

template <class F>
int guarded(l0l2_ctx *ctx, F &&f) {
    if (!ctx) return L0L2_E_INVALID;
    // work of the call runs on the context's stream after everything already
    // queued on the caller's stream, and the caller's stream waits for it
    auto order_out = [&] {
        if (hipEventRecord(ctx->ev_out, ctx->stream) == hipSuccess)
            (void)hipStreamWaitEvent(ctx->user_stream, ctx->ev_out, 0);
    };
    // allocations made by this call are charged to ctx
    struct Charge {
        l0l2::MemCount *prev;
        explicit Charge(l0l2::MemCount *m) : prev(l0l2::thread_mem()) { l0l2::thread_mem() = m; }
        ~Charge() { l0l2::thread_mem() = prev; }
    } charge(&ctx->mem);
    try {
        if (hipSetDevice(ctx->device) != hipSuccess) l0l2::fail(L0L2_E_DEVICE, "hipSetDevice failed");
        HIPCHK(hipEventRecord(ctx->ev_in, ctx->user_stream));
        HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
        f();
        order_out();
        ctx->err.clear();
        return L0L2_OK;
    } catch (const Error &e) {
        order_out();
        ctx->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        order_out();
        ctx->err = "host allocation failed";
        return L0L2_E_OOM;
    } catch (...) {
        order_out();
        ctx->err = "unexpected internal error";
        return L0L2_E_DEVICE;
    }
}

void need_data(l0l2_ctx *ctx) {
    if (!ctx->has_data) l0l2::fail(L0L2_E_NODATA, "l0l2_set_data has not been called");
}

void check_K(int K) {
    if (K < 0) l0l2::fail(L0L2_E_INVALID, "K must be >= 0");
}

}  // namespace

extern "C" {

int l0l2_create(int device, void *hip_stream, l0l2_ctx **out) {
    if (!out) return L0L2_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        g_create_err = "no HIP device available";
        return L0L2_E_DEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_err = "device index out of range";
        return L0L2_E_INVALID;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_create_err = "hipSetDevice failed";
        return L0L2_E_DEVICE;
    }
    l0l2_ctx *c = new (std::nothrow) l0l2_ctx();
    if (!c) return L0L2_E_OOM;
    c->device = device;
    c->user_stream = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
        g_create_err = "stream or event creation failed";
        if (c->stream) (void)hipStreamDestroy(c->stream);
        if (c->ev_in) (void)hipEventDestroy(c->ev_in);
        delete c;
        return L0L2_E_DEVICE;
    }
    // address of the allocation-free entry point's scratch on this device, looked
    // up here (once per device) so that the entry point itself allocates nothing
    try {
        (void)l0l2::noalloc_scratch(device);
    } catch (const l0l2::Error &e) {
        c->noalloc_err = e.msg;
    }
    *out = c;
    return L0L2_OK;
}

void l0l2_destroy(l0l2_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    l0l2::drop_graphs(ctx);
    if (ctx->ws.host_counter) (void)hipHostFree(ctx->ws.host_counter);
    l0l2::prof_release(ctx->prof);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
    (void)hipEventDestroy(ctx->ev_in);
    (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ev_group) (void)hipEventDestroy(ctx->ev_group);
    delete ctx;
}

const char *l0l2_last_error(const l0l2_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int l0l2_state_bytes(const l0l2_ctx *ctx) {
    if (!ctx) return L0L2_E_INVALID;
    return (int)l0l2::state_bytes(ctx->inst.prec);
}

int l0l2_set_data(l0l2_ctx *ctx, const double *X, const double *y, int64_t n, int64_t p, double lambda0,
                  double lambda2, double M, double rho, int x_precision, int ptrs_on_device) {
    return guarded(ctx, [&] {
        if (!X || !y) l0l2::fail(L0L2_E_INVALID, "X and y must be non-null");
        if (n < 1 || p < 1) l0l2::fail(L0L2_E_INVALID, "need n >= 1 and p >= 1");
        if (!(std::isfinite(lambda0) && lambda0 >= 0)) l0l2::fail(L0L2_E_INVALID, "lambda0 must be finite and >= 0");
        if (!(std::isfinite(lambda2) && lambda2 > 0)) l0l2::fail(L0L2_E_INVALID, "lambda2 must be finite and > 0");
        if (!(M > 0) || std::isnan(M)) l0l2::fail(L0L2_E_INVALID, "M must be > 0 (INFINITY allowed)");
        if (!(std::isfinite(rho) && rho > 0)) l0l2::fail(L0L2_E_INVALID, "rho must be finite and > 0");
        if (x_precision != L0L2_FP64 && x_precision != L0L2_FP32 && x_precision != L0L2_BF16 &&
            x_precision != L0L2_FP8)
            l0l2::fail(L0L2_E_INVALID, "unknown x_precision");
        if (!ptrs_on_device) {
            for (int64_t e = 0; e < n * p; ++e)
                if (!std::isfinite(X[e])) l0l2::fail(L0L2_E_INVALID, "X has a non-finite entry");
            for (int64_t e = 0; e < n; ++e)
                if (!std::isfinite(y[e])) l0l2::fail(L0L2_E_INVALID, "y has a non-finite entry");
        }
        l0l2::set_data(ctx, X, y, n, p, lambda0, lambda2, M, rho, x_precision, ptrs_on_device);
    });
}

int l0l2_admm_sweeps(l0l2_ctx *ctx, int K, const uint8_t *codes, void *beta, void *v, void *b_out, int sweeps) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (sweeps < 1) l0l2::fail(L0L2_E_INVALID, "sweeps must be >= 1");
        if (ctx->inst.prec == L0L2_FP8)
            l0l2::fail(L0L2_E_UNSUPPORTED, "FP8 storage runs anchored solves only (l0l2_solve_node_batch)");
        if (K == 0) return;
        if (!codes || !beta || !v) l0l2::fail(L0L2_E_INVALID, "null buffer");
        l0l2::load_batch(ctx, K, codes, beta, v, false);
        l0l2::run_sweeps(ctx, K, sweeps, true);
        l0l2::store_batch(ctx, K, beta, v, b_out);
    });
}

int l0l2_dual_bound(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *b, double *lb) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (K == 0) return;
        if (!codes || !b || !lb) l0l2::fail(L0L2_E_INVALID, "null buffer");
        // b goes into the sweep's b slot through the beta loader, then is moved.
        l0l2::load_batch(ctx, K, codes, b, b, false);
        auto &ws = ctx->ws;
        const int64_t Kp = l0l2::round_up(K, l0l2::kPadNodes);
        size_t sb = l0l2::state_bytes(ctx->inst.prec);
        HIPCHK(hipMemcpyAsync(ws.B.ptr, ws.beta.ptr, sb * Kp * ctx->inst.ldp, hipMemcpyDeviceToDevice, ctx->stream));
        l0l2::run_dual_bound(ctx, K, nullptr);
        HIPCHK(hipMemcpyAsync(lb, ws.lb.ptr, sizeof(double) * K, hipMemcpyDeviceToDevice, ctx->stream));
    });
}

int l0l2_solve_node_batch(l0l2_ctx *ctx, int K, const uint8_t *codes, void *beta, void *v,
                          const l0l2_admm_opts *opts, double *lb, double *primal, int32_t *iters, int32_t *status) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (!opts) l0l2::fail(L0L2_E_INVALID, "null options");
        if (opts->max_iter < 1 || opts->check_every < 1 || !(opts->tol_node >= 0))
            l0l2::fail(L0L2_E_INVALID, "need max_iter >= 1, check_every >= 1, tol_node >= 0");
        if (K == 0) return;
        if (!codes || !beta || !v || !lb || !primal || !iters || !status) l0l2::fail(L0L2_E_INVALID, "null buffer");
        l0l2::load_batch(ctx, K, codes, beta, v, false);
        l0l2::run_solve(ctx, K, *opts);
        l0l2::store_batch(ctx, K, beta, v, nullptr);
        auto &ws = ctx->ws;
        hipStream_t s = ctx->stream;
        HIPCHK(hipMemcpyAsync(lb, ws.lb.ptr, sizeof(double) * K, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(primal, ws.primal.ptr, sizeof(double) * K, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(iters, ws.iters.ptr, sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(status, ws.status.ptr, sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s));
    });
}

int l0l2_solve_node_queue(l0l2_ctx *ctx, int N, const uint8_t *codes, void *beta, void *v, int K,
                          const l0l2_admm_opts *opts, double *lb, double *primal, int32_t *iters, int32_t *status) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (N < 0 || K < 1) l0l2::fail(L0L2_E_INVALID, "need N >= 0 and K >= 1");
        if (!opts) l0l2::fail(L0L2_E_INVALID, "null options");
        if (opts->max_iter < 1 || opts->check_every < 1 || !(opts->tol_node >= 0))
            l0l2::fail(L0L2_E_INVALID, "need max_iter >= 1, check_every >= 1, tol_node >= 0");
        if (N == 0) return;
        if (!codes || !beta || !v || !lb || !primal || !iters || !status) l0l2::fail(L0L2_E_INVALID, "null buffer");
        const int Ks = (int)std::min<int64_t>(K, N);
        l0l2::ensure_workspace(ctx, Ks);
        l0l2::run_queue(ctx, N, codes, beta, v, Ks, *opts, lb, primal, iters, status);
    });
}

int l0l2_batch_stats(l0l2_ctx *ctx, int64_t *blocks, int64_t *sparse_blocks, int64_t *node_blocks) {
    if (!ctx) return L0L2_E_INVALID;
    if (blocks) *blocks = ctx->ws.stat_blocks;
    if (sparse_blocks) *sparse_blocks = ctx->ws.stat_sparse;
    if (node_blocks) *node_blocks = ctx->ws.stat_node_blocks;
    return L0L2_OK;
}

int l0l2_round_branch(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *beta, uint8_t *support,
                      int32_t *support_size, int32_t *branch_j, int32_t *z_up) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (K == 0) return;
        if (!codes || !beta || !support || !support_size || !branch_j || !z_up)
            l0l2::fail(L0L2_E_INVALID, "null buffer");
        // free-coordinate counts go to a context buffer (grown, never freed in the call)
        if (ctx->ws.nfree.bytes < sizeof(int32_t) * (size_t)K) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            ctx->ws.nfree.ensure(sizeof(int32_t) * (size_t)K);
        }
        l0l2::run_round_branch(ctx, K, codes, ctx->inst.p, beta, ctx->inst.p, support, support_size, branch_j, z_up,
                               ctx->ws.nfree.as<int32_t>());
    });
}

int l0l2_refine_incumbent(l0l2_ctx *ctx, int K, const uint8_t *support, const void *beta_start, double *beta_out,
                          const l0l2_fista_opts *opts, double *obj, int32_t *iters) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (!opts || opts->max_iter < 1 || !(opts->tol >= 0)) l0l2::fail(L0L2_E_INVALID, "bad FISTA options");
        if (K == 0) return;
        if (!support || !beta_start || !beta_out || !obj) l0l2::fail(L0L2_E_INVALID, "null buffer");
        const int64_t p = ctx->inst.p;
        l0l2::state_to_f64(ctx, K, beta_start, p, beta_out, p);
        l0l2::run_fista(ctx, K, support, p, beta_out, p, *opts, obj, iters);
    });
}

int l0l2_refine_incumbent_noalloc(l0l2_ctx *ctx, int K, const uint8_t *support, const void *beta_start,
                                  double *beta_out, const l0l2_fista_opts *opts, double *obj, int32_t *iters) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_K(K);
        if (!opts || opts->max_iter < 1 || !(opts->tol >= 0)) l0l2::fail(L0L2_E_INVALID, "bad FISTA options");
        if (K == 0) return;
        if (!support || !beta_start || !beta_out || !obj) l0l2::fail(L0L2_E_INVALID, "null buffer");
        const size_t need = sizeof(double) * (size_t)K * (size_t)ctx->inst.np;
        if (need > l0l2::kNoAllocScratchBytes)
            l0l2::fail(L0L2_E_INVALID, "K x padded n x 8 = " + std::to_string(need) + " bytes exceeds the " +
                                           std::to_string(l0l2::kNoAllocScratchBytes) +
                                           "-byte device scratch of the allocation-free refinement");
        if (!ctx->noalloc_err.empty()) l0l2::fail(L0L2_E_DEVICE, ctx->noalloc_err);
        // looked up at l0l2_create; this only reads the stored address
        double *scr = static_cast<double *>(l0l2::noalloc_scratch(ctx->device));
        const int64_t p = ctx->inst.p;
        l0l2::state_to_f64(ctx, K, beta_start, p, beta_out, p);
        l0l2::run_fista(ctx, K, support, p, beta_out, p, *opts, obj, iters, scr);
    });
}

int l0l2_exact_objective(l0l2_ctx *ctx, const uint8_t *support, double *beta_out, double *obj) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (!support || !beta_out || !obj) l0l2::fail(L0L2_E_INVALID, "null buffer");
        *obj = l0l2::run_exact_objective(ctx, support, beta_out);
    });
}

int l0l2_matching_pursuit(l0l2_ctx *ctx, int max_moves, uint8_t *support, double *beta, double *obj,
                          int32_t *moves, int32_t *n_moves) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (max_moves < 1) l0l2::fail(L0L2_E_INVALID, "max_moves must be >= 1");
        if (!support || !beta || !obj || !n_moves) l0l2::fail(L0L2_E_INVALID, "null buffer");
        l0l2::run_matching_pursuit(ctx, max_moves, support, beta, moves, n_moves, obj);
    });
}

int l0l2_bnb_solve(l0l2_ctx *ctx, const l0l2_bnb_opts *opts, l0l2_bnb_result *out) {
    if (out) std::memset(out, 0, sizeof(*out));
    return guarded(ctx, [&] {
        need_data(ctx);
        if (!opts || !out) l0l2::fail(L0L2_E_INVALID, "null argument");
        if (opts->K < 0 || opts->admm.max_iter < 1 || opts->admm.check_every < 1 || opts->max_iter_root < 1 ||
            opts->fista.max_iter < 1 || !(opts->eps_prune >= 0) || !(opts->gap_tol >= 0) || opts->max_nodes < 1 ||
            (opts->policy != L0L2_BEST_FIRST && opts->policy != L0L2_DFS) || opts->root_heuristic < 0 ||
            opts->root_heuristic > 1 || opts->warm_root < 0 || opts->warm_root > 1)
            l0l2::fail(L0L2_E_INVALID, "bad branch-and-bound options");
        l0l2_bnb_opts o = *opts;
        if (o.K == 0) {
            // batch size by measurement, once per instance
            std::vector<double> rates;
            o.K = ctx->inst.tuned_K > 0 ? ctx->inst.tuned_K : l0l2::tune_batch_size(ctx, 1024, 0.9, rates);
        }
        l0l2::bnb_solve(ctx, o, out);
    });
}

void check_penalties(double lambda0, double lambda2, double M) {
    if (!(std::isfinite(lambda0) && lambda0 >= 0)) l0l2::fail(L0L2_E_INVALID, "lambda0 must be finite and >= 0");
    if (!(std::isfinite(lambda2) && lambda2 > 0)) l0l2::fail(L0L2_E_INVALID, "lambda2 must be finite and > 0");
    if (!(M > 0) || std::isnan(M)) l0l2::fail(L0L2_E_INVALID, "M must be > 0 (INFINITY allowed)");
}

int l0l2_set_penalties(l0l2_ctx *ctx, double lambda0, double lambda2, double M) {
    return guarded(ctx, [&] {
        need_data(ctx);
        check_penalties(lambda0, lambda2, M);
        l0l2::set_penalties(ctx, lambda0, lambda2, M);
    });
}

int l0l2_lambda0_max(l0l2_ctx *ctx, double *out) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (!out) l0l2::fail(L0L2_E_INVALID, "null argument");
        *out = l0l2::lambda0_max(ctx);
    });
}

int l0l2_bnb_path(l0l2_ctx *ctx, const l0l2_bnb_opts *opts, int m, const double *lambda0s,
                  l0l2_bnb_result *results) {
    if (results && m > 0) std::memset(results, 0, sizeof(*results) * (size_t)m);
    if (!ctx) return L0L2_E_INVALID;
    if (!opts || !lambda0s || !results || m < 1) {
        ctx->err = "need opts, m >= 1 lambda0 values and m results";
        return L0L2_E_INVALID;
    }
    const double l2 = ctx->inst.mp.l2, M = ctx->inst.mp.M;
    std::vector<uint8_t> prev;
    for (int i = 0; i < m; ++i) {
        int rc = l0l2_set_penalties(ctx, lambda0s[i], l2, M);
        if (rc != L0L2_OK) return rc;
        l0l2_bnb_opts o = *opts;
        if (i > 0) {
            o.warm_root = 1;
            if (!prev.empty()) o.init_support = prev.data();
        }
        rc = l0l2_bnb_solve(ctx, &o, &results[i]);
        if (rc != L0L2_OK) return rc;
        prev.assign((size_t)ctx->inst.p, 0);
        for (int64_t e = 0; e < results[i].support_len; ++e) prev[(size_t)results[i].support[e]] = 1;
    }
    return L0L2_OK;
}

int l0l2_tune_batch_size(l0l2_ctx *ctx, int k_max, double frac, int *k_out, double *rates, int *n_rates) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (!k_out) l0l2::fail(L0L2_E_INVALID, "null argument");
        if (k_max < 32 || k_max > 65536 || !(frac > 0.0 && frac <= 1.0))
            l0l2::fail(L0L2_E_INVALID, "need 32 <= k_max <= 65536 and 0 < frac <= 1");
        std::vector<double> r;
        *k_out = l0l2::tune_batch_size(ctx, k_max, frac, r);
        if (n_rates) *n_rates = (int)r.size();
        if (rates)
            for (size_t i = 0; i < r.size(); ++i) rates[i] = r[i];
    });
}

int l0l2_set_tiles(l0l2_ctx *ctx, int xw_shape, int xtu_shape) {
    return guarded(ctx, [&] {
        bool auto_ = xw_shape < 0 && xtu_shape < 0;
        if (!auto_ && (xw_shape < 0 || xw_shape > 17 || xtu_shape < 0 || xtu_shape > 11))
            l0l2::fail(L0L2_E_INVALID, "tile shapes are 0..17 for xw, 0..11 for xtu (or both -1)");
        // captured blocks hold the shapes they were captured with
        if (ctx->force_xw != (auto_ ? -1 : xw_shape) || ctx->force_xtu != (auto_ ? -1 : xtu_shape)) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            l0l2::drop_graphs(ctx);
        }
        ctx->force_xw = auto_ ? -1 : xw_shape;
        ctx->force_xtu = auto_ ? -1 : xtu_shape;
    });
}

int l0l2_set_bupdate_form(l0l2_ctx *ctx, int form) {
    return guarded(ctx, [&] {
        if (form < 0 || form > 2) l0l2::fail(L0L2_E_INVALID, "form is 0 (auto), 1 (folded operand) or 2 (Gram)");
        if (ctx->bform != form) {
            // captured blocks hold the form they were captured with
            HIPCHK(hipStreamSynchronize(ctx->stream));
            l0l2::drop_graphs(ctx);
        }
        ctx->bform = form;
    });
}

int l0l2_memory_stats(l0l2_ctx *ctx, size_t *in_use, size_t *peak, int reset_peak) {
    l0l2::MemCount &m = ctx ? ctx->mem : l0l2::global_mem();
    if (in_use) *in_use = m.in_use.load();
    if (peak) *peak = m.peak.load();
    if (reset_peak) m.peak.store(m.in_use.load());
    return L0L2_OK;
}

int l0l2_cancel(l0l2_ctx *ctx) {
    if (!ctx) return L0L2_E_INVALID;
    ctx->cancel.store(1);
    return L0L2_OK;
}

int l0l2_set_bf16_terms(l0l2_ctx *ctx, int terms) {
    return guarded(ctx, [&] {
        if (terms != 1 && terms != 3) l0l2::fail(L0L2_E_INVALID, "terms is 1 (single-term blocks) or 3 (split)");
        if (ctx->bf16_terms != terms) {
            // captured blocks hold the sweeps they were captured with
            HIPCHK(hipStreamSynchronize(ctx->stream));
            l0l2::drop_graphs(ctx);
        }
        ctx->bf16_terms = terms;
    });
}

int l0l2_set_bf16_tile_rows(l0l2_ctx *ctx, int rows) {
    return guarded(ctx, [&] {
        if (rows != 128 && rows != 256) l0l2::fail(L0L2_E_INVALID, "rows is 128 or 256");
        if (ctx->bf16_rows != rows) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            l0l2::drop_graphs(ctx);
        }
        ctx->bf16_rows = rows;
    });
}

int l0l2_bupdate_form(l0l2_ctx *ctx, int *form, double *ms_folded, double *ms_gram) {
    return guarded(ctx, [&] {
        need_data(ctx);
        if (!form) l0l2::fail(L0L2_E_INVALID, "null argument");
        double ms[2];
        *form = l0l2::bupdate_form(ctx, ms);
        if (ms_folded) *ms_folded = ms[0];
        if (ms_gram) *ms_gram = ms[1];
    });
}

int l0l2_profile_enable(l0l2_ctx *ctx, int enable) {
    return guarded(ctx, [&] {
        l0l2::prof_collect(ctx);
        ctx->prof.on = enable != 0;
        for (int i = 0; i < l0l2::kProfCount; ++i) {
            ctx->prof.total_ms[i] = 0.0;
            ctx->prof.count[i] = 0;
            ctx->prof.units[i] = 0;
        }
    });
}

int l0l2_profile_query(l0l2_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms, int64_t *units) {
    return guarded(ctx, [&] {
        if (!kernel || !launches || !total_ms) l0l2::fail(L0L2_E_INVALID, "null argument");
        l0l2::prof_collect(ctx);
        for (int i = 0; i < l0l2::kProfCount; ++i)
            if (std::strcmp(kernel, l0l2::kProfNames[i]) == 0) {
                *launches = ctx->prof.count[i];
                *total_ms = ctx->prof.total_ms[i];
                if (units) *units = ctx->prof.units[i];
                return;
            }
        l0l2::fail(L0L2_E_INVALID, std::string("unknown kernel name ") + kernel);
    });
}

void l0l2_result_free(l0l2_bnb_result *res) {
    if (!res) return;
    std::free(res->support);
    std::free(res->beta);
    res->support = nullptr;
    res->beta = nullptr;
}

}  // extern "C"
