// Serving: branch and bound for many independent instances on one device.
//
// Requests (X, y, lambda0, lambda2, M, rho, precision) arrive at any time.  A
// request is admitted, in arrival order, as soon as a worker slot is free and
// its estimated device footprint fits in what the HBM budget has left; it then
// runs its branch and bound on its own context and HIP stream (default
// priority), and its footprint returns to the budget when it finishes.  The
// blocks of ADMM sweeps of all admitted instances go through one executor
// (admm.hip), which runs every block waiting when it becomes free in shared
// launches: the node solves of several instances are batched into one grid
// per contraction (continuous batching across instances; instances join and
// leave between blocks).  With batching off, each instance replays its own
// blocks on its stream and the device overlaps the streams.  Server contexts take their tile shapes from a
// size rule instead of timing them (timings taken while other instances load
// the device would vary, and with them the summation order), so each
// instance's computation is the same sequence of kernels whether it runs alone
// or beside others.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "serve_core.hpp"

namespace l0l2 {

size_t footprint_bytes(int64_t n, int64_t p, int prec, int K) {
    // padded extents plus the largest leading-dimension gap (64 bytes of BF16)
    const double np = (double)ld_pad(round_up(n, kPadRows), 2), pp = (double)ld_pad(round_up(p, kPadRows), 2);
    const double Kp = (double)round_up(std::max(K, 1), kPadNodes);
    const double sb = prec == L0L2_FP64 ? 8.0 : 4.0;
    double inst = 8.0 * np * pp + 32.0 * (np + pp);
    // the copies of Xh and X beside X64 (FP64 X64R everywhere; FP64 Xh and its
    // row-major copy for the anchors; the working-precision layouts)
    if (prec == L0L2_FP64) inst += 24.0 * np * pp;
    else if (prec == L0L2_FP32) inst += 32.0 * np * pp;
    else if (prec == L0L2_BF16) inst += 32.0 * np * pp;
    else inst += 26.0 * np * pp;
    double transient = 8.0 * np * np + 8.0 * (double)n * (double)p;
    double ws = 4.0 * sb * Kp * pp + sb * Kp * np + 24.0 * Kp * np + Kp * pp + 1.0 * Kp * pp / 4.0 + 128.0 * Kp;
    if (prec != L0L2_FP64) ws += 32.0 * Kp * pp + 8.0 * Kp * np;
    ws += 8.0 * Kp * np;                                   // refinement residuals
    ws += 8.0 * 8.0 * Kp * np;                             // partial products of the sliced contraction over p
    double bnb = 9.0 * Kp * (double)p + 2.0 * sb * pp * 16.0 * Kp;   // supports, starts, pool reserve
    // Gram form of the b-update where it is a candidate (FP32 and BF16 modes,
    // padded p at most twice padded n and at most 8192): G in FP64 and FP32 (and
    // a BF16 pair), and a second W buffer
    const int64_t np0 = round_up(n, kPadRows), pp0 = round_up(p, kPadRows);
    if ((prec == L0L2_FP32 || prec == L0L2_BF16) && pp0 <= 2 * np0 && pp0 <= 8192) {
        inst += (prec == L0L2_BF16 ? 16.0 : 12.0) * pp * pp;
        ws += 4.0 * Kp * pp;
    }
    // slots of the refinement of supports wider than 1024 coordinates
    if (p > 1024) {
        const double stride = 8.0 * (5.0 * (double)p + (double)((p + 1) / 2));
        ws += std::min({Kp, 64.0, std::max(1.0, std::floor(268435456.0 / stride))}) * stride + 4.0 * Kp;
    }
    // the terms above are the large buffers; a tenth more and 16 MiB cover the
    // small ones (gap-check partials, lists, refinement staging, captured graphs)
    return (size_t)(1.1 * (inst + std::max(transient, ws + bnb)) + 16.0 * 1048576.0);
}

}  // namespace l0l2

struct l0l2_server {
    struct Request {
        int64_t id;
        std::vector<double> X, y;
        int64_t n, p;
        double l0, l2, M, rho;
        int prec;
        size_t bytes;
        double t_submit = 0, t_admit = 0, t_done = 0;
        bool done = false, taken = false, cancel = false;
        l0l2_ctx *ctx = nullptr;   // while running (guarded by mu)
        size_t peak = 0;           // device bytes its context held at most
        int rc = L0L2_OK;
        std::string err;
        l0l2_bnb_result res{};
    };

    int device = 0;
    l0l2::GroupExec *exec = nullptr;  // shared executor of the admitted instances' blocks
    std::atomic<int> batching{1};     // attach newly admitted instances to exec
    std::unique_ptr<l0l2::Admission<Request>> adm;   // guarded by mu
    int max_concurrent = 1;
    l0l2_bnb_opts opts{};
    std::string err;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int64_t, std::shared_ptr<Request>> all;
    std::vector<std::thread> workers;
    int64_t next_id = 1;
    bool stopping = false;
    int waiters = 0;                  // threads inside l0l2_server_wait
    std::condition_variable cv_waiters;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // Next admissible request (serve_core.hpp: arrival order, HBM budget).
    std::shared_ptr<Request> admit_locked() {
        auto r = adm->admit();
        if (r) r->t_admit = now();
        return r;
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t stream = nullptr;
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
        for (;;) {
            std::shared_ptr<Request> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || (r = admit_locked()) != nullptr; });
                if (!r) break;
            }
            run(*r, stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                adm->finish(*r);
                r->t_done = now();
                r->done = true;
                r->X.clear();
                r->X.shrink_to_fit();
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (stream) (void)hipStreamDestroy(stream);
    }

    void run(Request &r, hipStream_t stream) {
        l0l2_ctx *ctx = nullptr;
        int rc = l0l2_create(device, stream, &ctx);
        if (rc == L0L2_OK) {
            ctx->tune = false;   // rule-based tile shapes: the same kernels alone and in the mix
            std::lock_guard<std::mutex> lk(mu);
            r.ctx = ctx;
            if (r.cancel) l0l2_cancel(ctx);
        }
        if (rc == L0L2_OK)
            rc = l0l2_set_data(ctx, r.X.data(), r.y.data(), r.n, r.p, r.l0, r.l2, r.M, r.rho, r.prec, 0);
        // attached once its precompute is done (the executor waits briefly for
        // every attached context); FP8 sweeps have no grouped kernels: those
        // instances keep their own streams rather than queue behind it
        if (rc == L0L2_OK && batching.load() && r.prec != L0L2_FP8) {
            ctx->group = exec;
            l0l2::group_exec_attach(exec, 1);
        }
        if (rc == L0L2_OK) rc = l0l2_bnb_solve(ctx, &opts, &r.res);
        r.rc = rc;
        if (rc != L0L2_OK) r.err = ctx ? l0l2_last_error(ctx) : l0l2_last_error(nullptr);
        if (ctx) {
            if (ctx->group) l0l2::group_exec_attach(ctx->group, -1);
            (void)l0l2_memory_stats(ctx, nullptr, &r.peak, 0);
            {
                std::lock_guard<std::mutex> lk(mu);
                r.ctx = nullptr;
            }
            l0l2_destroy(ctx);
        }
    }
};

extern "C" {

size_t l0l2_footprint_bytes(int64_t n, int64_t p, int precision, int K) {
    return l0l2::footprint_bytes(n, p, precision, K);
}

int l0l2_server_create(int device, size_t hbm_budget_bytes, int max_concurrent, const l0l2_bnb_opts *opts,
                       l0l2_server **out) {
    if (!out || !opts || max_concurrent < 1 || opts->K < 1) return L0L2_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return L0L2_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return L0L2_E_DEVICE;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return L0L2_E_DEVICE;
    l0l2_server *s = new (std::nothrow) l0l2_server();
    if (!s) return L0L2_E_OOM;
    s->device = device;
    s->adm.reset(new (std::nothrow) l0l2::Admission<l0l2_server::Request>(
        hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)freeb), max_concurrent));
    if (!s->adm) {
        delete s;
        return L0L2_E_OOM;
    }
    try {
        s->exec = l0l2::group_exec_create(device);
    } catch (...) {
        delete s;
        return L0L2_E_DEVICE;
    }
    s->max_concurrent = max_concurrent;
    s->opts = *opts;
    s->opts.trace = nullptr;
    s->opts.trace_cap = 0;
    for (int i = 0; i < max_concurrent; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return L0L2_OK;
}

int l0l2_server_submit(l0l2_server *s, const double *X, const double *y, int64_t n, int64_t p, double lambda0,
                       double lambda2, double M, double rho, int precision, int64_t *req_id) {
    if (!s || !X || !y || !req_id || n < 1 || p < 1) return L0L2_E_INVALID;
    if (precision != L0L2_FP64 && precision != L0L2_FP32 && precision != L0L2_BF16 && precision != L0L2_FP8)
        return L0L2_E_INVALID;
    auto r = std::make_shared<l0l2_server::Request>();
    try {
        r->X.assign(X, X + n * p);
        r->y.assign(y, y + n);
    } catch (...) {
        return L0L2_E_OOM;
    }
    r->n = n; r->p = p; r->l0 = lambda0; r->l2 = lambda2; r->M = M; r->rho = rho; r->prec = precision;
    r->bytes = l0l2::footprint_bytes(n, p, precision, s->opts.K);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return L0L2_E_INVALID;
        if (!s->adm->fits_at_all(*r)) {
            s->err = "request footprint exceeds the server's HBM budget";
            return L0L2_E_OOM;
        }
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->adm->push(r);
        s->all[r->id] = r;
        *req_id = r->id;
    }
    s->cv_work.notify_all();
    return L0L2_OK;
}

int l0l2_server_wait(l0l2_server *s, int64_t req_id, double timeout_s, l0l2_bnb_result *out,
                     l0l2_request_stats *stats) {
    if (!s || !out) return L0L2_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end() || it->second->taken) return L0L2_E_INVALID;
    auto r = it->second;
    auto pred = [&] { return r->done; };
    // l0l2_server_destroy waits for the threads counted here before it frees s
    ++s->waiters;
    struct Leave {
        l0l2_server *s;
        ~Leave() {
            if (--s->waiters == 0) s->cv_waiters.notify_all();
        }
    } leave{s};
    if (timeout_s < 0) s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return L0L2_E_TIMEOUT;
    it = s->all.find(req_id);
    if (it == s->all.end() || it->second->taken) return L0L2_E_INVALID;
    *out = r->res;
    r->res.support = nullptr;
    r->res.beta = nullptr;
    r->taken = true;
    if (stats) {
        stats->submit_s = r->t_submit;
        stats->admit_s = r->t_admit;
        stats->done_s = r->t_done;
        stats->footprint_bytes = r->bytes;
        stats->peak_bytes = r->peak;
    }
    int rc = r->rc;
    if (rc != L0L2_OK) s->err = r->err;
    s->all.erase(it);
    return rc;
}

const char *l0l2_server_last_error(const l0l2_server *s) { return s ? s->err.c_str() : ""; }

int l0l2_server_cancel(l0l2_server *s, int64_t req_id) {
    if (!s) return L0L2_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(req_id);
        if (it == s->all.end() || it->second->taken) return L0L2_E_INVALID;
        auto r = it->second;
        if (r->done) return L0L2_OK;
        r->cancel = true;
        if (s->adm->remove(r)) {
            // not admitted yet: finished here
            r->done = true;
            r->rc = L0L2_E_CANCELLED;
            r->err = "cancelled before admission";
            r->t_done = s->now();
        } else if (r->ctx) {
            l0l2_cancel(r->ctx);
        }
    }
    s->cv_done.notify_all();
    return L0L2_OK;
}

int l0l2_server_destroy(l0l2_server *s) {
    if (!s) return L0L2_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        // queued requests end as cancelled (their waiters return), running ones
        // are asked to stop at their next batch
        s->adm->drain([](l0l2_server::Request &r) {
            r.done = true;
            r.rc = L0L2_E_CANCELLED;
            r.err = "server destroyed before admission";
        });
        for (auto &kv : s->all)
            if (kv.second->ctx) l0l2_cancel(kv.second->ctx);
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto &t : s->workers) t.join();
    {
        // threads still inside l0l2_server_wait leave before s is freed
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_waiters.wait(lk, [&] { return s->waiters == 0; });
    }
    for (auto &kv : s->all) l0l2_result_free(&kv.second->res);
    l0l2::group_exec_destroy(s->exec);
    delete s;
    return L0L2_OK;
}

int l0l2_server_set_batching(l0l2_server *s, int on) {
    if (!s || (on != 0 && on != 1)) return L0L2_E_INVALID;
    s->batching.store(on);
    return L0L2_OK;
}

int l0l2_server_batching_stats(l0l2_server *s, int64_t *rounds, int64_t *blocks, int64_t *launches,
                               int64_t *members) {
    if (!s) return L0L2_E_INVALID;
    const l0l2::GroupStats st = l0l2::group_exec_stats(s->exec);
    if (rounds) *rounds = st.rounds;
    if (blocks) *blocks = st.blocks;
    if (launches) *launches = st.launches;
    if (members) *members = st.members;
    return L0L2_OK;
}

}  // extern "C"
