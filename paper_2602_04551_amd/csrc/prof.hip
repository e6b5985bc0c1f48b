// Opt-in per-kernel timing with HIP events recorded on the context stream
// around each instrumented launch.
#include <cstring>

#include "internal.hpp"

namespace l0l2 {

const char *const kProfNames[kProfCount] = {"gemm_xw.f32",  "admm_xtu.f32", "gemm_xw.f64",
                                             "admm_xtu.f64", "gemm_xw.bf16", "admm_xtu.bf16",
                                             "gap_check",    "round_branch", "fista",
                                             "anchor.f64",   "gemm_xw.fp8",  "admm_xtu.fp8"};

static hipEvent_t pool_event(Profiler &p) {
    if (p.next < p.pool.size()) return p.pool[p.next++];
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    p.pool.push_back(e);
    ++p.next;
    return e;
}

void prof_begin(l0l2_ctx *ctx, int id) {
    Profiler &p = ctx->prof;
    if (!p.on) return;
    hipEvent_t e = pool_event(p);
    HIPCHK(hipEventRecord(e, ctx->stream));
    p.open.push_back({id, e});
}

void prof_end(l0l2_ctx *ctx, int id, int64_t units) {
    Profiler &p = ctx->prof;
    if (!p.on) return;
    p.units[id] += units;
    hipEvent_t e = pool_event(p);
    HIPCHK(hipEventRecord(e, ctx->stream));
    for (size_t i = p.open.size(); i-- > 0;) {
        if (p.open[i].first == id) {
            p.pairs.push_back({id, {p.open[i].second, e}});
            p.open.erase(p.open.begin() + (long)i);
            return;
        }
    }
}

void prof_collect(l0l2_ctx *ctx) {
    Profiler &p = ctx->prof;
    if (p.pairs.empty()) return;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (auto &pr : p.pairs) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, pr.second.first, pr.second.second));
        p.total_ms[pr.first] += ms;
        p.count[pr.first] += 1;
    }
    p.pairs.clear();
    p.open.clear();
    p.next = 0;
}

void prof_release(Profiler &p) {
    for (hipEvent_t e : p.pool) (void)hipEventDestroy(e);
    p.pool.clear();
}

}  // namespace l0l2
