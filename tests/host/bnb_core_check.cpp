// CPU check of the branch-and-bound host logic (paper_2602_04551_amd/csrc/bnb_core.hpp):
// the library's frontier / selection / decision code driven with the FP64 CPU
// oracle as the node solver.  Reads an instance file, prints the trace and the
// result as JSON lines.  Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../../oracle/l0l2_oracle.h"
#include "../../paper_2602_04551_amd/csrc/bnb_core.hpp"

int main(int argc, char **argv) {
    if (argc < 6) {
        std::fprintf(stderr, "usage: %s instance.bin K policy(0 best,1 dfs) tol max_iter_root\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n, p;
    double l0, l2, M;
    if (std::fread(&n, 8, 1, f) != 1 || std::fread(&p, 8, 1, f) != 1 || std::fread(&l0, 8, 1, f) != 1 ||
        std::fread(&l2, 8, 1, f) != 1 || std::fread(&M, 8, 1, f) != 1) return 2;
    std::vector<double> X((size_t)(n * p)), y((size_t)n);
    if (std::fread(X.data(), 8, X.size(), f) != X.size() || std::fread(y.data(), 8, y.size(), f) != y.size()) return 2;
    std::fclose(f);
    const int K = std::atoi(argv[2]);
    const int policy = std::atoi(argv[3]);
    const double tol = std::atof(argv[4]);
    const int max_iter_root = std::atoi(argv[5]);
    const int max_iter = 5000, check_every = 10;
    orc_inst *in = orc_create(X.data(), y.data(), n, p, l0, l2, M, 1.0);
    if (!in) return 3;

    std::vector<l0l2_trace_rec> trace(1 << 20);
    l0l2_bnb_opts o{};
    o.K = K;
    o.policy = policy;
    o.eps_prune = 2.0 * tol;
    o.gap_tol = 0.0;
    o.max_nodes = 1 << 30;
    o.max_iter_root = max_iter_root;
    o.admm = {tol, max_iter, check_every};
    o.fista = {1e-12, 1000};
    o.trace = trace.data();
    o.trace_cap = (int64_t)trace.size();
    l0l2::BnbCore core(o);

    std::map<int64_t, std::pair<std::vector<double>, std::vector<double>>> slots;
    std::vector<l0l2::OpenNode> batch;
    std::vector<int32_t> fx;
    std::vector<std::pair<int, int64_t>> saves;
    std::vector<uint8_t> inc_mask((size_t)p, 0), mask((size_t)p);
    while (!core.frontier_empty()) {
        core.select(K, batch);
        const int B = (int)batch.size();
        if (B == 0) continue;
        std::vector<std::vector<double>> fb(B), fv(B);
        std::vector<std::vector<uint8_t>> codes(B), sup(B);
        std::vector<l0l2::NodeOutcome> res(B);
        for (int k = 0; k < B; ++k) {
            codes[k].assign((size_t)p, 0);
            fx.clear();
            core.fixings(batch[k].id, fx);
            for (int32_t v : fx) codes[k][(size_t)(v >> 2)] = (uint8_t)(v & 3);
            if (batch[k].slot >= 0) {
                fb[k] = slots[batch[k].slot].first;
                fv[k] = slots[batch[k].slot].second;
            } else {
                fb[k].assign((size_t)p, 0.0);
                fv[k].assign((size_t)p, 0.0);
            }
        }
        core.gathered(batch);
        for (int k = 0; k < B; ++k) {
            std::vector<double> b((size_t)p, 0.0), bf;
            double lb, pr;
            int it;
            int st = orc_node_admm(in, codes[k].data(), fb[k].data(), fv[k].data(), b.data(), tol,
                                   batch[k].id == 0 ? max_iter_root : max_iter, check_every, &lb, &pr, &it);
            sup[k].assign((size_t)p, 0);
            int ss = orc_support(in, codes[k].data(), fb[k].data(), sup[k].data());
            bf = fb[k];
            int fit;
            double ub = orc_fista(in, sup[k].data(), bf.data(), 1e-12, 1000, &fit);
            int j = orc_branch(in, codes[k].data(), fb[k].data());
            int zup = j >= 0 ? orc_z(fb[k][(size_t)j], ORC_FREE, l0, l2, M) >= 0.5 : 0;
            res[k] = l0l2::NodeOutcome{lb, pr, it, st, ub, ss, j, zup};
        }
        int best_k;
        core.process(batch, res.data(), saves, best_k);
        if (best_k >= 0) inc_mask = sup[best_k];
        for (auto &sv : saves) slots[sv.second] = {fb[sv.first], fv[sv.first]};
    }
    std::vector<double> bex((size_t)p);
    double cert = orc_exact_objective(in, inc_mask.data(), bex.data());
    for (int64_t t = 0; t < core.trace_len() && t < (int64_t)trace.size(); ++t) {
        const l0l2_trace_rec &r = trace[(size_t)t];
        std::printf("{\"id\":%lld,\"parent\":%lld,\"depth\":%d,\"branch_j\":%d,\"decision\":%d,\"iters\":%d,"
                    "\"support_size\":%d,\"lb\":%.17g}\n",
                    (long long)r.id, (long long)r.parent, r.depth, r.branch_j, r.decision, r.iters, r.support_size,
                    r.lb);
    }
    std::printf("{\"result\":1,\"ub\":%.17g,\"certified\":%.17g,\"solved\":%lld,\"pruned\":%lld,\"slots_in_use\":%lld,"
                "\"support\":[",
                core.ub(), cert, (long long)core.solved(), (long long)core.pruned(), (long long)core.slots_in_use());
    bool first = true;
    for (int64_t j = 0; j < p; ++j)
        if (inc_mask[(size_t)j]) {
            std::printf("%s%lld", first ? "" : ",", (long long)j);
            first = false;
        }
    std::printf("]}\n");
    orc_free(in);
    return 0;
}
