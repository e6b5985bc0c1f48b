// CPU check of the server's admission logic (paper_2602_04551_amd/csrc/serve_core.hpp)
// driven the way the server drives it: worker threads admit under one mutex,
// run a request for a random while and finish it; a producer thread submits
// requests of random footprints with random gaps and cancels some while they
// wait.  Checks, at every admission, that the reserved footprint fits the
// budget (or the request runs alone) and the concurrency limit holds; at the
// end, that admissions followed arrival order, every request either ran or
// was cancelled, and nothing stays reserved.  Built with sanitizers by the
// tests.  Test infrastructure only.
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2602_04551_amd/csrc/serve_core.hpp"

struct Req {
    size_t bytes = 0;
    int id = 0;
    bool done = false, cancelled = false, admitted = false;
};

int main(int argc, char **argv) {
    const int n_req = argc > 1 ? std::atoi(argv[1]) : 300;
    const int workers = argc > 2 ? std::atoi(argv[2]) : 4;
    const size_t budget = 1000;
    l0l2::Admission<Req> adm(budget, workers);
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    int violations = 0, max_running = 0;
    std::vector<int> order;
    std::vector<std::shared_ptr<Req>> reqs;

    auto worker = [&](unsigned seed) {
        std::mt19937 rng(seed);
        for (;;) {
            std::shared_ptr<Req> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || (r = adm.admit()) != nullptr; });
                if (!r) break;
                r->admitted = true;
                order.push_back(r->id);
                if (adm.running() > workers) ++violations;
                if (adm.reserved() > budget && adm.running() > 1) ++violations;
                if (adm.running() > max_running) max_running = adm.running();
            }
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
            {
                std::lock_guard<std::mutex> lk(mu);
                adm.finish(*r);
                r->done = true;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    };
    std::vector<std::thread> ws;
    for (int i = 0; i < workers; ++i) ws.emplace_back(worker, 1000u + (unsigned)i);

    std::mt19937 rng(7);
    for (int i = 0; i < n_req; ++i) {
        auto r = std::make_shared<Req>();
        r->id = i;
        r->bytes = 1 + rng() % budget;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!adm.fits_at_all(*r)) ++violations;
            reqs.push_back(r);
            adm.push(r);
        }
        cv_work.notify_all();
        if (rng() % 5 == 0) {
            // cancel a random earlier request if it is still waiting
            std::lock_guard<std::mutex> lk(mu);
            auto &c = reqs[rng() % reqs.size()];
            if (!c->admitted && !c->cancelled && adm.remove(c)) c->cancelled = true;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
    }
    {
        std::unique_lock<std::mutex> lk(mu);
        cv_done.wait(lk, [&] {
            for (auto &r : reqs)
                if (!r->done && !r->cancelled) return false;
            return true;
        });
        stopping = true;
    }
    cv_work.notify_all();
    for (auto &t : ws) t.join();

    int ran = 0, cancelled = 0;
    for (auto &r : reqs) {
        if (r->done == r->cancelled) ++violations;   // exactly one of the two
        ran += r->done;
        cancelled += r->cancelled;
    }
    for (size_t i = 1; i < order.size(); ++i)
        if (order[i] <= order[i - 1]) ++violations;   // arrival order
    if (adm.reserved() != 0 || adm.running() != 0 || !adm.empty()) ++violations;
    std::printf("{\"ran\": %d, \"cancelled\": %d, \"max_running\": %d, \"violations\": %d}\n", ran, cancelled,
                max_running, violations);
    return violations == 0 ? 0 : 1;
}
