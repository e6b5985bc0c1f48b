// Admission of serving requests, independent of any device: requests wait in
// arrival order and the head is admitted when fewer than max_concurrent run and
// its estimated footprint fits in what the HBM budget has left (or nothing runs,
// so that a request larger than the remaining budget but within the total is
// not starved); the head blocks later arrivals, so large instances are not
// overtaken.  Not thread-safe by itself: the server calls it under its mutex.
#pragma once

#include <algorithm>
#include <cstddef>
#include <deque>
#include <memory>

namespace l0l2 {

template <class R>   // R: a request with a `bytes` member (its footprint)
class Admission {
  public:
    Admission(size_t budget, int max_concurrent) : budget_(budget), max_(max_concurrent) {}

    size_t budget() const { return budget_; }
    size_t reserved() const { return reserved_; }
    int running() const { return running_; }
    bool empty() const { return pending_.empty(); }

    // A request whose footprint alone exceeds the budget can never run.
    bool fits_at_all(const R &r) const { return r.bytes <= budget_; }

    void push(std::shared_ptr<R> r) { pending_.push_back(std::move(r)); }

    // The next request to start (its footprint reserved), or null.
    std::shared_ptr<R> admit() {
        if (pending_.empty() || running_ >= max_) return nullptr;
        const std::shared_ptr<R> &h = pending_.front();
        if (running_ > 0 && reserved_ + h->bytes > budget_) return nullptr;
        std::shared_ptr<R> r = h;
        pending_.pop_front();
        reserved_ += r->bytes;
        ++running_;
        return r;
    }

    // A started request has ended: its footprint returns to the budget.
    void finish(const R &r) {
        reserved_ -= r.bytes;
        --running_;
    }

    // Take a request out of the queue before admission; false if it is not queued.
    bool remove(const std::shared_ptr<R> &r) {
        auto q = std::find(pending_.begin(), pending_.end(), r);
        if (q == pending_.end()) return false;
        pending_.erase(q);
        return true;
    }

    // Empty the queue, calling f on each request still waiting.
    template <class F>
    void drain(F &&f) {
        for (auto &r : pending_) f(*r);
        pending_.clear();
    }

  private:
    std::deque<std::shared_ptr<R>> pending_;
    size_t budget_, reserved_ = 0;
    int max_, running_ = 0;
};

}  // namespace l0l2
