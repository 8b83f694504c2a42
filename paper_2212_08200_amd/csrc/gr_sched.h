// Admission and batching policy of the query server (plain C++, no HIP, so
// that it can be unit-tested on the host with an injected clock).
//
// Queries wait in one FIFO.  When an executor slot is free, the policy forms
// a batch for the graph of the OLDEST waiting query (so no graph starves):
// up to max_batch of that graph's queries, in arrival order.  The batch
// launches when it is full, when its oldest query has waited max_wait_ns, or
// when draining; otherwise the slot waits until that deadline or the next
// arrival.  A batch is admitted only if the device memory it needs fits in
// the budget next to the batches already running; otherwise the slot waits
// for a running batch to finish.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <vector>

namespace gr {

struct SchedQuery {
    uint64_t ticket;
    int32_t graph;
    int32_t src;
    void *dst;
    int64_t t_submit_ns;
};

struct SchedBatch {
    int32_t graph = -1;
    std::vector<SchedQuery> queries;
    size_t bytes = 0;
};

class BatchPolicy {
   public:
    // footprint(graph): device bytes one batch on that graph needs.
    BatchPolicy(int max_batch, int64_t max_wait_ns, size_t budget, std::function<size_t(int32_t)> footprint)
        : max_batch_(max_batch), max_wait_ns_(max_wait_ns), budget_(budget), footprint_(std::move(footprint)) {}

    void push(const SchedQuery &q) { q_.push_back(q); }
    size_t pending() const { return q_.size(); }

    enum Decision { kLaunch = 1, kWaitUntil = 2, kWaitForEvent = 3 };

    // Called for a free slot at time now with in_flight bytes already admitted.
    // kLaunch: *out holds the batch (removed from the queue).  kWaitUntil:
    // retry at *wake_ns (or on an arrival).  kWaitForEvent: retry after an
    // arrival or a completion.
    Decision next(int64_t now_ns, size_t in_flight, bool draining, SchedBatch *out, int64_t *wake_ns) {
        if (q_.empty()) return kWaitForEvent;
        const SchedQuery &head = q_.front();
        const int32_t g = head.graph;
        std::vector<size_t> pick;
        for (size_t i = 0; i < q_.size() && (int)pick.size() < max_batch_; ++i)
            if (q_[i].graph == g) pick.push_back(i);
        const bool full = (int)pick.size() >= max_batch_;
        const bool aged = now_ns - head.t_submit_ns >= max_wait_ns_;
        if (!full && !aged && !draining) {
            *wake_ns = head.t_submit_ns + max_wait_ns_;
            return kWaitUntil;
        }
        const size_t bytes = footprint_(g);
        if (in_flight + bytes > budget_) return kWaitForEvent;
        out->graph = g;
        out->bytes = bytes;
        out->queries.clear();
        std::deque<SchedQuery> rest;
        size_t j = 0;
        for (size_t i = 0; i < q_.size(); ++i) {
            if (j < pick.size() && pick[j] == i) {
                out->queries.push_back(q_[i]);
                ++j;
            } else {
                rest.push_back(q_[i]);
            }
        }
        q_.swap(rest);
        return kLaunch;
    }

   private:
    int max_batch_;
    int64_t max_wait_ns_;
    size_t budget_;
    std::function<size_t(int32_t)> footprint_;
    std::deque<SchedQuery> q_;
};

}  // namespace gr
