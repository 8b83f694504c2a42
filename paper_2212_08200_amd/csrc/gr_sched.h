// Admission policy of the query server (plain C++, no HIP, so that it can be
// unit-tested on the host with injected sizes).
//
// The server runs continuous batching: each executor keeps a multi-query
// session whose rounds advance every live query together, and new queries
// join it between chunks of rounds as slots and memory free up.  Queries wait
// in one FIFO; an executor with free slots admits queries from the head, in
// arrival order, while each one fits:
//   - a free slot of the session;
//   - the device-memory budget, next to the workspace of every query already
//     admitted by any executor;
//   - the session's queue capacity (the sum of the vertex counts of its live
//     queries) and the int32 arc range of one round (the sum of their arc
//     counts).
// The head is never overtaken by a query that needs a slot, so no query
// starves: when the head does not fit, admission stops until a query
// completes.  Queries on graphs that run outside the session (each one a
// workgroup of its own, with no slot and no workspace) are taken out of the
// FIFO in arrival order wherever they stand: they take nothing the head
// waits for.
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
    bool direct = false;  // its graph runs outside the session (no slot, no workspace)
};

// Sizes of a query on a graph.
struct QuerySize {
    size_t bytes;  // device workspace while it is live
    int64_t n;     // vertices (its share of the session's queue)
    int64_t m;     // arcs (bound on its share of one round's arcs)
};

// What an executor has left when it asks for admissions.
struct SessionRoom {
    int free_slots;
    int64_t free_queue;  // queue entries not reserved by live queries
    int64_t free_arcs;   // arcs of one round not reserved by live queries
};

class SlotPolicy {
   public:
    SlotPolicy(size_t budget, std::function<QuerySize(int32_t)> size) : budget_(budget), size_(std::move(size)) {}

    void push(const SchedQuery &q) {
        q_.push_back(q);
        ndirect_ += q.direct ? 1 : 0;
    }
    size_t pending() const { return q_.size(); }
    const SchedQuery *head() const { return q_.empty() ? nullptr : &q_.front(); }

    // Takes queries from the head while they fit (see above); in_flight is the
    // workspace already admitted, and grows by what is admitted here.
    std::vector<SchedQuery> admit(SessionRoom room, size_t *in_flight) {
        std::vector<SchedQuery> out;
        while (!q_.empty() && room.free_slots > 0) {
            const QuerySize z = size_(q_.front().graph);
            if (*in_flight + z.bytes > budget_ || z.n > room.free_queue || z.m > room.free_arcs) break;
            out.push_back(q_.front());
            ndirect_ -= q_.front().direct ? 1 : 0;
            q_.pop_front();
            *in_flight += z.bytes;
            room.free_slots -= 1;
            room.free_queue -= z.n;
            room.free_arcs -= z.m;
        }
        return out;
    }

    // Takes up to max direct queries (their graph runs outside the session),
    // in arrival order; they hold no slot and no budget.
    std::vector<SchedQuery> take_direct(size_t max) {
        std::vector<SchedQuery> out;
        for (auto it = q_.begin(); it != q_.end() && ndirect_ > 0 && out.size() < max;) {
            if (it->direct) {
                out.push_back(*it);
                it = q_.erase(it);
                --ndirect_;
            } else {
                ++it;
            }
        }
        return out;
    }

    // Whether a direct query is waiting.
    bool has_direct() const { return ndirect_ > 0; }

    // Empties the queue (the executor failed): every waiting query.
    std::vector<SchedQuery> take_all() {
        std::vector<SchedQuery> out(q_.begin(), q_.end());
        q_.clear();
        ndirect_ = 0;
        return out;
    }

   private:
    size_t budget_;
    std::function<QuerySize(int32_t)> size_;
    std::deque<SchedQuery> q_;
    size_t ndirect_ = 0;  // direct queries in q_
};

}  // namespace gr
