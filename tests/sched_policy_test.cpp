// Host unit test of the server's admission / batching policy (gr_sched.h):
// an injected clock and footprints, no GPU.  Exits non-zero on failure.
#include <cstdio>
#include <cstdlib>

#include "gr_sched.h"

#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);         \
            std::exit(1);                                            \
        }                                                            \
    } while (0)

using gr::BatchPolicy;
using gr::SchedBatch;
using gr::SchedQuery;

static SchedQuery q(uint64_t t, int32_t g, int64_t at) { return SchedQuery{t, g, (int32_t)t, nullptr, at}; }

int main() {
    const int64_t W = 1000;  // max wait
    // footprint: graph 0 = 100 bytes, graph 1 = 300 bytes
    BatchPolicy p(4, W, 400, [](int32_t g) { return g == 0 ? (size_t)100 : (size_t)300; });
    SchedBatch b;
    int64_t wake = -1;

    // empty queue: wait for an event
    CHECK(p.next(0, 0, false, &b, &wake) == BatchPolicy::kWaitForEvent);

    // a partial batch waits until the oldest query is max_wait old
    p.push(q(1, 0, 10));
    p.push(q(2, 1, 20));
    p.push(q(3, 0, 30));
    CHECK(p.next(100, 0, false, &b, &wake) == BatchPolicy::kWaitUntil);
    CHECK(wake == 10 + W);
    // ...then launches the oldest query's graph, keeping arrival order
    CHECK(p.next(10 + W, 0, false, &b, &wake) == BatchPolicy::kLaunch);
    CHECK(b.graph == 0 && b.queries.size() == 2 && b.queries[0].ticket == 1 && b.queries[1].ticket == 3);
    CHECK(b.bytes == 100);
    CHECK(p.pending() == 1);

    // graph 1 does not fit next to 200 bytes in flight (budget 400)
    CHECK(p.next(5000, 200, false, &b, &wake) == BatchPolicy::kWaitForEvent);
    CHECK(p.next(5000, 100, false, &b, &wake) == BatchPolicy::kLaunch);
    CHECK(b.graph == 1 && b.queries.size() == 1 && b.queries[0].ticket == 2);

    // a full batch launches at once, at most max_batch queries, FIFO
    for (uint64_t t = 10; t < 16; ++t) p.push(q(t, 0, 6000));
    CHECK(p.next(6000, 0, false, &b, &wake) == BatchPolicy::kLaunch);
    CHECK(b.queries.size() == 4 && b.queries[0].ticket == 10 && b.queries[3].ticket == 13);
    CHECK(p.pending() == 2);

    // draining ignores max_wait
    CHECK(p.next(6001, 0, true, &b, &wake) == BatchPolicy::kLaunch);
    CHECK(b.queries.size() == 2 && b.queries[0].ticket == 14);
    CHECK(p.pending() == 0);

    // no starvation: the oldest query's graph goes first even if another graph has more queries
    p.push(q(20, 1, 7000));
    for (uint64_t t = 21; t < 25; ++t) p.push(q(t, 0, 7001));
    CHECK(p.next(7000 + W, 0, false, &b, &wake) == BatchPolicy::kLaunch);
    CHECK(b.graph == 1 && b.queries[0].ticket == 20);
    CHECK(p.next(7001, 0, false, &b, &wake) == BatchPolicy::kLaunch);  // graph 0 now full (4)
    CHECK(b.graph == 0 && b.queries.size() == 4);

    std::printf("ok\n");
    return 0;
}
