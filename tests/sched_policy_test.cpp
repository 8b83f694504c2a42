// Host unit test of the server's admission policy (gr_sched.h): injected
// query sizes, no GPU.  Exits non-zero on failure.
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

using gr::QuerySize;
using gr::SchedQuery;
using gr::SessionRoom;
using gr::SlotPolicy;

static SchedQuery q(uint64_t t, int32_t g) { return SchedQuery{t, g, (int32_t)t, nullptr, (int64_t)t}; }

int main() {
    // graph 0: 100 bytes, 10 vertices, 40 arcs; graph 1: 300 bytes, 50 vertices, 200 arcs
    SlotPolicy p(400, [](int32_t g) { return g == 0 ? QuerySize{100, 10, 40} : QuerySize{300, 50, 200}; });
    size_t in_flight = 0;

    // empty queue: nothing admitted
    CHECK(p.admit(SessionRoom{4, 1000, 1000}, &in_flight).empty());

    // FIFO order, as many as fit: 0, 1 fit the budget (400); the next 0 does not
    p.push(q(1, 0));
    p.push(q(2, 1));
    p.push(q(3, 0));
    std::vector<SchedQuery> a = p.admit(SessionRoom{4, 1000, 1000}, &in_flight);
    CHECK(a.size() == 2 && a[0].ticket == 1 && a[1].ticket == 2);
    CHECK(in_flight == 400 && p.pending() == 1);

    // the head waits for memory; a completion (100 bytes back) lets it in
    CHECK(p.admit(SessionRoom{4, 1000, 1000}, &in_flight).empty());
    in_flight -= 100;
    a = p.admit(SessionRoom{4, 1000, 1000}, &in_flight);
    CHECK(a.size() == 1 && a[0].ticket == 3 && in_flight == 400);

    // slots bound admission
    in_flight = 0;
    for (uint64_t t = 10; t < 16; ++t) p.push(q(t, 0));
    a = p.admit(SessionRoom{2, 1000, 1000}, &in_flight);
    CHECK(a.size() == 2 && a[0].ticket == 10 && a[1].ticket == 11 && in_flight == 200);
    // queue capacity bounds admission (10 vertices each: 25 entries admit two)
    in_flight = 0;
    a = p.admit(SessionRoom{8, 25, 1000}, &in_flight);
    CHECK(a.size() == 2 && a[0].ticket == 12);
    // one round's arcs bound admission (40 arcs each: 79 admit one)
    in_flight = 0;
    a = p.admit(SessionRoom{8, 1000, 79}, &in_flight);
    CHECK(a.size() == 1 && a[0].ticket == 14);
    a = p.admit(SessionRoom{8, 1000, 1000}, &in_flight);
    CHECK(a.size() == 1 && a[0].ticket == 15 && p.pending() == 0);

    // no overtaking: a large head blocks smaller queries behind it
    in_flight = 200;
    p.push(q(20, 1));
    p.push(q(21, 0));
    CHECK(p.admit(SessionRoom{8, 1000, 1000}, &in_flight).empty());
    CHECK(p.head()->ticket == 20);
    in_flight = 0;
    a = p.admit(SessionRoom{8, 1000, 1000}, &in_flight);
    CHECK(a.size() == 2 && a[0].ticket == 20 && a[1].ticket == 21);

    // direct queries leave the FIFO wherever they stand, in arrival order, up
    // to the maximum, and charge nothing; the rest keep their order
    in_flight = 0;
    auto qd = [](uint64_t t, int32_t g, bool d) {
        SchedQuery x = q(t, g);
        x.direct = d;
        return x;
    };
    CHECK(!p.has_direct());
    p.push(qd(30, 1, false));
    p.push(qd(31, 0, true));
    p.push(qd(32, 0, false));
    p.push(qd(33, 0, true));
    p.push(qd(34, 0, true));
    CHECK(p.has_direct());
    a = p.take_direct(2);
    CHECK(a.size() == 2 && a[0].ticket == 31 && a[1].ticket == 33 && in_flight == 0);
    CHECK(p.pending() == 3 && p.head()->ticket == 30);
    a = p.take_direct(64);
    CHECK(a.size() == 1 && a[0].ticket == 34 && p.pending() == 2);
    CHECK(p.take_direct(64).empty() && !p.has_direct());
    a = p.admit(SessionRoom{8, 1000, 1000}, &in_flight);
    CHECK(a.size() == 2 && a[0].ticket == 30 && a[1].ticket == 32);
    // a direct query admitted into a session (from the head) is no longer counted
    in_flight = 0;
    p.push(qd(40, 0, true));
    a = p.admit(SessionRoom{8, 1000, 1000}, &in_flight);
    CHECK(a.size() == 1 && a[0].ticket == 40 && !p.has_direct());
    // and take_all forgets them too
    p.push(qd(41, 0, true));
    CHECK(p.take_all().size() == 1 && !p.has_direct());

    std::printf("ok\n");
    return 0;
}
