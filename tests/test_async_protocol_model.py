"""CPU model of the asynchronous loop's worklist protocol (the counters,
in-queue flags, list positions, spills and relists of the asynchronous
kernel), run under random interleavings of its shared-memory steps.

Each block is a generator that yields after every access to shared state, and
a seeded scheduler picks which block steps next, so the races the protocol
must survive (a vertex improved while it waits in the list, a consumer
reserving a position before its producer has written it, blocks finding the
list empty while others still expand) happen in many orders.  Pre-reads of a
distance may return any value the vertex held before (a stale cache line).
Checked: every phase ends (done == tail), no position is written twice or
past the capacity, the list and the in-queue flags are empty at the end, and
the distances equal the oracle's.  A consumer that reads dist[v] before
clearing v's in-queue flag (losing a decrease that lands in between) fails
these seeds."""
import random

import numpy as np
import pytest

import graphgen as gg
import oracle

EMPTY = -1
CHUNK = 4  # positions a block reserves at once (the kernel: up to 256)


class Shared:
    def __init__(self, n, src, cap):
        self.dist = [2**32 - 1] * n
        self.hist = [[2**32 - 1] for _ in range(n)]  # values each vertex held
        self.dist[src] = 0
        self.hist[src].append(0)
        self.inq = {src}
        self.spill = set()
        self.cap = cap
        self.list = [EMPTY] * cap
        self.list[0] = src
        self.head, self.tail, self.done = 0, 1, 0
        self.expansions = 0


def block(sh, adj, rng):
    mine = []
    while True:
        if not mine:
            d = sh.done
            yield
            t = sh.tail
            yield
            h = sh.head
            yield
            if d == t:
                return
            if h < t:
                k = min(CHUNK, t - h)
                base = sh.head
                sh.head += k
                yield
                mine = [p for p in range(base, base + k) if p < sh.cap]
        took = []
        for p in list(mine):
            x = sh.list[p]
            sh.list[p] = EMPTY
            yield
            if x != EMPTY:
                took.append(x)
                mine.remove(p)
        if not took:
            d = sh.done
            yield
            t = sh.tail
            yield
            if d == t:
                return
            continue
        items = []
        for v in took:
            assert v in sh.inq  # an entry carries its vertex's flag
            sh.inq.discard(v)
            yield
            items.append((v, sh.dist[v]))
            yield
        sh.expansions += len(items)
        pushes = []
        for v, du in items:
            for x, w in adj[v]:
                nd = min(du + w, 2**32 - 1)
                cur = rng.choice(sh.hist[x][-3:])  # possibly stale pre-read
                yield
                if nd < cur:
                    old = sh.dist[x]
                    if nd < old:
                        sh.dist[x] = nd
                        sh.hist[x].append(nd)
                    yield
                    if nd < old:
                        was = x in sh.inq
                        sh.inq.add(x)
                        yield
                        if not was:
                            pushes.append(x)
        spilled = 0
        if pushes:
            b = sh.tail
            sh.tail += len(pushes)
            yield
            for i, x in enumerate(pushes):
                pos = b + i
                if pos < sh.cap:
                    assert sh.list[pos] == EMPTY, "position written twice"
                    sh.list[pos] = x
                    yield
                else:
                    sh.spill.add(x)
                    spilled += 1
        sh.done += len(took) + spilled
        yield


def run_model(g, src, cap, nblocks, seed):
    adj = [[(int(g.col[e]), int(g.w[e])) for e in range(g.ro[v], g.ro[v + 1])] for v in range(g.n)]
    rng = random.Random(seed)
    sh = Shared(g.n, src, cap)
    phases = 0
    while True:
        phases += 1
        blocks = [block(sh, adj, rng) for _ in range(nblocks)]
        steps = 0
        while blocks:
            i = rng.randrange(len(blocks))
            try:
                next(blocks[i])
            except StopIteration:
                blocks.pop(i)
            steps += 1
            assert steps < 10**7, "no termination"
        assert sh.done == sh.tail
        if sh.tail <= cap:
            break
        # relist: spilled vertices restart the list, those past cap stay spilled
        sh.head = sh.tail = sh.done = 0
        for v in sorted(sh.spill):
            pos = sh.tail
            sh.tail += 1
            if pos < cap:
                sh.list[pos] = v
                sh.spill.discard(v)
        sh.done = max(0, sh.tail - cap)
        assert phases < 10**5
    assert all(x == EMPTY for x in sh.list) and not sh.inq and not sh.spill
    return np.array(sh.dist, dtype=np.uint32), phases, sh.expansions


CASES = [("grid6", lambda: gg.grid(6, wseed=3)),
         ("uniform40", lambda: gg.uniform(40, 160, gseed=5, wseed=6, wtype=gg.W_U32, wlo=0, whi=5)),
         ("rmat6", lambda: gg.rmat(6, 8, gseed=7, pseed=8, wseed=9)),
         ("road8", lambda: gg.grid(8, wseed=11, wtype=gg.W_U32, wlo=1, whi=1000, shortcuts=3, sseed=12))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("cap", [1, 5, 10**6])
def test_async_protocol_model(name, make, cap):
    g = make()
    src = int(gg.pick_sources(g, 13, 1)[0]) if g.m else 0
    want = oracle.dijkstra(g, src)
    for seed in range(24):
        got, phases, exp = run_model(g, src, cap, nblocks=1 + seed % 8, seed=seed)
        assert np.array_equal(got, want), (name, cap, seed)
        if cap == 1:
            assert phases == exp  # one expansion per phase
