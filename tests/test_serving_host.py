"""Host logic of the serving loop (no device): LRU key residency under a byte budget, admission by
ciphertext slots and key memory, batch formation, rejection, and a simulated run that checks the
scheduler's invariants on a random arrival trace."""
import collections
import random

import pytest

from paper_2205_11935_amd.serving import KeyCache, PsetConfig, Request, Scheduler, latency_stats, poisson_arrivals


class FakeKeys:
    def __init__(self, sizes):
        self.sizes = sizes
        self.live = {}
        self.log = []

    def size_of(self, c):
        return self.sizes[c]

    def load(self, c):
        h = ("keys", c, len(self.log))
        self.live[h] = c
        self.log.append(("load", c))
        return h, self.sizes[c]

    def unload(self, h):
        c = self.live.pop(h)
        self.log.append(("unload", c))


def test_keycache_lru_and_pins():
    fk = FakeKeys({1: 4, 2: 4, 3: 4, 4: 6, 5: 11})
    kc = KeyCache(10, fk.size_of, fk.load, fk.unload)
    assert kc.acquire(1) and kc.acquire(2)
    assert kc.used == 8 and kc.resident() == [1, 2]
    assert not kc.acquire(3)                       # both pinned: nothing can go
    kc.release(1)
    assert kc.acquire(3)                           # evicts 1, the only unpinned client
    assert kc.resident() == [2, 3] and kc.evictions == 1
    assert kc.acquire(2)                           # hit: 2 becomes most recent
    assert kc.resident() == [3, 2]
    kc.release(2), kc.release(2), kc.release(3)
    assert kc.acquire(4)                           # needs 6 of 10: evicts 3 (least recent), keeps 2
    assert kc.resident() == [2, 4]
    assert fk.log == [("load", 1), ("load", 2), ("unload", 1), ("load", 3), ("unload", 3), ("load", 4)]
    with pytest.raises(ValueError):
        kc.acquire(5)                              # larger than the whole budget
    with pytest.raises(RuntimeError):
        kc.release(3)                              # not pinned
    kc.release(4)
    kc.clear()
    assert not fk.live


def test_scheduler_admission_batches_and_rejection():
    fk = FakeKeys({0: 1, 1: 1, 2: 1})
    kc = KeyCache(100, fk.size_of, fk.load, fk.unload)
    s = Scheduler([PsetConfig("a", slots=3, max_batch=2, lanes=1)], kc, max_pending=5, mix_clients=False)
    reqs = [Request(i, client=[0, 1, 0, 0, 2, 1][i], pset="a") for i in range(6)]
    for i, r in enumerate(reqs[:5]):
        assert s.arrive(r, float(i))
    assert not s.arrive(reqs[5], 5.0) and reqs[5].status == "rejected" and s.rejected == 1
    got = s.admit(5.0)
    assert [r.rid for r in got] == [0, 1, 2]       # three slots, arrival order
    assert sorted(r.slot for r in got) == [0, 1, 2]
    b1 = s.next_batch("a", 6.0)
    assert [r.rid for r in b1] == [0, 2]           # client 0 has the oldest query; at most 2
    b2 = s.next_batch("a", 6.0)
    assert [r.rid for r in b2] == [1]
    assert s.next_batch("a", 6.0) == []
    assert s.admit(6.0) == []                      # no slot free
    s.finish(b1, 7.0)
    got = s.admit(7.0)
    assert [r.rid for r in got] == [3, 4]
    assert {r.slot for r in got} == {b1[0].slot, b1[1].slot}
    s.finish(b2, 8.0)
    for _ in range(2):
        s.finish(s.next_batch("a", 8.0), 9.0)
    assert s.idle()
    assert all(r.status == "done" for r in reqs[:5])
    st = latency_stats(reqs)
    assert st["completed"] == 5 and st["rejected"] == 1


def test_scheduler_mixed_batches_take_the_oldest_queries_grouped_by_client():
    fk = FakeKeys({0: 1, 1: 1, 2: 1})
    kc = KeyCache(100, fk.size_of, fk.load, fk.unload)
    s = Scheduler([PsetConfig("a", slots=8, max_batch=5, lanes=1)], kc)
    owners = [1, 0, 1, 2, 0, 0, 1]
    reqs = [Request(i, client=c, pset="a") for i, c in enumerate(owners)]
    for i, r in enumerate(reqs):
        s.arrive(r, float(i))
    assert len(s.admit(7.0)) == 7
    b1 = s.next_batch("a", 8.0)
    # the five oldest (0..4), client 1's run first (its oldest query is 0), then 0's, then 2's
    assert [r.rid for r in b1] == [0, 2, 1, 4, 3]
    assert [r.client for r in b1] == [1, 1, 0, 0, 2]
    b2 = s.next_batch("a", 8.0)
    assert [r.rid for r in b2] == [5, 6]
    assert s.next_batch("a", 8.0) == []
    s.finish(b1 + b2, 9.0)
    assert s.idle() and kc.used == 3 and all(kc._pins.get(c, 0) == 0 for c in range(3))


def test_scheduler_waits_for_keys_and_lets_others_pass():
    fk = FakeKeys({0: 6, 1: 6, 2: 2})
    kc = KeyCache(10, fk.size_of, fk.load, fk.unload)
    s = Scheduler([PsetConfig("a", slots=8, max_batch=8, lanes=1)], kc)
    rs = [Request(0, 0, "a"), Request(1, 1, "a"), Request(2, 2, "a")]
    for i, r in enumerate(rs):
        s.arrive(r, float(i))
    got = s.admit(3.0)
    assert [r.rid for r in got] == [0, 2]          # client 1's keys do not fit while 0 is pinned
    assert rs[1].status == "pending"
    s.finish(s.next_batch("a", 3.0), 4.0)          # client 0 done: its keys can go
    s.finish(s.next_batch("a", 4.0), 4.0)
    got = s.admit(5.0)
    assert [r.rid for r in got] == [1] and kc.evictions == 1


@pytest.mark.parametrize("mix", [False, True])
def test_simulated_trace_invariants(mix):
    """Discrete-event run: two parameter sets, eight clients, Poisson arrivals, batch time affine in
    the batch size; checks slots, key residency, batch composition (one client, or contiguous runs
    of the oldest queries) and that every query finishes once."""
    rnd = random.Random(5)
    sizes = {c: (3 if c < 4 else 7) for c in range(8)}
    fk = FakeKeys(sizes)
    kc = KeyCache(20, fk.size_of, fk.load, fk.unload)
    cfgs = [PsetConfig("mid", slots=16, max_batch=8, lanes=2), PsetConfig("large", slots=6, max_batch=4, lanes=2)]
    s = Scheduler(cfgs, kc, mix_clients=mix)
    arr = poisson_arrivals(400.0, 600, seed=3)
    reqs = []
    for i, t in enumerate(arr):
        pset = "mid" if rnd.random() < 0.8 else "large"
        client = rnd.randrange(0, 4) if pset == "mid" else rnd.randrange(4, 8)
        reqs.append(Request(i, client, pset, t_arrive=float(t)))
    lanes = {c.name: [None] * c.lanes for c in cfgs}      # (finish time, batch)
    cost = {"mid": (1e-3, 2e-4), "large": (3e-3, 8e-4)}
    now, nxt, done = 0.0, 0, 0
    occupied = collections.defaultdict(set)
    while done < len(reqs):
        events = [arr[nxt]] if nxt < len(reqs) else []
        events += [ln[0] for lns in lanes.values() for ln in lns if ln]
        now = max(now, min(events))
        while nxt < len(reqs) and arr[nxt] <= now:
            assert s.arrive(reqs[nxt], now)
            nxt += 1
        for name, lns in lanes.items():
            for i, ln in enumerate(lns):
                if ln and ln[0] <= now:
                    for r in ln[1]:
                        occupied[name].remove(r.slot)
                    s.finish(ln[1], now)
                    done += len(ln[1])
                    lns[i] = None
        for r in s.admit(now):
            assert r.slot not in occupied[r.pset]
            occupied[r.pset].add(r.slot)
            assert r.client in kc.resident()
        assert kc.used <= kc.budget
        for name, lns in lanes.items():
            for i, ln in enumerate(lns):
                if ln is None:
                    waiting = sorted((r.t_arrive, r.rid) for q in s.admitted[name].values() for r in q)
                    b = s.next_batch(name, now)
                    if b:
                        assert {r.pset for r in b} == {name}
                        clients = [r.client for r in b]
                        if mix:
                            assert sorted((r.t_arrive, r.rid) for r in b) == waiting[:len(b)]
                            runs = [c for i, c in enumerate(clients) if i == 0 or clients[i - 1] != c]
                            assert len(runs) == len(set(runs))          # each client one run
                        else:
                            assert len(set(clients)) == 1
                        assert set(clients) <= set(kc.resident())
                        a, per = cost[name]
                        lns[i] = (now + a + per * len(b), b)
    assert all(r.status == "done" for r in reqs)
    assert len({r.rid for r in reqs}) == len(reqs)
    st = latency_stats(reqs)
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    assert kc.evictions > 0                        # the budget (20) cannot hold all eight clients (40)
