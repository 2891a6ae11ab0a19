"""Admission and continuous batching of the served form, without a GPU (a
fake executor that only records what it is given)."""
import threading
import time

from paper_2407_14801_amd.serve import Request, Server, device_bytes, percentiles, replay


class FakeExec:
    def __init__(self, delay=0.02):
        self.delay = delay
        self.batches = []
        self.mu = threading.Lock()
        self.active = 0
        self.max_active = 0

    def __call__(self, kind, batch):
        with self.mu:
            self.batches.append((kind, [r.id for r in batch]))
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        time.sleep(self.delay)
        with self.mu:
            self.active -= 1


def _reqs(specs):
    return [Request(id=i, kind=k, n=n, seed=i + 1) for i, (k, n) in enumerate(specs)]


def test_all_requests_done_each_once():
    ex = FakeExec(0.005)
    srv = Server(ex).start()
    reqs = _reqs([("u32" if i % 3 else "kv", 1000 + i) for i in range(60)])
    replay(srv, reqs, [0.001 * i for i in range(60)])
    srv.drain(60)
    ids = sorted(i for _, b in ex.batches for i in b)
    assert ids == list(range(60))
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert all(all(reqs[i].kind == k for i in b) for k, b in ex.batches)


def test_requests_arriving_during_a_batch_join_the_next():
    ex = FakeExec(0.2)
    srv = Server(ex).start()
    reqs = _reqs([("u32", 100)] * 6)
    srv.submit(reqs[0])                  # starts alone
    time.sleep(0.05)
    for r in reqs[1:]:                   # arrive while batch 0 runs
        srv.submit(r)
    srv.drain(6)
    assert ex.batches[0] == ("u32", [0])
    assert ex.batches[1] == ("u32", [1, 2, 3, 4, 5])


def test_budget_bounds_admitted_bytes_and_keeps_arrival_order():
    ex = FakeExec(0.02)
    one = device_bytes(Request(id=0, kind="u32", n=1000, seed=1))
    srv = Server(ex, budget_bytes=3 * one).start()
    reqs = _reqs([("u32", 1000)] * 12)
    for r in reqs:
        srv.submit(r)
    srv.drain(12)
    assert srv.peak_used <= 3 * one
    order = [i for _, b in ex.batches for i in b]
    assert order == sorted(order)        # admitted and served in arrival order
    assert max(len(b) for _, b in ex.batches) <= 3


def test_kinds_overlap_and_plain_mode_serialises():
    ex = FakeExec(0.1)
    srv = Server(ex).start()
    reqs = _reqs([("u32", 10), ("kv", 10)])
    for r in reqs:
        srv.submit(r)
    srv.drain(2)
    assert ex.max_active == 2            # one worker per kind
    ex2 = FakeExec(0.02)
    plain = Server(ex2, max_batch_keys=0, lanes=("all",), lane_of=lambda r: "all").start()
    reqs = _reqs([("u32", 10), ("kv", 10), ("u32", 10)])
    for r in reqs:
        plain.submit(r)
    plain.drain(3)
    assert ex2.max_active == 1 and [b for _, b in ex2.batches] == [[0], [1], [2]]


def test_percentiles():
    p = percentiles(list(range(101)))
    assert p["p50"] == 50.0 and p["p99"] == 99.0
