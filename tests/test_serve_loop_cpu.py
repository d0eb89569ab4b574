"""CPU tests of the request loop (serve.run) against a host-side stand-in
for the continuous-batching server: every request is collected once, with
its own result; a server without a tolerance is polled only when one of its
requests has reached its iteration cap (or every poll_every turns), one with
a tolerance every turn."""
import numpy as np

from paper_1807_08692_amd import serve


class FakeServer:
    """Columns run one iteration per step until their cap (tol <= 0) or a
    seeded earlier stop (tol > 0); poll returns the finished ones."""

    def __init__(self, slots, tol=0.0, seed=0):
        self.slots, self.tol = slots, tol
        self.cols = {}          # ticket -> [iterations done, cap, stop]
        self.next_ticket = 0
        self.polls = 0
        self.steps = 0
        self.rng = np.random.default_rng(seed)

    @property
    def in_use(self):
        return len(self.cols)

    def submit(self, y_ids=None, y_val=None, q_desc=None, max_iter=None):
        n = len(max_iter)
        free = self.slots - len(self.cols)
        tickets = []
        for k in range(min(n, free)):
            cap = int(max_iter[k])
            stop = cap if self.tol <= 0 else int(self.rng.integers(0, cap + 1))
            self.cols[self.next_ticket] = [0, cap, stop]
            tickets.append(self.next_ticket)
            self.next_ticket += 1
        return np.array(tickets, np.int64)

    def step(self, iters=1):
        self.steps += 1
        for c in self.cols.values():
            c[0] = min(c[0] + iters, c[2])

    def poll(self, max_out=1024):
        self.polls += 1
        done = [t for t, c in self.cols.items() if c[0] >= c[2]][:max_out]
        res = {"tickets": np.array(done, np.int64), "ids": np.array([[t] for t in done]),
               "scores": np.zeros((len(done), 1)), "iters": np.array([self.cols[t][0] for t in done]),
               "relres": np.zeros(len(done)), "status": np.zeros(len(done), np.int32)}
        for t in done:
            del self.cols[t]
        return res


def make_requests(n, db, seed):
    rng = np.random.default_rng(seed)
    caps = rng.integers(0, 9, size=n)
    return [serve.Request(i, 0.0, db, y_ids=np.zeros(2, np.int32), y_val=np.ones(2, np.float32),
                          max_iter=int(caps[i])) for i in range(n)]


def test_every_request_collected_once_with_its_iterations():
    srv = FakeServer(slots=16)
    reqs = make_requests(100, "a", 1)
    out, _ = serve.run({"a": srv}, reqs)
    assert all(r.finished >= r.admitted >= 0 for r in out)
    # the ticket order is admission order, which is request order here
    assert [int(r.result["ids"][0]) for r in out] == list(range(100))
    assert all(int(r.result["iters"]) == r.max_iter for r in out)


def test_capped_server_polled_only_when_a_request_is_due():
    srv = FakeServer(slots=8)
    reqs = make_requests(60, "a", 2)
    serve.run({"a": srv}, reqs, poll_every=1000)
    # a poll happens only on a turn at which some admitted request has run
    # to its cap; each such poll collects at least one request
    assert srv.polls <= len(reqs)


def test_server_with_tolerance_polled_every_turn():
    capped, tolerant = FakeServer(slots=8, tol=0.0), FakeServer(slots=8, tol=1e-6, seed=3)
    serve.run({"a": capped}, make_requests(40, "a", 4), poll_every=1000)
    serve.run({"b": tolerant}, make_requests(40, "b", 4), poll_every=1000)
    # every turn that stepped the tolerant server also polled it; the capped
    # one skipped the turns on which no request had reached its cap
    assert tolerant.polls >= tolerant.steps
    assert capped.polls < capped.steps
    # early stops (tol > 0) are collected although they precede their caps
    assert tolerant.in_use == 0 and capped.in_use == 0
