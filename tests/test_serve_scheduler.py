"""The serving scheduler against a scripted executor (no GPU): admission
stays under the memory budget, evaluations wait for their tree, slots bound
concurrency, least-recently-used trees are evicted (never one an evaluation
is reading), and every request completes with its latency recorded."""
import pytest

from paper_1511_01353_amd.serve import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Work finishes a scripted time after it starts (per point/query)."""

    def __init__(self, clock, fit_rate=1e6, eval_rate=1e7):
        self.clock = clock
        self.fit_rate = fit_rate
        self.eval_rate = eval_rate
        self.live_trees = set()
        self.released = []
        self.concurrent_evals = 0
        self.max_concurrent_evals = 0
        self.reads = []   # (tree, start, end) of every evaluation
        self.fit_starts = []   # (start, end, slot) of every fit batch

    def fit_footprint(self, req):
        return 100 * req.n

    def eval_footprint(self, req):
        return 10 * req.n

    def tree_bytes(self, req, tree):
        return 20 * req.n

    def release_tree(self, tree):
        self.live_trees.discard(tree)
        self.released.append((tree, self.clock()))

    def start_fit_batch(self, reqs, slot=0):
        end = self.clock() + sum(r.n for r in reqs) / self.fit_rate
        self.fit_starts.append((self.clock(), end, slot))
        return {"kind": "fit", "end": end, "reqs": reqs}

    def start_eval(self, req, tree):
        assert tree in self.live_trees, "evaluation on a released tree"
        self.concurrent_evals += 1
        self.max_concurrent_evals = max(self.max_concurrent_evals, self.concurrent_evals)
        end = self.clock() + req.n / self.eval_rate
        self.reads.append((tree, self.clock(), end))
        return {"kind": "eval", "end": end, "req": req}

    def done(self, h):
        return self.clock() >= h["end"]

    def result(self, h):
        if h["kind"] == "fit":
            trees = []
            for r in h["reqs"]:
                t = f"tree{r.rid}"
                self.live_trees.add(t)
                trees.append(t)
            return trees
        self.concurrent_evals -= 1
        return h["req"].n


def drive(server, reqs, ex, clock, dt=1e-4, limit=100000):
    for r in reqs:
        server.submit(r)
    steps = 0
    while not server.idle():
        server.tick()
        assert server.used() <= server.budget, (server.used(), server.budget)
        clock.t += dt
        steps += 1
        assert steps < limit
    return server.finished


def make_stream():
    reqs, rid = [], 0
    for k in range(4):
        reqs.append(Request(rid=rid, kind="fit", arrival=0.001 * k, n=2000 + 500 * k, opts={"p": 4}))
        rid += 1
    for k in range(12):
        reqs.append(Request(rid=rid, kind="eval", arrival=0.0005 * k, n=5000, tree=k % 4))
        rid += 1
    return reqs


def test_all_requests_complete_under_budget():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=2_000_000, eval_slots=3, clock=clock)
    done = drive(srv, make_stream(), ex, clock)
    assert len(done) == 16 and all(r.error is None for r in done)
    assert srv.peak <= srv.budget
    assert ex.max_concurrent_evals <= 3
    for r in done:
        assert r.arrival <= r.admitted <= r.done
        if r.kind == "eval":
            fit = next(f for f in done if f.rid == r.tree)
            assert r.admitted >= fit.done      # waited for its tree
    st = srv.stats()
    assert st["fit"]["count"] == 4 and st["eval"]["count"] == 12
    assert st["eval"]["p99_ms"] >= st["eval"]["p50_ms"]


def test_fits_arriving_together_are_batched():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=10_000_000, clock=clock)
    reqs = [Request(rid=i, kind="fit", arrival=0.0, n=1000, opts={"p": 4}) for i in range(5)]
    batches = []
    orig = ex.start_fit_batch
    ex.start_fit_batch = lambda rs, slot=0: (batches.append(len(rs)), orig(rs, slot))[1]
    drive(srv, reqs, ex, clock)
    assert batches == [5]


def test_lru_eviction_and_in_use_trees_are_kept():
    clock = FakeClock()
    ex = FakeExecutor(clock, eval_rate=1e5)
    # room for about two resident trees next to one running evaluation
    srv = Server(ex, budget_bytes=2 * 20 * 10000 + 10 * 20000 + 1000, eval_slots=1, clock=clock)
    reqs = [Request(rid=0, kind="fit", arrival=0.0, n=10000, opts={"p": 4}),
            Request(rid=1, kind="fit", arrival=0.0, n=10000, opts={"p": 4}),
            Request(rid=2, kind="eval", arrival=0.0, n=20000, tree=0),
            Request(rid=3, kind="fit", arrival=0.0, n=10000, opts={"p": 4}),
            Request(rid=4, kind="eval", arrival=0.0, n=20000, tree=1)]
    srv.budget = 10_000_000       # the three fits need room at first
    for r in reqs:
        srv.submit(r)
    while not srv.idle():
        srv.tick()
        if all(f in srv.trees for f in (0, 1, 3)):
            srv.budget = 2 * 20 * 10000 + 10 * 20000 + 1000
        clock.t += 1e-4
    # every evaluation read a live tree (asserted inside the executor), and a
    # released tree was never read after its release
    for tree, t_rel in ex.released:
        for t, s0, s1 in ex.reads:
            if t == tree:
                assert s1 <= t_rel + 1e-12
    assert all(r.error is None for r in srv.finished)


def test_eval_of_failed_fit_is_reported():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=10_000_000, clock=clock)
    orig = ex.result

    def res(h):
        out = orig(h)
        if h["kind"] == "fit":
            return [RuntimeError("boom")] * len(out)
        return out

    ex.result = res
    reqs = [Request(rid=0, kind="fit", arrival=0.0, n=1000, opts={"p": 4}),
            Request(rid=1, kind="eval", arrival=0.0, n=100, tree=0)]
    done = drive(srv, reqs, ex, clock)
    assert {r.rid: r.error is not None for r in done} == {0: True, 1: True}


def test_oversized_request_is_rejected_not_stalled():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget_bytes=50_000, clock=clock)
    reqs = [Request(rid=0, kind="fit", arrival=0.0, n=100_000, opts={"p": 4}),
            Request(rid=1, kind="eval", arrival=0.0, n=10, tree=0),
            Request(rid=2, kind="fit", arrival=0.0, n=100, opts={"p": 4})]
    done = drive(srv, reqs, ex, clock)
    errs = {r.rid: r.error for r in done}
    assert errs[0] and errs[1] and errs[2] is None


def max_overlap(spans):
    ev = sorted([(a, 1) for a, b, _ in spans] + [(b, -1) for a, b, _ in spans], key=lambda t: (t[0], t[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


@pytest.mark.parametrize("slots", [1, 2])
def test_fit_batches_in_flight_bounded_by_slots(slots):
    """A fit arriving while a batch runs starts at once in a free fit slot
    (on its own stream) when memory allows; with one slot it waits."""
    clock = FakeClock()
    ex = FakeExecutor(clock, fit_rate=1e6)
    srv = Server(ex, budget_bytes=100_000_000, clock=clock, fit_slots=slots)
    reqs = [Request(rid=0, kind="fit", arrival=0.0, n=20000, opts={"p": 4}),
            Request(rid=1, kind="fit", arrival=0.001, n=20000, opts={"p": 4}),
            Request(rid=2, kind="fit", arrival=0.002, n=20000, opts={"p": 4})]
    drive(srv, reqs, ex, clock)
    # with one slot the two later fits wait together and go as one batch
    assert len(ex.fit_starts) == (3 if slots == 2 else 2)
    assert max_overlap(ex.fit_starts) == slots
    # concurrent batches never share a slot
    for i, (a, b, s) in enumerate(ex.fit_starts):
        for a2, b2, s2 in ex.fit_starts[i + 1:]:
            if a2 < b and a < b2:
                assert s != s2


def test_workspace_counted_against_the_budget():
    """The library's per-stream fit workspace (grow-only) is part of the
    memory in use: a second slot's workspace is admitted only if it fits."""
    clock = FakeClock()
    ex = FakeExecutor(clock, fit_rate=1e6)
    ex.workspace_bytes = lambda rs: 50 * sum(r.n for r in rs)
    # one fit (footprint 100 n) plus its workspace (50 n) fits; two do not
    n = 10000
    srv = Server(ex, budget_bytes=int(1.6 * 150 * n), clock=clock, fit_slots=2)
    reqs = [Request(rid=0, kind="fit", arrival=0.0, n=n, opts={"p": 4}),
            Request(rid=1, kind="fit", arrival=0.001, n=n, opts={"p": 4})]
    drive(srv, reqs, ex, clock)   # asserts used() <= budget at every tick
    assert max_overlap(ex.fit_starts) == 1
    assert all(r.error is None for r in srv.finished)
    assert srv.peak <= srv.budget
