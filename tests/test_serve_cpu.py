"""Scheduler logic of the request loop on the CPU (fake executor, fake clock):
admission by footprint, FIFO order, slot reuse, overlap, latency statistics."""
from paper_2601_11621_amd.serve import DONE, FAILED, FakeExecutor, Server


def _drive(srv, ex, dt=0.001, limit=100000):
    k = 0
    while not srv.idle() and k < limit:
        if not srv.step():
            if srv.active:
                ex.tick(dt)
            elif srv.queue:
                ex.wait_until(srv.queue[0].arrival)
        k += 1
    assert srv.idle()


def test_budget_limits_concurrency_and_keeps_fifo():
    ex = FakeExecutor(lambda n: 0.01, lambda n: 0.02)
    srv = Server(ex, budget_bytes=250, max_slots=8, clock=ex.clock)
    reqs = [srv.submit(100, arrival=0.0) for _ in range(6)]
    _drive(srv, ex)
    assert all(r.state == DONE for r in reqs)
    assert srv.peak_used <= 250 and srv.peak_active == 2        # two footprints of 100 fit
    begins = [rid for (what, rid, t) in ex.log if what == "begin"]
    assert begins == sorted(begins)                               # FIFO admission


def test_slots_limit_and_reuse():
    ex = FakeExecutor(lambda n: 0.005, lambda n: 0.005)
    srv = Server(ex, budget_bytes=10**9, max_slots=3, clock=ex.clock)
    reqs = [srv.submit(10, arrival=0.0) for _ in range(10)]
    _drive(srv, ex)
    assert srv.peak_active == 3
    assert sorted({r.slot for r in reqs}) == [0, 1, 2]
    assert all(r.state == DONE and r.n_limbs == 10 for r in reqs)


def test_late_arrivals_are_admitted_while_others_run():
    """Continuous admission: a request arriving while a long one runs starts
    before the long one finishes."""
    ex = FakeExecutor(lambda n: 0.001, lambda n: n * 0.001)
    srv = Server(ex, budget_bytes=10**6, max_slots=4, clock=ex.clock)
    long = srv.submit(1000, arrival=0.0)      # runs for ~1 s
    short = srv.submit(5, arrival=0.1)
    _drive(srv, ex)
    assert short.admitted < long.finished
    assert short.finished < long.finished
    assert abs(short.admitted - 0.1) < 0.01


def test_head_too_large_is_failed_not_blocking():
    ex = FakeExecutor(lambda n: 0.001, lambda n: 0.001)
    srv = Server(ex, budget_bytes=100, max_slots=2, clock=ex.clock)
    big = srv.submit(1000, arrival=0.0)
    small = srv.submit(10, arrival=0.0)
    _drive(srv, ex)
    assert big.state == FAILED and small.state == DONE


def test_large_head_waits_for_memory():
    ex = FakeExecutor(lambda n: 0.001, lambda n: 0.05)
    srv = Server(ex, budget_bytes=100, max_slots=4, clock=ex.clock)
    a = srv.submit(60, arrival=0.0)
    b = srv.submit(60, arrival=0.0)      # must wait for a
    c = srv.submit(10, arrival=0.0)      # behind b: FIFO, waits too
    _drive(srv, ex)
    assert b.admitted >= a.finished
    assert c.admitted >= b.admitted


def test_latency_percentiles():
    ex = FakeExecutor(lambda n: 0.0, lambda n: n * 0.001)
    srv = Server(ex, budget_bytes=10**9, max_slots=100, clock=ex.clock)
    for k in range(1, 101):
        srv.submit(k, arrival=0.0)
    _drive(srv, ex, dt=0.0005)
    st = srv.stats()
    assert st["completed"] == 100
    assert 45 <= st["p50_ms"] <= 56
    assert 95 <= st["p99_ms"] <= 102


def test_cancel_frees_slot_and_budget():
    """A running request that is cancelled gives its slot and its memory back
    at once (its device work drained by the executor's abort), so the request
    waiting behind it is admitted; a queued one simply leaves the queue."""
    from paper_2601_11621_amd.serve import CANCELLED

    ex = FakeExecutor(lambda n: 0.001, lambda n: 1.0)
    srv = Server(ex, budget_bytes=100, max_slots=1, clock=ex.clock)
    a = srv.submit(80, arrival=0.0)
    b = srv.submit(80, arrival=0.0)       # waits for a's slot and memory
    c = srv.submit(10, arrival=0.0)
    srv.step()
    assert srv.active == [a] and srv.used == 80
    assert srv.cancel(c) and c.state == CANCELLED and c not in srv.queue
    assert srv.cancel(a)
    assert a.state == CANCELLED and srv.used == 0 and srv.free_slots == [0]
    assert ("abort", a.rid, ex.now) in ex.log and a.rid not in ex.open
    _drive(srv, ex)
    assert b.state == DONE and b.admitted <= a.finished + 1e-9
    assert not srv.cancel(b)              # already finished
    st = srv.stats()
    assert st["completed"] == 1 and st["cancelled"] == 2


def test_failed_finish_releases_once_and_server_continues():
    """An executor whose finish raises (e.g. a capacity or device error from
    the library) has its request failed exactly once: the executor drops the
    handle before raising, the server's abort then finds nothing to release,
    and later requests are served normally."""
    ex = FakeExecutor(lambda n: 0.001, lambda n: 0.002, fail_finish=lambda n: n == 13)
    srv = Server(ex, budget_bytes=1000, max_slots=2, clock=ex.clock)
    bad = srv.submit(13, arrival=0.0)
    good = [srv.submit(20 + k, arrival=0.0) for k in range(4)]
    _drive(srv, ex)
    assert bad.state == FAILED and "finish failed" in bad.error
    assert all(r.state == DONE for r in good)
    aborts = [rid for (what, rid, t) in ex.log if what == "abort"]
    assert aborts == [bad.rid] and not ex.open
    assert srv.used == 0 and sorted(srv.free_slots) == [0, 1]


def test_on_done_sees_every_request_once():
    seen = []
    ex = FakeExecutor(lambda n: 0.001, lambda n: 0.001)
    srv = Server(ex, budget_bytes=50, max_slots=2, clock=ex.clock, on_done=lambda r: seen.append(r.rid))
    rs = [srv.submit(n, arrival=0.0) for n in (10, 100, 20)]   # 100 exceeds the budget
    _drive(srv, ex)
    assert sorted(seen) == [r.rid for r in rs]
    assert rs[1].state == FAILED


class _FakeBatching(FakeExecutor):
    """Fake executor that, like the batch executor, starts the requests of one
    admission step together when the server flushes."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.forming, self.batches = [], []

    def begin(self, r):
        r.handle = None
        self.forming.append(r)
        self.log.append(("begin", r.rid, self.now))

    def flush(self):
        if self.forming:
            self.batches.append([r.rid for r in self.forming])
            for r in self.forming:
                r.handle = self.now + self.p1(r.n)
            self.forming = []
        return []


def test_flush_batches_each_admission_step():
    """Requests admitted in the same step are flushed as one batch; requests
    arriving while that batch runs form the next one (continuous batching)."""
    ex = _FakeBatching(lambda n: 0.001, lambda n: 0.01)
    srv = Server(ex, budget_bytes=10**6, max_slots=8, clock=ex.clock)
    first = [srv.submit(10, arrival=0.0) for _ in range(3)]
    late = [srv.submit(20, arrival=0.005) for _ in range(2)]
    _drive(srv, ex)
    assert all(r.state == DONE for r in first + late)
    assert ex.batches[0] == [r.rid for r in first]
    assert ex.batches[1] == [r.rid for r in late]
    assert late[0].admitted < first[0].finished          # admitted while the first batch ran
