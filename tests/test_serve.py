"""Continuous-batching server logic on the CPU (fake executor, simulated clock)."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from paper_1604_04689_amd import serve


def make_requests(n, rate, seed=3, small=True):
    specs = mg.batch_specs(n_mesh=n, seed=seed, tri_range=(4, 40) if small else (8, 512),
                           cell_range=(1, 6) if small else (4, 48))
    arr = mg.poisson_arrivals(n, rate, seed=seed + 1)
    out = []
    for i, (s, t) in enumerate(zip(specs, arr)):
        m = s.build()
        out.append(serve.Request(i, float(t), m.conn, m.etype, m.n_vert))
    return out


def run(reqs, **kw):
    clock = serve.SimClock()
    ex = serve.FakeExecutor(clock, t0=kw.pop("t0", 1e-4), per_elem=kw.pop("per_elem", 1e-8),
                            compute=kw.pop("compute", None))
    srv = serve.Server(ex, clock, **kw)
    done = srv.run(reqs)
    return srv, done


def test_all_complete_in_order_and_within_budget():
    reqs = make_requests(60, rate=2000.0)
    budget = 3 * max(serve.reserve_bytes(r.n_elem, r.etype, r.n_vert) for r in reqs)
    srv, done = run(reqs, n_slots=3, budget_bytes=budget, max_batch=8)
    assert all(r.completed >= r.admitted >= r.arrival for r in done)
    assert srv.peak_in_use <= budget
    assert srv.in_use == 0
    # admission is FIFO
    adm = [r.admitted for r in sorted(done, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert max(srv.batch_sizes) <= 8


def test_budget_makes_requests_wait():
    reqs = make_requests(30, rate=1e6)  # all arrive at once
    one = max(serve.reserve_bytes(r.n_elem, r.etype, r.n_vert) for r in reqs)
    srv, done = run(reqs, n_slots=8, budget_bytes=one, max_batch=64)
    # the budget holds about one large request: memory, not slots, gates admission
    assert srv.peak_in_use <= one
    assert srv.batches > 8  # more launches than slots: requests waited for memory
    waits = [r.admitted - r.arrival for r in done]
    assert max(waits) > 0


def test_oversize_request_refused():
    reqs = make_requests(5, rate=100.0)
    with pytest.raises(serve.BudgetError):
        run(reqs, budget_bytes=10)


def test_continuous_admission_while_running():
    # a long first batch; later arrivals start on other slots before it ends
    reqs = make_requests(12, rate=50000.0)
    srv, done = run(reqs, n_slots=4, budget_bytes=1 << 40, max_batch=1, per_elem=1e-6)
    first = min(done, key=lambda r: r.arrival)
    overlapped = [r for r in done if r is not first and r.admitted < first.completed]
    assert overlapped, "no request was admitted while the first batch was running"


def test_results_same_alone_and_in_mix(oracle_mod):
    reqs = make_requests(25, rate=5000.0)
    got = {}

    def on_complete(batch, ex):
        for r, res in zip(batch.requests, ex.results(batch)):
            got[r.rid] = res

    def compute(r):
        return (oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert),
                oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert))

    srv, done = run(reqs, n_slots=2, budget_bytes=1 << 40, max_batch=6, compute=compute, on_complete=on_complete)
    for r in reqs:
        alone = compute(r)
        for k in range(2):
            assert np.array_equal(got[r.rid][k][0], alone[k][0]) and np.array_equal(got[r.rid][k][1], alone[k][1])


def test_latency_summary():
    reqs = make_requests(20, rate=1000.0)
    srv, done = run(reqs, n_slots=2, budget_bytes=1 << 40)
    s = serve.latency_summary(done)
    assert s["requests"] == 20 and s["p99_ms"] >= s["p50_ms"] >= 0 and s["elements_per_s"] > 0


def test_arena_first_fit_and_merge():
    a = serve.Arena(1024, align=64)
    x = a.alloc(100)   # 128
    y = a.alloc(64)
    z = a.alloc(500)   # 512
    assert (x, y, z) == (0, 128, 192)
    assert a.alloc(400) is None           # 1024 - 704 = 320 left
    a.release(y)
    assert a.alloc(64) == 128             # first fit reuses the hole
    a.release(x)
    a.release(128)
    assert a.free[0] == (0, 192)          # holes merged
    a.release(z)
    assert a.free == [(0, 1024)] and a.in_use() == 0
    assert a.alloc(1024) == 0 and a.alloc(1) is None


def test_staged_executor_admits_only_prepared():
    """An executor with a prepare step: a request whose upload cannot start
    (arena full) waits, and later requests wait behind it (FIFO)."""
    clock = serve.SimClock()

    class Staged(serve.FakeExecutor):
        def __init__(self, clock):
            super().__init__(clock, t0=1.0, per_elem=0.0)
            self.room = 1

        def prepare(self, r):
            if self.room == 0:
                return False
            self.room -= 1
            r.prep = ("slot", r.rid)
            return True

        def release(self, batch):
            for r in batch.requests:
                r.prep = None
                self.room += 1
            super().release(batch)

    ex = Staged(clock)
    conn = np.zeros((4, 3), dtype=np.int32)
    reqs = [serve.Request(i, 0.0, conn, 0, 3) for i in range(3)]
    srv = serve.Server(ex, clock, n_slots=4, budget_bytes=1 << 40, max_batch=8, reserve=lambda *a: 1)
    done = srv.run(reqs)
    # one arena room: the requests run one at a time, one second each
    assert sorted(r.completed for r in done) == [1.0, 2.0, 3.0]
    assert srv.batches == 3


def test_results_resident_until_released(oracle_mod):
    """keep_results: every request's result handle stays valid after later
    batches ran, holds its bytes in the budget until released, and equals
    the request computed alone."""
    reqs = make_requests(20, rate=5000.0, seed=31)

    def compute(r):
        return (oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert),
                oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert))

    srv, done = run(reqs, n_slots=2, budget_bytes=1 << 40, max_batch=4, compute=compute, keep_results=True)
    held = sum(serve.output_bytes(r.n_elem, r.etype, r.n_vert) for r in reqs)
    assert srv.resident_bytes == held and srv.in_use == held and srv.unreleased == len(reqs)
    for r in done:
        (nr, nc), (er, ec) = r.result.to_host()
        (wnr, wnc), (wer, wec) = compute(r)
        assert np.array_equal(nr, wnr) and np.array_equal(nc, wnc)
        assert np.array_equal(er, wer) and np.array_equal(ec, wec)
    for r in done:
        r.result.release()
        r.result.release()  # idempotent
    assert srv.resident_bytes == 0 and srv.in_use == 0 and srv.unreleased == 0
    with pytest.raises(ValueError):
        done[0].result.node()


def test_unreleased_results_hold_the_budget():
    """A client that keeps its last two results: later requests are admitted
    only as older results are released; one that keeps everything under a
    budget too small for that is told why the server cannot go on.  Sizes
    are set by hand: 10 bytes in flight, of which 4 stay with the result."""
    sizes = dict(reserve=lambda *a: 10, resident=lambda *a: 4)
    budget = 10 + 2 * 4  # one request in flight beside two kept results
    kept = []

    def keep_two(batch, ex):
        kept.extend(r.result for r in batch.requests)
        while len(kept) > 2:
            kept.pop(0).release()

    srv, done = run(make_requests(16, rate=1e6, seed=32), n_slots=2, budget_bytes=budget, max_batch=1,
                    keep_results=True, on_complete=keep_two, **sizes)
    assert len(done) == 16 and srv.peak_in_use <= budget and srv.unreleased == 2 and srv.in_use == 8
    with pytest.raises(serve.BudgetError, match="unreleased results"):
        run(make_requests(16, rate=1e6, seed=32), n_slots=2, budget_bytes=budget, max_batch=1, keep_results=True,
            **sizes)


def test_frozen_gc_restores_the_collector():
    import gc
    from paper_1604_04689_amd import serve
    before = gc.get_freeze_count()
    with serve.frozen_gc():
        assert gc.get_freeze_count() > before
    assert gc.get_freeze_count() == before
