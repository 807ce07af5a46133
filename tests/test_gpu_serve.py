"""Served results on the GPU equal the results of each mesh built alone."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests.test_serve import make_requests

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_served_equals_alone(oracle_mod):
    from paper_1604_04689_amd import serve
    reqs = make_requests(40, rate=20000.0, seed=11)
    got = {}

    def on_complete(batch, ex):
        ex.check(batch)
        for r, res in zip(batch.requests, ex.results(batch)):
            got[r.rid] = res

    clock = serve.RealClock()
    srv = serve.Server(serve.GpuExecutor(3), clock, n_slots=3, budget_bytes=1 << 34, max_batch=8,
                       on_complete=on_complete)
    done = srv.run(reqs)
    assert len(got) == len(reqs)
    assert srv.batches < len(reqs)  # some batching happened
    for r in reqs:
        wn = oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert)
        we = oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert)
        (gnr, gnc), (ger, gec) = got[r.rid]
        assert np.array_equal(gnr, wn[0]) and np.array_equal(gnc, wn[1]), r.rid
        assert np.array_equal(ger, we[0]) and np.array_equal(gec, we[1]), r.rid
    s = serve.latency_summary(done)
    print("served:", s, "batches:", srv.batches, flush=True)


def test_served_device_inputs_equal_alone(oracle_mod):
    """Requests whose connectivity is already a device tensor (copied into
    the arena on the upload stream, runs of adjacent ranges in one
    concatenation) give the same results as the oracle."""
    from paper_1604_04689_amd import serve
    reqs = make_requests(40, rate=20000.0, seed=13)
    host = {r.rid: r.conn for r in reqs}
    for r in reqs:
        r.conn = torch.as_tensor(r.conn).to("cuda:0")
    got = {}

    def on_complete(batch, ex):
        ex.check(batch)
        for r, res in zip(batch.requests, ex.results(batch)):
            got[r.rid] = res

    srv = serve.Server(serve.GpuExecutor(3), serve.RealClock(), n_slots=3, budget_bytes=1 << 34, max_batch=8,
                       on_complete=on_complete)
    srv.run(reqs)
    assert len(got) == len(reqs) and srv.batches < len(reqs)
    for r in reqs:
        conn = host[r.rid]
        wn = oracle_mod.node_neighbors(conn, r.etype, r.n_vert)
        we = oracle_mod.elem_neighbors(conn, r.etype, r.n_vert)
        (gnr, gnc), (ger, gec) = got[r.rid]
        assert np.array_equal(gnr, wn[0]) and np.array_equal(gnc, wn[1]), r.rid
        assert np.array_equal(ger, we[0]) and np.array_equal(gec, we[1]), r.rid


def test_served_with_small_arena(oracle_mod):
    """A connectivity arena that holds only two requests at a time: uploads
    wait for batches to release their ranges, results stay exact."""
    from paper_1604_04689_amd import serve
    reqs = make_requests(16, rate=50000.0, seed=12)
    biggest = max(r.conn.size for r in reqs)
    got = {}

    def on_complete(batch, ex):
        ex.check(batch)
        for r, res in zip(batch.requests, ex.results(batch)):
            got[r.rid] = res

    ex = serve.GpuExecutor(2, arena_ids=2 * (biggest + 64))
    srv = serve.Server(ex, serve.RealClock(), n_slots=2, budget_bytes=1 << 34, max_batch=8,
                       on_complete=on_complete)
    srv.run(reqs)
    assert len(got) == len(reqs) and ex.arena.in_use() == 0
    for r in reqs:
        wn = oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert)
        we = oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert)
        (gnr, gnc), (ger, gec) = got[r.rid]
        assert np.array_equal(gnr, wn[0]) and np.array_equal(gnc, wn[1]), r.rid
        assert np.array_equal(ger, we[0]) and np.array_equal(gec, we[1]), r.rid


@pytest.mark.slow
def test_served_full_distribution_equals_alone(oracle_mod):
    """Requests drawn from the full size distribution of the batch workload
    (triangle grids up to 512^2 vertices, Kuhn and hex cubes up to 48^3
    cells, three of them forced to 48^3 Kuhn), served with continuous
    batching: every result equals the oracle's, element by element."""
    from paper_1604_04689_amd import serve
    reqs = make_requests(40, rate=2000.0, seed=21, small=False)
    for i in (3, 17, 29):
        m = mg.kuhn_tet_grid(48, 100 + i)
        reqs[i] = serve.Request(i, reqs[i].arrival, m.conn, m.etype, m.n_vert)
    print(f"[serve] {len(reqs)} requests, {sum(r.n_elem for r in reqs)} elements", flush=True)
    got = {}

    def on_complete(batch, ex):
        ex.check(batch)
        for r, res in zip(batch.requests, ex.results(batch)):
            got[r.rid] = res

    srv = serve.Server(serve.GpuExecutor(4), serve.RealClock(), n_slots=4, budget_bytes=64 << 30, max_batch=16,
                       on_complete=on_complete)
    srv.run(reqs)
    assert len(got) == len(reqs) and srv.batches < len(reqs)
    for r in reqs:
        wn = oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert)
        we = oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert)
        (gnr, gnc), (ger, gec) = got[r.rid]
        assert np.array_equal(gnr, wn[0]) and np.array_equal(gnc, wn[1]), r.rid
        assert np.array_equal(ger, we[0]) and np.array_equal(gec, we[1]), r.rid


def test_served_results_stay_resident_until_released(oracle_mod):
    """keep_results: each request's CSRs stay in device memory, untouched by
    the later batches that reuse its slot, until the client releases them;
    every one equals the oracle's, element by element."""
    from paper_1604_04689_amd import serve
    reqs = make_requests(30, rate=20000.0, seed=13)
    srv = serve.Server(serve.GpuExecutor(2), serve.RealClock(), n_slots=2, budget_bytes=1 << 34, max_batch=4,
                       keep_results=True, on_complete=lambda b, ex: ex.check(b))
    done = srv.run(reqs)
    assert srv.batches > 2 and srv.unreleased == len(reqs)  # slots were reused while results were held
    for r in done:
        rp, cols = r.result.node()
        assert rp.device.type == "cuda" and cols.device.type == "cuda"
        wn = oracle_mod.node_neighbors(r.conn, r.etype, r.n_vert)
        we = oracle_mod.elem_neighbors(r.conn, r.etype, r.n_vert)
        (gnr, gnc), (ger, gec) = r.result.to_host()
        assert np.array_equal(gnr, wn[0]) and np.array_equal(gnc, wn[1]), r.rid
        assert np.array_equal(ger, we[0]) and np.array_equal(gec, we[1]), r.rid
    for r in done:
        r.result.release()
    assert srv.resident_bytes == 0 and srv.in_use == 0
