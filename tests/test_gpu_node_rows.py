"""The row-based node algorithms give bit-identical results to the oracle:
vertex-rows (sort by the vertex bits only, then per-row sort and
deduplication) and edge-rows (each edge once by its lower vertex, then
transposed by its higher vertex)."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests import pins
from tests.test_gpu_parity import assert_same, gpu_csr

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[1, 2], ids=["vertex_rows", "edge_rows"])
def rows_mode(request):
    """Every test of this file runs under both row-based node algorithms
    (the options of each call)."""
    return {"node_sort": request.param}


def check_node(oracle_mod, conn, etype, n_vert, what="", opts=None):
    print(f"[rows] {what} n_vert={n_vert} {opts}", flush=True)
    assert_same(gpu_csr("node", conn, etype, n_vert, options=opts), oracle_mod.node_neighbors(conn, etype, n_vert),
                what)


def test_golden_rows(rows_mode, oracle_mod):
    for case in pins.read_golden():
        conn = case["conn"].reshape(-1, pins.NPE[case["etype"]])
        assert_same(gpu_csr("node", conn, case["etype"], case["n_vert"], options=rows_mode),
                    (case["node_row_ptr"], case["node_cols"]), case["name"])


@pytest.mark.parametrize("etype", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("size", [(1, 1), (300, 90), (5000, 4096), (60000, 9000), (20000, 2 ** 16), (30000, 2 ** 25 - 3)])
def test_random_rows(rows_mode, oracle_mod, etype, size):
    n_elem, n_vert = size
    m = mg.random_mesh(n_elem, n_vert, etype, seed=n_elem + 3 * etype + 1)
    check_node(oracle_mod, m.conn, etype, n_vert, m.name, rows_mode)


def test_top_vertex_used(rows_mode, oracle_mod):
    # n_vert a power of two and the last vertex in use: its keys must not tie
    # with the key of a dropped pair
    for nv in (2, 4, 1024):
        conn = np.array([[nv - 1, 0, 1 % nv], [nv - 1, nv - 1, 0], [0, 0, 0]], dtype=np.int32)
        check_node(oracle_mod, conn, 0, nv, f"top vertex {nv}", rows_mode)
    m = mg.tri_grid(64, "coin", 9)  # 4096 vertices
    check_node(oracle_mod, m.conn, 0, m.n_vert, "tri64 coin", rows_mode)


def test_long_rows(rows_mode, oracle_mod):
    # hub vertex 0 with rows of 200 (short), 300 (long, LDS), 18000 pairs (long, global memory)
    for n in (100, 150, 5000, 9000):
        rim = np.arange(1, n + 2, dtype=np.int32)
        conn = np.stack([np.zeros(n, np.int32), rim[:-1], rim[1:]], 1)
        conn = conn[np.random.default_rng(n).permutation(n)]
        check_node(oracle_mod, conn, 0, n + 2, f"fan{n}", rows_mode)
    # many hubs with repeated neighbors
    rng = np.random.default_rng(4)
    conn = rng.integers(0, 40, size=(20000, 4)).astype(np.int32)
    check_node(oracle_mod, conn, 1, 40, "dense40", rows_mode)


def test_degenerate_rows(rows_mode, oracle_mod):
    rng = np.random.default_rng(9)
    conn = rng.integers(0, 6, size=(4000, 4)).astype(np.int32)
    check_node(oracle_mod, conn, 1, 8, "degenerate", rows_mode)
    check_node(oracle_mod, np.zeros((50, 3), np.int32), 0, 1, "all-self", rows_mode)
    r, c = gpu_csr("node", np.zeros((0, 3), np.int32), 0, 5, options=rows_mode)
    assert r.tolist() == [0] * 6 and c.shape == (0,)


def test_every_shape_rows(rows_mode, oracle_mod):
    m = mg.kuhn_tet_grid(14, 3)
    want = oracle_mod.node_neighbors(m.conn, m.etype, m.n_vert)
    for shape in range(7):
        assert_same(gpu_csr("node", m.conn, m.etype, m.n_vert, options={**rows_mode, "radix_shape": shape}), want,
                    f"shape {shape}")


@pytest.mark.slow
def test_full_meshes_rows(rows_mode, oracle_mod):
    for m in (mg.tri2048(), mg.kuhn96()):
        check_node(oracle_mod, m.conn, m.etype, m.n_vert, m.name, rows_mode)
