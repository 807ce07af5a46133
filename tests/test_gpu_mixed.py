"""Meshes whose elements carry their own types, through mesh_mixed_neighbors,
against the oracle's mixed entry points: hand cases, random mixes (with
degenerate elements), hybrid hex/wedge/pyramid/tet grids, meshes of one
type given as mixed, malformed elements and empty meshes.  Bit-exact."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests import pins

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _nb():
    import paper_1604_04689_amd as nb
    return nb


def gpu_mixed(conn, etypes, n_vert, options=None):
    nb = _nb()
    c = torch.as_tensor(np.ascontiguousarray(conn, dtype=np.int32)).to(DEV)
    t = torch.as_tensor(np.ascontiguousarray(etypes, dtype=np.uint8)).to(DEV)
    (nr, nc), (er, ec) = nb.mixed_neighbors(c, t, n_vert, options=options)
    return (nr.cpu().numpy(), nc.cpu().numpy()), (er.cpu().numpy(), ec.cpu().numpy())


def check(oracle_mod, conn, etypes, n_vert, what=""):
    print(f"[mixed] {what} n_elem={len(etypes)} n_vert={n_vert}", flush=True)
    (nr, nc), (er, ec) = gpu_mixed(conn, etypes, n_vert)
    wnr, wnc = oracle_mod.mixed_node_neighbors(conn, etypes, n_vert)
    wer, wec = oracle_mod.mixed_elem_neighbors(conn, etypes, n_vert)
    assert np.array_equal(nr, wnr), f"{what}: node row_ptr differs at {np.flatnonzero(nr != wnr)[:8]}"
    assert np.array_equal(nc, wnc), f"{what}: node cols"
    assert np.array_equal(er, wer), f"{what}: elem row_ptr"
    assert np.array_equal(ec, wec), f"{what}: elem cols"


@pytest.mark.parametrize("case", pins.read_golden("mixed_cases.txt"), ids=lambda c: c["name"])
def test_mixed_hand_cases(case):
    (nr, nc), (er, ec) = gpu_mixed(case["conn"], case["etypes"], case["n_vert"])
    assert np.array_equal(nr, case["node_row_ptr"]) and np.array_equal(nc, case["node_cols"])
    assert np.array_equal(er, case["elem_row_ptr"]) and np.array_equal(ec, case["elem_cols"])


@pytest.mark.parametrize("size", [(1, 3), (40, 14), (3000, 900), (50000, 20000), (20000, 2 ** 22 + 3)])
@pytest.mark.parametrize("types", [(0, 1, 2, 3, 4, 5), (1, 5), (2, 4), (0, 3)], ids=["all", "tet_pyr", "hex_wedge",
                                                                                   "tri_quad"])
def test_random_mixed(oracle_mod, size, types):
    m = mg.random_mixed(size[0], size[1], seed=size[0] + len(types), types=types)
    check(oracle_mod, m.conn, m.etypes, m.n_vert, m.name)


@pytest.mark.parametrize("m_cells", [1, 4, 13])
def test_hybrid_grids(oracle_mod, m_cells):
    m = mg.hybrid_grid(m_cells, seed=m_cells)
    check(oracle_mod, m.conn, m.etypes, m.n_vert, m.name)


def test_hybrid_grid_large(oracle_mod):
    m = mg.hybrid_grid(40, seed=40)  # ~240k elements
    check(oracle_mod, m.conn, m.etypes, m.n_vert, m.name)


def test_one_type_as_mixed_equals_uniform_call(oracle_mod):
    nb = _nb()
    for et, m in ((0, mg.tri_grid(60, "coin", 3)), (4, mg.wedge_grid(12, 4, 4)), (5, mg.pyramid_grid(5, 5)),
                  (3, mg.quad_grid(40, 6))):
        types = np.full(m.n_elem, et, dtype=np.uint8)
        got = gpu_mixed(m.conn.ravel(), types, m.n_vert)
        c = torch.as_tensor(m.conn).to(DEV)
        (nr, nc), (er, ec) = nb.neighbors(c, et, m.n_vert)
        assert np.array_equal(got[0][0], nr.cpu().numpy()) and np.array_equal(got[0][1], nc.cpu().numpy())
        assert np.array_equal(got[1][0], er.cpu().numpy()) and np.array_equal(got[1][1], ec.cpu().numpy())


def test_fan_of_mixed_elements_long_rows(oracle_mod):
    # vertex 0 in 6000 elements of every type: element rows far past the LDS limit
    rng = np.random.default_rng(12)
    etypes = rng.integers(0, 6, size=6000).astype(np.uint8)
    conn = []
    for i, t in enumerate(etypes):
        n = pins.NPE[int(t)]
        conn += [0] + list(1 + rng.integers(0, 3000, size=n - 1))
    check(oracle_mod, np.asarray(conn), etypes, 3001, "fan6000")


def test_malformed_elements_are_reported():
    """An unknown type code is refused on the device (INDEX_RANGE); the call
    stays in bounds."""
    nb = _nb()
    conn = np.array([0, 1, 2, 1, 2, 3], dtype=np.int32)
    elem_off = torch.as_tensor(np.array([0, 3, 6], dtype=np.int32)).to(DEV)
    etypes = torch.as_tensor(np.array([0, 9], dtype=np.uint8)).to(DEV)  # 9: no such type
    b = nb.MixedBuild(2, 6, 12, 4, DEV)
    b.launch(torch.as_tensor(conn).to(DEV), elem_off, etypes)
    with pytest.raises(nb.MeshError) as e:
        b.result()
    assert e.value.status == nb.Status.INDEX_RANGE
    # an id out of range
    with pytest.raises(nb.MeshError) as e:
        gpu_mixed(np.array([0, 1, 7]), np.array([0]), 4)
    assert e.value.status == nb.Status.INDEX_RANGE


def test_empty_mixed():
    (nr, nc), (er, ec) = gpu_mixed(np.zeros(0), np.zeros(0), 5)
    assert nr.tolist() == er.tolist() == [0] * 6 and nc.shape == ec.shape == (0,)
