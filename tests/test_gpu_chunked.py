"""Parity of the bounded-memory build (mesh_options.chunk_keys) against the
CPU oracle, through the C ABI.  Both relations are exact integer work with
one canonical answer: bit-exact, tolerance 0.

A small pair budget cuts the vertices into many ranges, each sorted on its
own.  The cases cover every element type, ragged last ranges, budgets that
are not powers of two, vertices used by no element (ranges without pairs),
degenerate elements, a vertex whose bin holds more pairs than the budget
(MESH_ERR_CHUNK), ids out of range (MESH_ERR_INDEX_RANGE), the no-allocation
entry point, and byte equality with the whole-mesh build on large grids."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests.test_gpu_parity import assert_same, check_both, gpu_csr

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("etype", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("n_vert,cap", [(300, 4096), (5000, 6151), (70_000, 4096), (3_000_000, 65_536)])
def test_chunked_random(oracle_mod, etype, n_vert, cap):
    """Random connectivity (degenerate and duplicate elements, unused
    vertices): from about 20 ranges (4096 pairs each) to one."""
    n_elem = 25_013 if etype != 2 else 9_001
    m = mg.random_mesh(n_elem, n_vert, etype, seed=900 + etype + n_vert % 89)
    check_both(oracle_mod, m.conn, etype, n_vert, f"chunked cap={cap}", options={"chunk_keys": cap})


@pytest.mark.parametrize("cap", [4096, 10_007])
def test_chunked_grids(oracle_mod, cap):
    """Structured meshes: a coin-flip triangle grid and a Kuhn tetrahedral
    grid, ranges cut inside their vertex order."""
    for m in (mg.tri_grid(96, "coin", 3), mg.kuhn_tet_grid(14, 5), mg.hex_grid(16, 4)):
        check_both(oracle_mod, m.conn, m.etype, m.n_vert, f"chunked {m.name} cap={cap}",
                   options={"chunk_keys": cap})


def test_chunked_unused_vertex_spans(oracle_mod):
    """Ids drawn from two narrow windows of 2^20 vertices (bins of 512
    vertices, about 2300 pairs each inside the windows): the bins between
    them hold no pairs, and the vertex bound (at most chunk_keys vertices
    per range) cuts that span into ranges with no pairs at all."""
    rng = np.random.default_rng(5)
    n_vert = 1 << 20
    a = rng.integers(0, 1000, size=(1500, 3))
    b = rng.integers(500_000, 501_000, size=(1500, 3))
    conn = np.concatenate([a, b]).astype(np.int32)
    check_both(oracle_mod, conn, 0, n_vert, "chunked unused spans", options={"chunk_keys": 4096})


def test_chunked_hub_vertex(oracle_mod):
    """A fan of 5000 triangles around vertex 0: its element row alone holds
    5000 pairs.  A budget below that is refused (MESH_ERR_CHUNK, after the
    histogram); one above it gives the oracle's rows."""
    from paper_1604_04689_amd import binding as nb
    k = 5000
    conn = np.stack([np.zeros(k), np.arange(1, k + 1), np.arange(2, k + 2)], axis=1).astype(np.int32)
    n_vert = k + 2
    with pytest.raises(nb.MeshError) as e:
        gpu_csr("elem", conn, 0, n_vert, options={"chunk_keys": 4096})
    assert e.value.status == nb.Status.CHUNK
    check_both(oracle_mod, conn, 0, n_vert, "chunked hub", options={"chunk_keys": 8192})


def test_chunked_index_range_reported():
    from paper_1604_04689_amd import binding as nb
    rng = np.random.default_rng(9)
    conn = rng.integers(0, 20_000, size=(20_000, 4)).astype(np.int32)
    conn[777, 2] = 20_000  # one past the last vertex
    for kind in ("node", "elem", "both"):
        with pytest.raises(nb.MeshError) as e:
            gpu_csr(kind, conn, 1, 20_000, options={"chunk_keys": 4096})
        assert e.value.status == nb.Status.INDEX_RANGE, kind


def test_chunked_equals_whole_mesh_build():
    """A 1024^2 coin-flip triangle grid (about 2.1 M triangles) and a 48^3
    Kuhn grid (about 660 K tetrahedra): a 2^18-pair budget gives the bytes of
    the whole-mesh build."""
    for m in (mg.tri_grid(1024, "coin", 41), mg.kuhn_tet_grid(48, 4)):
        print(f"[chunked] {m.name} n_elem={m.n_elem}", flush=True)
        whole = gpu_csr("both", m.conn, m.etype, m.n_vert)
        part = gpu_csr("both", m.conn, m.etype, m.n_vert, options={"chunk_keys": 1 << 18})
        for (a, b), rel in zip(zip(part, whole), ("node", "elem")):
            assert_same(a, b, f"chunked vs whole {m.name} {rel}")
        node_only = gpu_csr("node", m.conn, m.etype, m.n_vert, options={"chunk_keys": 1 << 18})
        assert_same(node_only, whole[0], f"chunked node-only {m.name}")


def test_chunked_noalloc(oracle_mod):
    """mesh_neighbors_noalloc under a pair budget on a mesh whose whole-mesh
    workspace exceeds the fixed scratch: twice in a row (the scratch keeps
    the first call's contents), the second call on a smaller mesh."""
    from paper_1604_04689_amd import binding as nb
    dev = torch.device("cuda:0")
    opts = {"chunk_keys": 1 << 18}
    for n in (1100, 300):
        m = mg.tri_grid(n, "coin", 17)
        assert n < 1000 or nb.query("both", m.n_elem, 0, m.n_vert)[0] > nb.NOALLOC_SCRATCH_BYTES
        _, ncap, ecap = nb.query("both", m.n_elem, 0, m.n_vert, opts)
        out = (torch.empty(m.n_vert + 1, dtype=torch.int32, device=dev), torch.empty(ncap, dtype=torch.int32, device=dev),
               torch.empty(m.n_vert + 1, dtype=torch.int32, device=dev), torch.empty(ecap, dtype=torch.int32, device=dev))
        print(f"[chunked] noalloc {m.name} n_elem={m.n_elem}", flush=True)
        c = torch.as_tensor(m.conn).to(dev)
        (nr, nc), (er, ec) = nb.neighbors_noalloc(c, 0, m.n_vert, out, options=opts)
        whole = gpu_csr("both", m.conn, 0, m.n_vert)
        assert_same((nr.cpu().numpy(), nc.cpu().numpy()), whole[0], "noalloc chunked node")
        assert_same((er.cpu().numpy(), ec.cpu().numpy()), whole[1], "noalloc chunked elem")
        if n == 300:
            assert_same(whole[0], oracle_mod.node_neighbors(m.conn, 0, m.n_vert), "noalloc chunked vs oracle")


def test_chunked_unaligned_connectivity(oracle_mod):
    """A connectivity that starts 4 bytes past an aligned address (a view of
    a larger buffer) gives the oracle's rows under a pair budget."""
    from paper_1604_04689_amd import binding as nb
    dev = torch.device("cuda:0")
    m = mg.random_mesh(30_011, 9_000, 0, seed=77)
    flat = torch.as_tensor(np.ascontiguousarray(m.conn, dtype=np.int32).reshape(-1))
    buf = torch.zeros(flat.numel() + 1, dtype=torch.int32, device=dev)
    buf[1:] = flat.to(dev)
    c = buf[1:].view(-1, 3)
    assert c.data_ptr() % 16 == 4
    print("[chunked] unaligned conn", flush=True)
    got = nb.neighbors(c, 0, m.n_vert, options={"chunk_keys": 4096})
    want_n = oracle_mod.node_neighbors(m.conn, 0, m.n_vert)
    want_e = oracle_mod.elem_neighbors(m.conn, 0, m.n_vert)
    assert_same((got[0][0].cpu().numpy(), got[0][1].cpu().numpy()), want_n, "unaligned chunked node")
    assert_same((got[1][0].cpu().numpy(), got[1][1].cpu().numpy()), want_e, "unaligned chunked elem")
