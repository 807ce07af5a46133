"""Batched builds: every mesh's slice of the batch result equals the oracle
(and the single-mesh call) on that mesh alone, bit for bit."""
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


@pytest.fixture(autouse=True, params=[0, 1, 2], ids=["full_key", "vertex_rows", "edge_rows"])
def node_sort(request):
    """Every batch test runs under every node algorithm (process-wide)."""
    nb = _nb()
    nb.set_node_sort(request.param)
    yield request.param
    nb.set_node_sort(0)


def run_batch(meshes):
    nb = _nb()
    desc = [(m.n_elem, m.etype, m.n_vert) for m in meshes]
    conn = torch.as_tensor(nb.concat_conn([m.conn for m in meshes])).to(DEV)
    out = {}
    for kind in ("node", "elem"):
        b = nb.BatchBuild(kind, desc, DEV)
        b.launch(conn)
        rp, cols = b.result()
        rp_h = rp.cpu().numpy()
        cols_h = cols.cpu().numpy()
        slices = []
        for i, seg in enumerate(b.seg_host):
            v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
            a, c = int(rp_h[v0]), int(rp_h[v0 + nv])
            slices.append((rp_h[v0:v0 + nv + 1] - a, cols_h[a:c]))
        out[kind] = slices
    return out


def check_slices(oracle_mod, meshes, got, only=None):
    for i, m in enumerate(meshes):
        if only is not None and i not in only:
            continue
        for kind, fn in (("node", oracle_mod.node_neighbors), ("elem", oracle_mod.elem_neighbors)):
            wr, wc = fn(m.conn, m.etype, m.n_vert)
            gr, gc = got[kind][i]
            assert np.array_equal(gr, wr), f"mesh {i} ({m.name}) {kind} row_ptr"
            assert np.array_equal(gc, wc), f"mesh {i} ({m.name}) {kind} cols"


def test_mixed_random_batch(oracle_mod):
    rng = np.random.default_rng(77)
    meshes = []
    for i in range(40):
        et = int(rng.integers(0, 3))
        nv = int(rng.integers(1, 3000))
        ne = int(rng.integers(0, 4000)) if i % 9 else 0  # some empty meshes
        meshes.append(mg.random_mesh(ne, nv, et, seed=100 + i))
    got = run_batch(meshes)
    check_slices(oracle_mod, meshes, got)


def test_structured_small_batch(oracle_mod):
    specs = mg.batch_specs(n_mesh=48, seed=5, tri_range=(4, 60), cell_range=(1, 9))
    meshes = [s.build() for s in specs]
    got = run_batch(meshes)
    check_slices(oracle_mod, meshes, got)


def test_batch_with_long_rows(oracle_mod):
    # few vertices, many elements: rows of hundreds to thousands of pairs
    meshes = [mg.random_mesh(3000, 40, 1, seed=51), mg.tri_grid(30, "coin", 52),
              mg.random_mesh(9000, 7, 2, seed=53), mg.random_mesh(400, 300, 0, seed=54)]
    got = run_batch(meshes)
    check_slices(oracle_mod, meshes, got)


def test_batch_with_gapped_and_reordered_conn(oracle_mod):
    """Meshes placed in the connectivity with gaps and out of order: tiles
    across meshes whose ids are not contiguous must take the per-key path,
    the contiguous ones the staged path, and both give the oracle's rows."""
    nb = _nb()
    rng = np.random.default_rng(91)
    meshes = [mg.random_mesh(int(rng.integers(50, 1500)), int(rng.integers(20, 600)), i % 3, seed=300 + i)
              for i in range(30)]
    # layout: meshes back to back except a few gaps, and meshes 10..12 stored in reverse order
    order = list(range(30))
    order[10:13] = [12, 11, 10]
    offs = [0] * 30
    pos = 0
    parts = []
    for j, i in enumerate(order):
        if j % 7 == 3:  # a gap of junk ids
            parts.append(np.full(5, 2 ** 30, dtype=np.int32))
            pos += 5
        offs[i] = pos
        parts.append(meshes[i].conn.reshape(-1))
        pos += meshes[i].conn.size
    conn = torch.as_tensor(np.concatenate(parts).astype(np.int32)).to(DEV)
    desc = [(m.n_elem, m.etype, m.n_vert) for m in meshes]
    got = {}
    for kind in ("node", "elem"):
        b = nb.BatchBuild(kind, desc, DEV, conn_offs=offs)
        b.launch(conn)
        rp, cols = b.result()
        rp_h, cols_h = rp.cpu().numpy(), cols.cpu().numpy()
        got[kind] = []
        for seg in b.seg_host:
            v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
            a, c = int(rp_h[v0]), int(rp_h[v0 + nv])
            got[kind].append((rp_h[v0:v0 + nv + 1] - a, cols_h[a:c]))
    check_slices(oracle_mod, meshes, got)


def test_batch_every_radix_shape_same_result(oracle_mod):
    """Every tile shape (each has its own tile table and histogram tiling)
    gives the same bytes as the default one, and the oracle's rows."""
    nb = _nb()
    specs = mg.batch_specs(n_mesh=24, seed=11, tri_range=(4, 90), cell_range=(1, 12))
    meshes = [s.build() for s in specs]
    ref = run_batch(meshes)
    check_slices(oracle_mod, meshes, ref)
    try:
        for shape in range(1, len(nb.radix_shapes())):
            nb.set_radix_shape(shape)
            got = run_batch(meshes)
            for kind in ("node", "elem"):
                for i in range(len(meshes)):
                    assert np.array_equal(got[kind][i][0], ref[kind][i][0]), (shape, kind, i)
                    assert np.array_equal(got[kind][i][1], ref[kind][i][1]), (shape, kind, i)
    finally:
        nb.set_radix_shape(0)


def test_single_mesh_batch_equals_single_call(oracle_mod):
    m = mg.kuhn_tet_grid(9, 3)
    got = run_batch([m])
    check_slices(oracle_mod, [m], got)


def test_batch_bad_id_is_reported():
    nb = _nb()
    a = mg.tri_grid(5, "main", 1)
    bad = mg.tri_grid(4, "main", 2)
    bad.conn[3, 1] = bad.n_vert  # outside its own mesh (valid in the batch's global range)
    desc = [(a.n_elem, 0, a.n_vert), (bad.n_elem, 0, bad.n_vert)]
    conn = torch.as_tensor(nb.concat_conn([a.conn, bad.conn])).to(DEV)
    for kind in ("node", "elem"):
        b = nb.BatchBuild(kind, desc, DEV)
        b.launch(conn)
        with pytest.raises(nb.MeshError) as e:
            b.result()
        assert e.value.status == nb.Status.INDEX_RANGE


@pytest.mark.slow
def test_full_batch_512(oracle_mod):
    nb = _nb()
    specs = mg.batch_specs()
    meshes = [s.build() for s in specs]
    got = run_batch(meshes)
    # every slice equals the single-mesh GPU call; a sample also the oracle
    for i in range(0, len(meshes), 37):
        m = meshes[i]
        c = torch.as_tensor(m.conn).to(DEV)
        for kind, fn in (("node", nb.node_neighbors), ("elem", nb.elem_neighbors)):
            r, cc = fn(c, m.etype, m.n_vert)
            assert np.array_equal(got[kind][i][0], r.cpu().numpy()), (i, kind)
            assert np.array_equal(got[kind][i][1], cc.cpu().numpy()), (i, kind)
    sample = set(range(0, len(meshes), 23))
    small = {i for i in sample if meshes[i].n_elem < 400000}
    check_slices(oracle_mod, meshes, got, only=small)
    # totals: every mesh of the batch, by closed form
    for kind in ("node", "elem"):
        for i, m in enumerate(meshes):
            nnz = got[kind][i][1].shape[0]
            if kind == "elem":
                assert nnz == m.npe * m.n_elem
            elif m.etype == 0:
                assert nnz == 2 * (m.n_vert + m.n_elem - 1)
            elif m.etype == 1:
                assert nnz == 2 * pins.kuhn_edge_count(round((m.n_vert) ** (1 / 3)) - 1)
            else:
                assert nnz == 2 * pins.hex_edge_count(round((m.n_vert) ** (1 / 3)) - 1)
