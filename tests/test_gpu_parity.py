"""Parity of the HIP pipelines (through the C ABI) with the CPU oracle.

The relation is exact integer work with one canonical answer (ascending,
duplicate-free rows), so every comparison is bit-exact: tolerance 0."""
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


def gpu_csr(kind, conn, etype, n_vert, stream=None, options=None):
    """The CSR of one relation ("node", "elem"), or of both from one call
    ("both": a pair of CSRs), as host arrays."""
    nb = _nb()
    npe = pins.NPE[etype]
    c = torch.as_tensor(np.ascontiguousarray(conn, dtype=np.int32).reshape(-1, npe)).to(DEV)
    if kind == "both":
        (nr, nc), (er, ec) = nb.neighbors(c, etype, n_vert, stream=stream, options=options)
        return (nr.cpu().numpy(), nc.cpu().numpy()), (er.cpu().numpy(), ec.cpu().numpy())
    fn = nb.node_neighbors if kind == "node" else nb.elem_neighbors
    row_ptr, cols = fn(c, etype, n_vert, stream=stream, options=options)
    return row_ptr.cpu().numpy(), cols.cpu().numpy()


def assert_same(got, want, what=""):
    gr, gc = got
    wr, wc = want
    assert gr.shape == wr.shape, what
    assert np.array_equal(gr, wr), f"{what}: row_ptr differs at {np.flatnonzero(gr != wr)[:10]}"
    assert gc.shape == wc.shape, f"{what}: nnz {gc.shape[0]} vs {wc.shape[0]}"
    assert np.array_equal(gc, wc), f"{what}: cols differ at {np.flatnonzero(gc != wc)[:10]}"


def check_both(oracle_mod, conn, etype, n_vert, what="", options=None):
    """Node call, element call and the call building both, against the oracle."""
    print(f"[parity] {what} etype={etype} n_elem={np.asarray(conn).reshape(-1, pins.NPE[etype]).shape[0]} "
          f"n_vert={n_vert} options={options}", flush=True)
    wn = oracle_mod.node_neighbors(conn, etype, n_vert)
    we = oracle_mod.elem_neighbors(conn, etype, n_vert)
    assert_same(gpu_csr("node", conn, etype, n_vert, options=options), wn, what + " node")
    assert_same(gpu_csr("elem", conn, etype, n_vert, options=options), we, what + " elem")
    gn, ge = gpu_csr("both", conn, etype, n_vert, options=options)
    assert_same(gn, wn, what + " both/node")
    assert_same(ge, we, what + " both/elem")


# the node algorithms of the parity suites here: the full-key sort and the
# rows gathered through the element relation (the row-based sorts have their
# own suite)
NODE_SORTS = [{"node_sort": 0}, {"node_sort": 3}]
SORT_IDS = ["full_key", "elem_rows"]


@pytest.mark.parametrize("opts", [None] + NODE_SORTS, ids=["default"] + SORT_IDS)
@pytest.mark.parametrize("case", pins.read_golden(), ids=lambda c: c["name"])
def test_golden(case, opts):
    conn = case["conn"].reshape(-1, pins.NPE[case["etype"]])
    want_n = (case["node_row_ptr"], case["node_cols"])
    want_e = (case["elem_row_ptr"], case["elem_cols"])
    assert_same(gpu_csr("node", conn, case["etype"], case["n_vert"], options=opts), want_n)
    assert_same(gpu_csr("elem", conn, case["etype"], case["n_vert"], options=opts), want_e)
    gn, ge = gpu_csr("both", conn, case["etype"], case["n_vert"], options=opts)
    assert_same(gn, want_n)
    assert_same(ge, want_e)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
@pytest.mark.parametrize("etype", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("size", [(1, 1), (7, 5), (300, 90), (5000, 4000), (60000, 9000), (20000, 2 ** 20 + 7)])
def test_random_meshes(oracle_mod, etype, size, opts):
    n_elem, n_vert = size
    m = mg.random_mesh(n_elem, n_vert, etype, seed=n_elem + 7 * etype)
    check_both(oracle_mod, m.conn, etype, n_vert, m.name, opts)


@pytest.mark.parametrize("maker", [lambda: mg.tri64(), lambda: mg.tri_grid(300, "coin", 3),
                                   lambda: mg.kuhn_tet_grid(20, 4), lambda: mg.hex_grid(16, 5),
                                   lambda: mg.tri_grid(2, "main", 1), lambda: mg.kuhn_tet_grid(1, 2),
                                   lambda: mg.hex_grid(1, 3)],
                         ids=["tri64", "tri300coin", "kuhn20", "hex16", "tri2", "kuhn1", "hex1"])
@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_structured(oracle_mod, maker, opts):
    m = maker()
    check_both(oracle_mod, m.conn, m.etype, m.n_vert, m.name, opts)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_large_ids_many_passes(oracle_mod, opts):
    # ids up to 2^25: 50 key bits, 7 radix passes
    m = mg.random_mesh(30000, 2 ** 25 - 3, 1, seed=3)
    check_both(oracle_mod, m.conn, 1, m.n_vert, "ids 2^25", opts)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_fans_long_element_rows(oracle_mod, opts):
    # vertex 0 lies in n triangles: element rows of 100 (long-row list),
    # 5000 (LDS bitonic) and 9000 (in-place bitonic in global memory)
    for n in (100, 5000, 9000):
        rim = np.arange(1, n + 2, dtype=np.int32)
        conn = np.stack([np.zeros(n, np.int32), rim[:-1], rim[1:]], 1)
        conn = conn[np.random.default_rng(n).permutation(n)]
        check_both(oracle_mod, conn, 0, n + 2, f"fan{n}", opts)


def star_mesh(lengths, etype, n_unused_block, seed):
    """Stars: hub k lies in lengths[k] elements (triangles (hub, r_i, r_i+1)
    or tetrahedra (hub, r_i, r_i+1, cap) around a path of fresh rim
    vertices), so the hubs' element rows have exactly those lengths and the
    rim and cap rows are short.  Vertex ids are a random subset of a larger
    range with one block of n_unused_block unused ids in its middle (runs of
    empty rows), elements shuffled."""
    rng = np.random.default_rng(seed)
    elems, nv = [], 0
    for L in lengths:
        hub, rim = nv, np.arange(nv + 1, nv + L + 2)
        nv += L + 2
        if etype == 0:
            elems.append(np.stack([np.full(L, hub), rim[:-1], rim[1:]], 1))
        else:
            cap = nv
            nv += 1
            elems.append(np.stack([np.full(L, hub), rim[:-1], rim[1:], np.full(L, cap)], 1))
    conn = np.concatenate(elems)
    n_ids = nv + nv // 4 + n_unused_block
    lo = rng.choice(n_ids // 2 - n_unused_block // 2, size=nv // 2, replace=False)
    hi = n_ids // 2 + n_unused_block // 2 + rng.choice(n_ids - n_ids // 2 - n_unused_block // 2, size=nv - nv // 2,
                                                       replace=False)
    ids = rng.permutation(np.concatenate([lo, hi]))
    conn = ids[conn][rng.permutation(conn.shape[0])]
    return np.ascontiguousarray(conn, dtype=np.int32), int(n_ids)


@pytest.mark.parametrize("opts", [None] + NODE_SORTS, ids=["default"] + SORT_IDS)
@pytest.mark.parametrize("etype", [0, 1])
def test_node_rows_tile_layouts(oracle_mod, opts, etype):
    """Element rows of every length class the node stage treats apart, mixed
    over many tiles of element-CSR entries: short rows of 1 to 60 entries,
    rows of exactly the longest length kept in LDS (256) and one more,
    long rows of a few hundred between short ones, and a run of 1500 empty
    rows inside one tile."""
    rng = np.random.default_rng(11 + etype)
    lengths = list(rng.integers(1, 7, size=3000)) + list(rng.integers(7, 61, size=120)) + [256, 257, 255, 300, 600]
    lengths += list(rng.integers(258, 420, size=6))
    lengths = [int(x) for x in rng.permutation(np.array(lengths))]
    conn, n_vert = star_mesh(lengths, etype, 1500, seed=5 + etype)
    counts = np.bincount(conn.ravel(), minlength=n_vert)
    assert counts.max() == 600 and (counts == 256).any() and (counts == 257).any()
    check_both(oracle_mod, conn, etype, n_vert, f"star layouts type {etype}", opts)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_degenerate_and_duplicate_elements(oracle_mod, opts):
    rng = np.random.default_rng(9)
    conn = rng.integers(0, 6, size=(4000, 4)).astype(np.int32)  # many repeats per tet
    conn[::7] = conn[1::7][: conn[::7].shape[0]]                   # duplicate rows
    conn[::11, 1] = conn[::11, 0]                                   # explicit repeated ids
    check_both(oracle_mod, conn, 1, 8, "degenerate", opts)
    check_both(oracle_mod, np.zeros((50, 3), np.int32), 0, 1, "all-self tri", opts)
    # a vertex repeated at positions that share no edge: hexahedra with 2-3
    # distinct ids, and wedges and pyramids with few distinct ids
    for etype, nv in ((2, 3), (4, 3), (5, 2), (3, 2)):
        conn = rng.integers(0, nv, size=(3000, pins.NPE[etype])).astype(np.int32)
        check_both(oracle_mod, conn, etype, nv + 1, f"degenerate type {etype}", opts)


@pytest.mark.parametrize("opts", [None] + NODE_SORTS)
def test_empty_and_no_vertices(opts):
    for kind in ("node", "elem"):
        r, c = gpu_csr(kind, np.zeros((0, 3), np.int32), 0, 5, options=opts)
        assert r.tolist() == [0] * 6 and c.shape == (0,)
        r, c = gpu_csr(kind, np.zeros((0, 4), np.int32), 1, 0, options=opts)
        assert r.tolist() == [0] and c.shape == (0,)
    (nr, nc), (er, ec) = gpu_csr("both", np.zeros((0, 4), np.int32), 1, 3, options=opts)
    assert nr.tolist() == er.tolist() == [0] * 4 and nc.shape == ec.shape == (0,)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_index_range_error(opts):
    nb = _nb()
    for kind in ("node", "elem", "both"):
        with pytest.raises(nb.MeshError) as e:
            gpu_csr(kind, np.array([[0, 1, 2], [1, 2, 9]], np.int32), 0, 4, options=opts)
        assert e.value.status == nb.Status.INDEX_RANGE
        with pytest.raises(nb.MeshError) as e:
            gpu_csr(kind, np.array([[0, -1, 2]], np.int32), 0, 4, options=opts)
        assert e.value.status == nb.Status.INDEX_RANGE


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_capacity_error(opts):
    nb = _nb()
    m = mg.tri_grid(20, "main", 1)
    for kind in ("node", "elem"):
        b = nb.NeighborBuild(kind, m.n_elem, m.etype, m.n_vert, DEV, cols_capacity=100, options=opts)
        b.launch(torch.as_tensor(m.conn).to(DEV))
        with pytest.raises(nb.MeshError) as e:
            b.result()
        assert e.value.status == nb.Status.CAPACITY


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_exact_capacity_is_enough(oracle_mod, opts):
    nb = _nb()
    m = mg.kuhn_tet_grid(6, 2)
    for kind, ref in (("node", oracle_mod.node_neighbors), ("elem", oracle_mod.elem_neighbors)):
        want = ref(m.conn, m.etype, m.n_vert)
        b = nb.NeighborBuild(kind, m.n_elem, m.etype, m.n_vert, DEV, cols_capacity=want[1].shape[0], options=opts)
        b.launch(torch.as_tensor(m.conn).to(DEV))
        r, c = b.result()
        assert_same((r.cpu().numpy(), c.cpu().numpy()), want, kind)


@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_deterministic_and_workspace_reuse(opts):
    nb = _nb()
    m = mg.kuhn_tet_grid(12, 8)
    conn = torch.as_tensor(m.conn).to(DEV)
    for kind in ("node", "elem"):
        b = nb.NeighborBuild(kind, m.n_elem, m.etype, m.n_vert, DEV, options=opts)
        outs = []
        for _ in range(3):  # the same workspace, reused without clearing
            b.launch(conn)
            r, c = b.result()
            outs.append((r.cpu().numpy().copy(), c.cpu().numpy().copy()))
        for o in outs[1:]:
            assert_same(o, outs[0], kind)


def test_kernel_timing_selection(oracle_mod):
    """With timing on and a selection, only the selected launches are timed
    (and the result is the same as untimed)."""
    nb = _nb()
    m = mg.tri_grid(300, "coin", 3)
    want = oracle_mod.node_neighbors(m.conn, m.etype, m.n_vert)
    nb.timing_read()
    try:
        nb.timing_enable(True)
        nb.timing_select(["node_erows", "node_erows_gather"])
        got = gpu_csr("node", m.conn, m.etype, m.n_vert, options={"node_sort": 3})
        sel = nb.timing_read()
        nb.timing_select(None)
        gpu_csr("node", m.conn, m.etype, m.n_vert, options={"node_sort": 3})
        every = nb.timing_read()
    finally:
        nb.timing_enable(False)
        nb.timing_select(None)
    assert_same(got, want, "timed")
    assert set(sel) == {"node_erows", "node_erows_gather"} and sel["node_erows"][0] == 1
    assert {"node_erows", "node_erows_gather", "node_erows_prep", "node_erows_scan"} <= set(every)


def test_side_stream(oracle_mod):
    m = mg.hex_grid(9, 4)
    s = torch.cuda.Stream(DEV)
    with torch.cuda.stream(s):
        got = gpu_csr("node", m.conn, m.etype, m.n_vert, stream=s)
    assert_same(got, oracle_mod.node_neighbors(m.conn, m.etype, m.n_vert))


# ---- full-size workloads ---------------------------------------------------

@pytest.fixture(scope="module")
def tri2048_mesh():
    return mg.tri2048()


@pytest.fixture(scope="module")
def kuhn96_mesh():
    return mg.kuhn96()


@pytest.mark.slow
@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_full_tri2048_vs_oracle(oracle_mod, tri2048_mesh, opts):
    m = tri2048_mesh
    check_both(oracle_mod, m.conn, m.etype, m.n_vert, "tri2048 coin", opts)


@pytest.mark.slow
@pytest.mark.parametrize("opts", NODE_SORTS, ids=SORT_IDS)
def test_full_kuhn96_vs_oracle(oracle_mod, kuhn96_mesh, opts):
    m = kuhn96_mesh
    check_both(oracle_mod, m.conn, m.etype, m.n_vert, "kuhn96", opts)


@pytest.mark.slow
def test_full_kuhn96_lattice_rows(kuhn96_mesh):
    # closed-form check without the oracle: every row from lattice offsets
    m = kuhn96_mesh
    want = pins.lattice_node_csr(m.dims, pins.KUHN_STEPS, m.perm)
    for opts in NODE_SORTS:
        assert_same(gpu_csr("node", m.conn, m.etype, m.n_vert, options=opts), want, f"kuhn96 lattice {opts}")


def test_every_radix_shape_same_result(oracle_mod):
    nb = _nb()
    cases = [mg.kuhn_tet_grid(14, 3), mg.random_mesh(33333, 5000, 2, 4), mg.random_mesh(20001, 2 ** 25 - 3, 0, 5)]
    for shape in range(len(nb.radix_shapes())):
        for m in cases:
            for ns in (0, 3):
                check_both(oracle_mod, m.conn, m.etype, m.n_vert, f"{m.name} shape {nb.radix_shapes()[shape]}",
                           {"radix_shape": shape, "node_sort": ns})


@pytest.mark.slow
def test_huge_vertex_count_sparse_use(oracle_mod):
    # n_vert = 2^29 + 5: 60-bit node keys (8 radix passes); the element
    # relation sorts 30 vertex bits (4 passes) over mostly empty rows.
    # Expected CSR: the oracle on the used ids relabelled 0..k-1, expanded
    # back.
    n_vert = 2 ** 29 + 5
    rng = np.random.default_rng(17)
    used = np.unique(np.concatenate([rng.integers(0, n_vert, 3000), [0, n_vert - 1]]))
    conn_local = rng.integers(0, used.shape[0], size=(4000, 4)).astype(np.int32)
    conn = used[conn_local].astype(np.int32)
    for kind, fn in (("node", oracle_mod.node_neighbors), ("elem", oracle_mod.elem_neighbors)):
        lr, lc = fn(conn_local, 1, used.shape[0])
        if kind == "node":
            lc = used[lc].astype(np.int32)
        counts = np.zeros(n_vert, dtype=np.int64)
        counts[used] = np.diff(lr)
        want_r = np.zeros(n_vert + 1, dtype=np.int64)
        np.cumsum(counts, out=want_r[1:])
        for opts in NODE_SORTS:
            gr, gc = gpu_csr(kind, conn, 1, n_vert, options=opts)
            assert np.array_equal(gr.astype(np.int64), want_r), (kind, opts)
            assert np.array_equal(gc, lc), (kind, opts)


@pytest.mark.slow
def test_elem_past_2_30_slots_wide_status_words():
    """At 2^30 keys or more a radix pass keeps 64-bit look-back words (below,
    32-bit ones with a 30-bit count).  360 M copies of one triangle give
    1.08 G element slots with a closed-form answer: each of the three
    vertices lists every element, in order."""
    nb = _nb()
    f = 360_000_000
    assert 3 * f >= 2 ** 30
    conn = torch.tensor([0, 1, 2], dtype=torch.int32, device=DEV).repeat(f)
    rp, cols = nb.elem_neighbors(conn, 0, 3)
    del conn
    assert rp.cpu().tolist() == [0, f, 2 * f, 3 * f]
    want = torch.arange(f, dtype=torch.int32, device=DEV)
    try:
        for v in range(3):
            assert torch.equal(cols[v * f:(v + 1) * f], want), v
    finally:
        del rp, cols, want
        torch.cuda.empty_cache()
