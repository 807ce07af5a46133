"""HIP graph replays of the pipelines: each replay, with the program's own
eager work and synchronisations in between and the input contents changed in
place, gives the oracle's CSR bit for bit, the same as an eager call."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _nb():
    import paper_1604_04689_amd as nb
    return nb


def _host(rp, cols):
    return rp.cpu().numpy(), cols.cpu().numpy()


def _want(oracle_mod, kind, m):
    if kind == "both":
        return (oracle_mod.node_neighbors(m.conn, m.etype, m.n_vert),
                oracle_mod.elem_neighbors(m.conn, m.etype, m.n_vert))
    fn = oracle_mod.node_neighbors if kind == "node" else oracle_mod.elem_neighbors
    return fn(m.conn, m.etype, m.n_vert)


def _host_result(build):
    res = build.result()
    if build.kind == "both":
        return tuple(_host(*r) for r in res)
    return _host(*res)


def _same(got, want):
    if isinstance(got[0], tuple):
        return all(_same(g, w) for g, w in zip(got, want))
    return np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def _same_size_variants(kind_of_mesh):
    # two meshes of identical sizes and different contents (other seeds)
    if kind_of_mesh == "tri":
        return mg.tri_grid(150, "coin", 11), mg.tri_grid(150, "coin", 12)
    if kind_of_mesh == "tet":
        return mg.kuhn_tet_grid(20, 13), mg.kuhn_tet_grid(20, 14)
    return mg.hex_grid(18, 15), mg.hex_grid(18, 16)


@pytest.mark.parametrize("kind,mode", [("node", 0), ("node", 1), ("node", 2), ("node", 3), ("elem", -1),
                                       ("both", 3), ("both", 2)])
@pytest.mark.parametrize("family", ["tri", "tet", "hex"])
def test_single_mesh_graph_replays(oracle_mod, kind, mode, family):
    nb = _nb()
    a, b = _same_size_variants(family)
    assert (a.n_elem, a.n_vert, a.etype) == (b.n_elem, b.n_vert, b.etype)
    opts = {"node_sort": mode}
    build = nb.NeighborBuild(kind, a.n_elem, a.etype, a.n_vert, DEV, options=opts)
    conn = torch.as_tensor(a.conn).to(DEV).contiguous()
    g = build.capture(conn)
    want = {"a": _want(oracle_mod, kind, a), "b": _want(oracle_mod, kind, b)}
    other = nb.NeighborBuild(kind, b.n_elem, b.etype, b.n_vert, DEV, options=opts)
    conn_b = torch.as_tensor(b.conn).to(DEV)
    for i, which in enumerate(["a", "b", "a", "b", "b"]):
        src = a if which == "a" else b
        conn.copy_(torch.as_tensor(src.conn).to(DEV))
        g.launch()
        # the program's own eager work between replays
        other.launch(conn_b)
        s = float(conn_b.float().sum().item())
        assert s >= 0
        assert _same(_host_result(build), want[which]), f"replay {i} ({which})"
    # eager call on the same build agrees with the last replay
    build.launch(conn)
    assert _same(_host_result(build), want["b"])
    g.destroy()


def test_graph_replay_reports_and_clears_errors(oracle_mod):
    nb = _nb()
    m = mg.tri_grid(40, "coin", 21)
    build = nb.NeighborBuild("node", m.n_elem, m.etype, m.n_vert, DEV)
    good = torch.as_tensor(m.conn).to(DEV)
    conn = good.clone()
    g = build.capture(conn)
    bad = m.conn.copy()
    bad[5, 1] = m.n_vert  # out of range
    conn.copy_(torch.as_tensor(bad).to(DEV))
    g.launch()
    with pytest.raises(nb.MeshError) as e:
        build.check()
    assert e.value.status == nb.Status.INDEX_RANGE
    conn.copy_(good)
    g.launch()
    rp, cols = _host(*build.result())  # the replay cleared the error word
    wr, wc = oracle_mod.node_neighbors(m.conn, m.etype, m.n_vert)
    assert np.array_equal(rp, wr) and np.array_equal(cols, wc)
    g.destroy()


def test_graph_capture_refuses_bad_arguments():
    import ctypes
    nb = _nb()
    b = nb.binding
    m = mg.tri_grid(16, "main", 1)
    build = nb.NeighborBuild("node", m.n_elem, m.etype, m.n_vert, DEV)
    conn = torch.as_tensor(m.conn).to(DEV)
    h = ctypes.c_void_p(123)
    st = b.lib().mesh_graph_node_neighbors(b._ptr(conn), m.n_elem, m.etype, m.n_vert, b._ptr(build.row_ptr),
                                           b._ptr(build.cols), build.cols_capacity, None, b._ptr(build.workspace),
                                           build.ws_bytes - 1, ctypes.byref(h))
    assert st == nb.Status.WORKSPACE and not h.value
    assert b.lib().mesh_graph_launch(None, None) == nb.Status.INVALID_ARG
    assert b.lib().mesh_graph_destroy(None) == nb.Status.OK


@pytest.mark.parametrize("mode", [2, 3])
def test_batch_graph_replays(oracle_mod, mode):
    nb = _nb()
    rng = np.random.default_rng(5)
    specs = []
    for i in range(24):
        et = int(rng.integers(0, 6))
        specs.append((int(rng.integers(0, 3000)) if i % 7 else 0, int(rng.integers(1, 2500)), et))
    batches = [[mg.random_mesh(ne, nv, et, seed=1000 * k + i) for i, (ne, nv, et) in enumerate(specs)]
               for k in range(2)]
    desc = [(m.n_elem, m.etype, m.n_vert) for m in batches[0]]
    conns = [torch.as_tensor(nb.concat_conn([m.conn for m in ms])).to(DEV) for ms in batches]
    for kind in ("node", "elem", "both"):
        build = nb.BatchBuild(kind, desc, DEV, options={"node_sort": mode})
        conn = conns[0].clone()
        g = build.capture(conn)
        for r, k in enumerate([0, 1, 1, 0]):
            conn.copy_(conns[k])
            g.launch()
            torch.cuda.synchronize()
            res = _host_result(build)
            parts = res if kind == "both" else (res,)
            rels = ("node", "elem") if kind == "both" else (kind,)
            for rel, (rp, cols) in zip(rels, parts):
                for i, (m, seg) in enumerate(zip(batches[k], build.seg_host)):
                    v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
                    lo, hi = int(rp[v0]), int(rp[v0 + nv])
                    wr, wc = _want(oracle_mod, rel, m)
                    assert np.array_equal(rp[v0:v0 + nv + 1] - lo, wr), f"{kind}/{rel} replay {r} mesh {i} row_ptr"
                    assert np.array_equal(cols[lo:hi], wc), f"{kind}/{rel} replay {r} mesh {i} cols"
        g.destroy()
