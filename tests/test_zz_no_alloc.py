"""mesh_neighbors_noalloc (no workspace: the library's fixed scratch array)
against mesh_neighbors with a caller workspace, through the C ABI.

Both relations are exact integer work with one canonical answer, so the
comparison is bit-exact (tolerance 0).  Two calls in a row share the scratch:
the second, on a smaller mesh, must not see anything the first left behind."""
import ctypes

import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _with_workspace(m, options=None):
    import paper_1604_04689_amd as nb
    conn = torch.as_tensor(m.conn).to(DEV)
    (nr, nc), (er, ec) = nb.neighbors(conn, m.etype, m.n_vert, options=options)
    return (nr.cpu().numpy(), nc.cpu().numpy()), (er.cpu().numpy(), ec.cpu().numpy())


def _noalloc(m, options=None, poison=True):
    import paper_1604_04689_amd as nb
    conn = torch.as_tensor(m.conn).to(DEV)
    _, ncap, ecap = nb.query("both", m.n_elem, m.etype, m.n_vert, options)
    # outputs pre-filled with junk, so nothing stale can pass for a result
    fill = -7 if poison else 0
    out = (torch.full((m.n_vert + 1,), fill, dtype=torch.int32, device=DEV),
           torch.full((max(ncap, 1),), fill, dtype=torch.int32, device=DEV),
           torch.full((m.n_vert + 1,), fill, dtype=torch.int32, device=DEV),
           torch.full((max(ecap, 1),), fill, dtype=torch.int32, device=DEV))
    (nr, nc), (er, ec) = nb.neighbors_noalloc(conn, m.etype, m.n_vert, out, options=options)
    return (nr.cpu().numpy(), nc.cpu().numpy()), (er.cpu().numpy(), ec.cpu().numpy())


def _same(got, want, what):
    for (gr, gc), (wr, wc), rel in zip(got, want, ("node", "elem")):
        assert np.array_equal(gr, wr), f"{what} {rel}: row_ptr differs at {np.flatnonzero(gr != wr)[:10]}"
        assert gc.shape == wc.shape and np.array_equal(gc, wc), f"{what} {rel}: cols differ"


def test_noalloc_matches_workspace_call_twice_shrinking():
    big = mg.kuhn_tet_grid(40, seed=11)       # 384,000 tets, 68,921 vertices
    small = mg.tri_grid(33, diag="coin", seed=12)
    for m in (big, small):
        print(f"[noalloc] {m.name} n_elem={m.n_elem} n_vert={m.n_vert}", flush=True)
        _same(_noalloc(m), _with_workspace(m), m.name)


def test_noalloc_every_node_algorithm():
    m = mg.random_mesh(5000, 1700, 2, seed=21)  # hexahedra with repeated ids and unused vertices
    for ns in (0, 1, 2, 3):
        print(f"[noalloc] random hex node_sort={ns}", flush=True)
        _same(_noalloc(m, {"node_sort": ns}), _with_workspace(m, {"node_sort": ns}), f"node_sort {ns}")


def test_noalloc_error_word_then_clean_call():
    """An id outside [0, n_vert) is reported by mesh_check(NULL); the next
    call on the same scratch starts clean."""
    import paper_1604_04689_amd as nb
    m = mg.tri_grid(20, seed=5)
    bad = m.conn.copy()
    bad[3, 1] = m.n_vert + 4
    conn = torch.as_tensor(bad).to(DEV)
    _, ncap, ecap = nb.query("both", m.n_elem, m.etype, m.n_vert)
    out = (torch.empty(m.n_vert + 1, dtype=torch.int32, device=DEV), torch.empty(ncap, dtype=torch.int32, device=DEV),
           torch.empty(m.n_vert + 1, dtype=torch.int32, device=DEV), torch.empty(ecap, dtype=torch.int32, device=DEV))
    with pytest.raises(nb.MeshError) as e:
        nb.neighbors_noalloc(conn, m.etype, m.n_vert, out)
    assert e.value.status == nb.Status.INDEX_RANGE
    _same(_noalloc(m), _with_workspace(m), "after an error")


def test_noalloc_refuses_meshes_past_the_scratch():
    import paper_1604_04689_amd as nb
    m = mg.tri_grid(1200, seed=3)  # 2.9 M triangles: workspace above 64 MiB
    ws, ncap, ecap = nb.query("both", m.n_elem, m.etype, m.n_vert)
    assert ws > nb.binding.NOALLOC_SCRATCH_BYTES
    conn = torch.as_tensor(m.conn).to(DEV)
    out = (torch.empty(m.n_vert + 1, dtype=torch.int32, device=DEV), torch.empty(ncap, dtype=torch.int32, device=DEV),
           torch.empty(m.n_vert + 1, dtype=torch.int32, device=DEV), torch.empty(ecap, dtype=torch.int32, device=DEV))
    with pytest.raises(nb.MeshError) as e:
        nb.neighbors_noalloc(conn, m.etype, m.n_vert, out)
    assert e.value.status == nb.Status.SCRATCH_LIMIT
    # and the scratch is still usable afterwards
    s = mg.tri64()
    _same(_noalloc(s), _with_workspace(s), "after a refusal")
