"""Seeded generators: exact sizes, determinism, valid relabelling."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg


def test_small_workload_sizes():
    m = mg.tri64()
    assert (m.n_elem, m.n_vert, m.npe) == (7938, 4096, 3)
    assert m.conn.dtype == np.int32 and m.conn.flags["C_CONTIGUOUS"]


@pytest.mark.parametrize("spec", [(mg.TRI3, 2048), (mg.TET4, 96), (mg.HEX8, 10)])
def test_closed_form_sizes(spec):
    s = mg.MeshSpec(spec[0], spec[1], 1)
    expect = {(0, 2048): (8380418, 4194304), (1, 96): (5308416, 912673), (2, 10): (1000, 1331)}
    assert (s.n_elem, s.n_vert) == expect[spec]


def test_determinism_and_relabel():
    a = mg.kuhn_tet_grid(6, seed=11)
    b = mg.kuhn_tet_grid(6, seed=11)
    c = mg.kuhn_tet_grid(6, seed=12)
    assert np.array_equal(a.conn, b.conn)
    assert not np.array_equal(a.conn, c.conn)
    assert np.array_equal(np.sort(a.perm), np.arange(a.n_vert))
    assert np.array_equal(np.sort(a.elem_order), np.arange(a.n_elem))
    assert a.conn.min() >= 0 and a.conn.max() < a.n_vert
    # every vertex is used by a structured grid
    assert np.unique(a.conn).shape[0] == a.n_vert


def test_unrelabelled_lattice_ids():
    m = mg.tri_grid(3, "main", relabel=False, shuffle=False)
    # cell (0,0): (0,1,4) and (0,4,3)
    assert m.conn[0].tolist() == [0, 1, 4] and m.conn[1].tolist() == [0, 4, 3]
    h = mg.hex_grid(1, relabel=False, shuffle=False)
    # VTK order on the unit cube, id = (x*2 + y)*2 + z
    assert h.conn[0].tolist() == [0, 4, 6, 2, 1, 5, 7, 3]


def test_batch_draw():
    specs = mg.batch_specs()
    assert len(specs) == 512
    kinds = {s.etype for s in specs}
    assert kinds == {0, 1, 2}
    assert all(8 <= s.size <= 512 for s in specs if s.etype == 0)
    assert all(4 <= s.size <= 48 for s in specs if s.etype != 0)
    assert specs[0].seed == mg.batch_specs()[0].seed
