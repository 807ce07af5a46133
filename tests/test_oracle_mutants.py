"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the pins catch every one of them: evidence that the pins constrain the
oracle's every part, not just its happy path."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

# (name, original text, replacement)
MUTANTS = [
    ("no_dedup", "if (lo < s->n && s->v[lo] == x) return 0;", ""),
    ("self_pairs_kept", "if (u == w) continue; /* no self pair */", ""),
    ("one_direction", "set_insert(&sets[u], w) || set_insert(&sets[w], u)", "set_insert(&sets[u], w)"),
    ("hex_edge_dropped", "*npe = 8; *n_edges = 12;", "*npe = 8; *n_edges = 11;"),
    ("hex_edge_wrong", "{2, 6}, {3, 7}}", "{2, 6}, {3, 6}}"),
    ("tet_edge_wrong", "{1, 3}, {2, 3}}", "{1, 2}, {2, 3}}"),
    ("tri_edge_dropped", "*npe = 3; *n_edges = 3;", "*npe = 3; *n_edges = 2;"),
    ("elem_id_shifted", "set_insert(&sets[el[j]], e)", "set_insert(&sets[el[j]], e + 1)"),
    ("elem_last_node_missed", "for (int j = 0; j < npe; ++j) {", "for (int j = 0; j + 1 < npe; ++j) {"),
    ("descending_insert", "if (s->v[mid] < x) lo = mid + 1; else hi = mid;",
     "if (s->v[mid] > x) lo = mid + 1; else hi = mid;"),
    ("row_ptr_shift", "row_ptr[v + 1] = (int32_t)at;", "row_ptr[v + 1] = (int32_t)at - sets[v].n;"),
    ("range_check_off_by_one", "conn[i] >= n_vert) return -2;", "conn[i] > n_vert) return -2;"),
    ("quad_diagonal", "{2, 3}, {3, 0}};", "{2, 3}, {0, 2}};"),
    ("wedge_vertical_wrong", "{1, 4}, {2, 5}};", "{1, 4}, {2, 4}};"),
    ("pyramid_apex_edge_dropped", "*npe = 5; *n_edges = 8;", "*npe = 5; *n_edges = 7;"),
    ("mixed_first_type_only", "type_info(etypes[e], &npe, &n_edges, &edges);\n        const int32_t* el",
     "type_info(etypes[0], &npe, &n_edges, &edges);\n        const int32_t* el"),
    ("mixed_ids_shifted", "const int32_t* el = conn + elem_off[e];", "const int32_t* el = conn + elem_off[e] / 2;"),
]


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    for fn in (lib.oracle_node_neighbors, lib.oracle_elem_neighbors):
        fn.restype = ctypes.c_int64
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    for fn in (lib.oracle_mixed_node_neighbors, lib.oracle_mixed_elem_neighbors):
        fn.restype = ctypes.c_int64
        fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    return lib


def _call(fn, conn, etype, n_vert):
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    n_elem = conn.shape[0]
    cap = max(1, 24 * n_elem)
    row_ptr = np.zeros(n_vert + 1, dtype=np.int32)
    cols = np.empty(cap, dtype=np.int32)
    r = fn(conn.ctypes.data, n_elem, etype, n_vert, row_ptr.ctypes.data, cols.ctypes.data, cap)
    return int(r), row_ptr, cols[:max(r, 0)]


def _call_mixed(fn, conn, etypes, n_vert):
    # a mutant that takes the wrong node count for an element reads up to 7
    # ids past its end: pad with valid ids (0) so that such a read stays in
    # bounds and the mutant shows as a wrong result, not a crash
    conn = np.concatenate([np.asarray(conn, dtype=np.int32).reshape(-1), np.zeros(8, dtype=np.int32)])
    etypes = np.ascontiguousarray(etypes, dtype=np.int32)
    off = np.zeros(etypes.shape[0] + 1, dtype=np.int64)
    np.cumsum([pins.NPE[int(t)] for t in etypes], out=off[1:])
    cap = max(1, 24 * etypes.shape[0])
    row_ptr = np.zeros(n_vert + 1, dtype=np.int32)
    cols = np.empty(cap, dtype=np.int32)
    r = fn(conn.ctypes.data, off.ctypes.data, etypes.ctypes.data, etypes.shape[0], n_vert, row_ptr.ctypes.data,
           cols.ctypes.data, cap)
    return int(r), row_ptr, cols[:max(r, 0)]


def _mixed_pins_pass(lib):
    fixtures = [(c["conn"], c["etypes"], c["n_vert"]) for c in pins.read_golden("mixed_cases.txt")]
    for seed in range(3):
        m = mg.random_mixed(30, 14, seed)
        fixtures.append((m.conn, m.etypes, m.n_vert))
    for conn, et, nv in fixtures:
        (bnr, bnc), (ber, bec) = pins.brute_force_mixed(conn, et, nv)
        r, nr, nc = _call_mixed(lib.oracle_mixed_node_neighbors, conn, et, nv)
        if r < 0 or not (np.array_equal(nr, bnr) and np.array_equal(nc, bnc)):
            return False
        r, er, ec = _call_mixed(lib.oracle_mixed_elem_neighbors, conn, et, nv)
        if r < 0 or not (np.array_equal(er, ber) and np.array_equal(ec, bec)):
            return False
    return True


def _pins_pass(lib):
    """True iff the mutant passes every pin below."""
    if not _mixed_pins_pass(lib):
        return False
    fixtures = [(c["conn"].reshape(-1, pins.NPE[c["etype"]]), c["etype"], c["n_vert"]) for c in pins.read_golden()]
    for et in (0, 1, 2, 3, 4, 5):
        m = mg.random_mesh(40, 15, et, seed=et)
        fixtures.append((m.conn, et, m.n_vert))
    for conn, et, nv in fixtures:
        (bnr, bnc), (ber, bec) = pins.brute_force(conn, et, nv)
        r, nr, nc = _call(lib.oracle_node_neighbors, conn, et, nv)
        if r < 0 or not (np.array_equal(nr, bnr) and np.array_equal(nc, bnc)):
            return False
        r, er, ec = _call(lib.oracle_elem_neighbors, conn, et, nv)
        if r < 0 or not (np.array_equal(er, ber) and np.array_equal(ec, bec)):
            return False
    # out-of-range ids must be refused
    r, _, _ = _call(lib.oracle_node_neighbors, np.array([[0, 1, 3]]), 0, 3)
    if r != -2:
        return False
    return True


def test_unmutated_passes(tmp_path):
    lib = _build(tmp_path, "identity", "#include <stdint.h>", "#include <stdint.h>")
    assert _pins_pass(lib)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    lib = _build(tmp_path, name, old, new)
    assert not _pins_pass(lib), f"mutant {name} survived the pins"
