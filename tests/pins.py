"""Independent checks used to pin the oracle (and, at full size, the HIP path).

Nothing here calls the oracle or the HIP library.  Each routine computes the
one-ring relation by a different route than the oracle's loop over elements:

* ``brute_force``     -- per vertex, scan every element (O(V*F)); hexahedron
                         edges derived from corner coordinates, not a table.
* ``scipy_csr``       -- sparse-matrix assembly (library route): node relation
                         as the pattern of A + A^T minus its diagonal, element
                         relation as the vertex-by-element incidence matrix.
* ``lattice_*``       -- closed-form neighbor sets of the structured grids from
                         lattice offsets, mapped through the seeded relabelling.
* ``read_golden``     -- hand-worked literal cases (tests/golden).
"""
from __future__ import annotations

import itertools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

NPE = {0: 3, 1: 4, 2: 8, 3: 4, 4: 6, 5: 5}

# Reference cells (VTK node orders) as coordinates.
REF_COORDS = {
    0: [(0, 0), (1, 0), (0, 1)],
    1: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
    3: [(0, 0), (1, 0), (1, 1), (0, 1)],
    4: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)],
    5: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0.5, 0.5, 1)],
}
# VTK hexahedron corner coordinates (unit cube).
_HEX_CORNERS = REF_COORDS[2]


def hull_edges(coords):
    """Edges of the convex polytope with the given corners, from geometry
    alone.  In the plane: a pair is an edge when every other corner lies on
    one side of the line through it.  In space: a facet is a plane through
    three corners with every corner on one side (or on it); a pair is an edge
    when two different facets contain it."""
    x = np.asarray(coords, dtype=np.float64)
    n, d = x.shape
    out = []
    if d == 2:
        for a, b in itertools.combinations(range(n), 2):
            t = x[b] - x[a]
            side = [t[0] * (x[c] - x[a])[1] - t[1] * (x[c] - x[a])[0] for c in range(n) if c not in (a, b)]
            if all(v > 1e-12 for v in side) or all(v < -1e-12 for v in side):
                out.append((a, b))
        return out
    facets = set()
    for tri in itertools.combinations(range(n), 3):
        nrm = np.cross(x[tri[1]] - x[tri[0]], x[tri[2]] - x[tri[0]])
        if np.linalg.norm(nrm) < 1e-12:
            continue
        h = (x - x[tri[0]]) @ nrm
        if np.all(h <= 1e-12) or np.all(h >= -1e-12):
            facets.add(frozenset(int(i) for i in np.flatnonzero(np.abs(h) <= 1e-12)))
    for a, b in itertools.combinations(range(n), 2):
        if sum(1 for f in facets if a in f and b in f) >= 2:
            out.append((a, b))
    return out


def edge_pairs(etype: int):
    """Node-position pairs joined by an element edge, derived from the
    reference cell's geometry (its convex hull), not from a table."""
    return hull_edges(REF_COORDS[etype])


def hex_edges_by_axis():
    """The cube's edges a second way: corner pairs that differ in exactly one
    coordinate."""
    out = []
    for a, b in itertools.combinations(range(8), 2):
        if sum(x != y for x, y in zip(_HEX_CORNERS[a], _HEX_CORNERS[b])) == 1:
            out.append((a, b))
    return out


def _to_csr(rows):
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int32)
    for v, r in enumerate(rows):
        row_ptr[v + 1] = row_ptr[v] + len(r)
    cols = np.array([x for r in rows for x in r], dtype=np.int32)
    return row_ptr, cols


def brute_force(conn, etype, n_vert):
    """(node_csr, elem_csr) by scanning all elements for each vertex."""
    conn = np.asarray(conn).reshape(-1, NPE[etype]).tolist()
    pairs = edge_pairs(etype)
    node_rows, elem_rows = [], []
    for v in range(n_vert):
        nb, el = set(), set()
        for e, row in enumerate(conn):
            if v in row:
                el.add(e)
            for i, j in pairs:
                if row[i] == v and row[j] != v:
                    nb.add(row[j])
                if row[j] == v and row[i] != v:
                    nb.add(row[i])
        node_rows.append(sorted(nb))
        elem_rows.append(sorted(el))
    return _to_csr(node_rows), _to_csr(elem_rows)


def _mixed_elements(conn, etypes):
    conn = np.asarray(conn).ravel().tolist()
    out, at = [], 0
    for t in np.asarray(etypes).ravel().tolist():
        out.append((int(t), conn[at:at + NPE[int(t)]]))
        at += NPE[int(t)]
    assert at == len(conn)
    return out


def brute_force_mixed(conn, etypes, n_vert):
    """(node_csr, elem_csr) of a mesh with one type per element, by scanning
    all elements for each vertex, each with its own type's edges."""
    elems = _mixed_elements(conn, etypes)
    pairs = {t: edge_pairs(t) for t in NPE}
    node_rows, elem_rows = [], []
    for v in range(n_vert):
        nb, el = set(), set()
        for e, (t, row) in enumerate(elems):
            if v in row:
                el.add(e)
            for i, j in pairs[t]:
                if row[i] == v and row[j] != v:
                    nb.add(row[j])
                if row[j] == v and row[i] != v:
                    nb.add(row[i])
        node_rows.append(sorted(nb))
        elem_rows.append(sorted(el))
    return _to_csr(node_rows), _to_csr(elem_rows)


def scipy_mixed(conn, etypes, n_vert):
    """(node_csr, elem_csr) of a mixed mesh by sparse assembly."""
    import scipy.sparse as sp

    elems = _mixed_elements(conn, etypes)
    u, w, vv, ee = [], [], [], []
    for e, (t, row) in enumerate(elems):
        for i, j in edge_pairs(t):
            u.append(row[i])
            w.append(row[j])
        vv += row
        ee += [e] * len(row)
    a = sp.coo_matrix((np.ones(len(u)), (np.asarray(u, dtype=np.int64), np.asarray(w, dtype=np.int64))),
                      shape=(n_vert, n_vert)).tocsr()
    a = (a + a.T).tocsr()
    a.setdiag(0)
    a.eliminate_zeros()
    a.sort_indices()
    b = sp.coo_matrix((np.ones(len(vv)), (np.asarray(vv, dtype=np.int64), np.asarray(ee, dtype=np.int64))),
                      shape=(n_vert, len(elems))).tocsr()
    b.sum_duplicates()
    b.sort_indices()
    return ((a.indptr.astype(np.int32), a.indices.astype(np.int32)),
            (b.indptr.astype(np.int32), b.indices.astype(np.int32)))


def scipy_csr(conn, etype, n_vert):
    """(node_csr, elem_csr) via scipy.sparse assembly and canonicalisation."""
    import scipy.sparse as sp

    conn = np.asarray(conn, dtype=np.int64).reshape(-1, NPE[etype])
    f = conn.shape[0]
    pairs = edge_pairs(etype)
    if f and pairs:
        u = np.concatenate([conn[:, i] for i, _ in pairs])
        w = np.concatenate([conn[:, j] for _, j in pairs])
    else:
        u = w = np.zeros(0, dtype=np.int64)
    a = sp.coo_matrix((np.ones(u.shape[0]), (u, w)), shape=(n_vert, n_vert)).tocsr()
    a = (a + a.T).tocsr()
    a.setdiag(0)
    a.eliminate_zeros()
    a.sort_indices()
    node = (a.indptr.astype(np.int32), a.indices.astype(np.int32))
    vv = conn.ravel()
    ee = np.repeat(np.arange(f), conn.shape[1])
    b = sp.coo_matrix((np.ones(vv.shape[0]), (vv, ee)), shape=(n_vert, f)).tocsr()
    b.sum_duplicates()
    b.sort_indices()
    elem = (b.indptr.astype(np.int32), b.indices.astype(np.int32))
    return node, elem


# ---------------------------------------------------------------------------
# Closed-form lattice neighbor sets
# ---------------------------------------------------------------------------

TRI_MAIN_STEPS = [(1, 0), (0, 1), (1, 1)]          # grid edges plus main diagonal
KUHN_STEPS = [s for s in itertools.product((0, 1), repeat=3) if any(s)]
HEX_STEPS = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
QUAD_STEPS = [(1, 0), (0, 1)]
WEDGE_STEPS = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1)]  # main-diagonal triangles, extruded


def lattice_node_csr(dims, steps, perm):
    """Node CSR of a lattice whose edges are the +/- ``steps`` offsets.

    Lattice point p (row-major over ``dims``) is adjacent to p +/- s for every
    s in ``steps`` that stays inside the grid.  The result is expressed in the
    relabelled ids ``perm[p]`` with ascending rows.
    """
    dims = tuple(dims)
    nd = len(dims)
    n = int(np.prod(dims))
    coords = np.stack(np.unravel_index(np.arange(n), dims), 1)
    src, dst = [], []
    for s in steps:
        for sign in (1, -1):
            q = coords + sign * np.asarray(s)
            ok = np.all((q >= 0) & (q < np.asarray(dims)), axis=1)
            qi = np.ravel_multi_index(tuple(q[ok].T), dims) if nd else q
            src.append(perm[np.arange(n)[ok]])
            dst.append(perm[qi])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), dst.astype(np.int32)


def kuhn_edge_count(m):
    """Edges of the Kuhn triangulation of an m^3 cube: one per lattice step
    s in {0,1}^3 minus 0 and start point with the step inside the cube."""
    return 3 * m * (m + 1) ** 2 + 3 * m ** 2 * (m + 1) + m ** 3


def tri_grid_edge_count(n):
    """Edges of an n x n vertex grid with one diagonal per cell."""
    return 2 * n * (n - 1) + (n - 1) ** 2


def hex_edge_count(m):
    return 3 * m * (m + 1) ** 2


# ---------------------------------------------------------------------------
# Golden fixtures
# ---------------------------------------------------------------------------

def read_golden(name="hand_cases.txt"):
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest.strip()}
            elif key == "end":
                cases.append(cur)
                cur = None
            else:
                vals = [int(x) for x in rest.split()]
                cur[key] = vals[0] if key in ("etype", "n_vert") else np.array(vals, dtype=np.int32)
    return cases


# ---------------------------------------------------------------------------
# Invariant checks on any (node_csr, elem_csr) pair
# ---------------------------------------------------------------------------

def check_csr_shape(row_ptr, cols, n_vert):
    assert row_ptr.shape == (n_vert + 1,)
    assert row_ptr[0] == 0
    assert np.all(np.diff(row_ptr.astype(np.int64)) >= 0)
    assert row_ptr[-1] == cols.shape[0]


def rows_strictly_increasing(row_ptr, cols):
    if cols.shape[0] < 2:
        return True
    d = np.diff(cols.astype(np.int64))
    # positions where a new row starts are exempt
    starts = np.zeros(cols.shape[0], dtype=bool)
    starts[row_ptr[:-1][row_ptr[:-1] < cols.shape[0]]] = True
    return bool(np.all((d > 0) | starts[1:]))


def row_ids(row_ptr):
    return np.repeat(np.arange(row_ptr.shape[0] - 1), np.diff(row_ptr.astype(np.int64)))


def is_symmetric(row_ptr, cols):
    r = row_ids(row_ptr).astype(np.int64)
    c = cols.astype(np.int64)
    n = row_ptr.shape[0] - 1
    a = np.sort(r * n + c)
    b = np.sort(c * n + r)
    return np.array_equal(a, b)
