"""Seeded synthetic mesh generators.

This module only builds input connectivity: it computes no neighbor relation
and shares nothing with either the HIP path or the CPU oracle, both of which
consume its arrays.  Every generator returns int32 connectivity, row-major
``[n_elem, nodes_per_element]``, with vertex ids relabelled by a seeded random
permutation and element rows shuffled by a second seeded permutation, so that
every radix digit of a neighbor key is uniform and every scatter is random.

Element types (VTK node orders):

* ``TRI3`` (0): 3 nodes.
* ``TET4`` (1): 4 nodes.
* ``HEX8`` (2): 8 nodes, nodes 0-3 the bottom face counter-clockwise and
  nodes 4-7 the top face above them.
* ``QUAD4`` (3): 4 nodes around the face.
* ``WEDGE6`` (4): triangle 0-1-2 and triangle 3-4-5 above it.
* ``PYRAMID5`` (5): quadrilateral base 0-1-2-3 and apex 4.

Meshes with several element types (``MixedMesh``) hold every element's ids
back to back with one type code per element.

The paper measures on scanned triangle surfaces (Stanford 3D Scanning
Repository, GIT Large Geometry Models Archive; Sec. 3.1, Table 1).  Those
meshes are not used: structured and coin-flip triangle grids with the same
F/V ratio (about 2) and mean valence (6) stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TRI3, TET4, HEX8, QUAD4, WEDGE6, PYRAMID5 = 0, 1, 2, 3, 4, 5
NODES_PER_ELEM = {TRI3: 3, TET4: 4, HEX8: 8, QUAD4: 4, WEDGE6: 6, PYRAMID5: 5}
TYPE_NAMES = {TRI3: "tri3", TET4: "tet4", HEX8: "hex8", QUAD4: "quad4", WEDGE6: "wedge6", PYRAMID5: "pyramid5"}

BASE_SEED = 160404689


@dataclasses.dataclass
class Mesh:
    """A generated mesh plus what is needed to reason about it in tests.

    ``conn``     int32 [n_elem, npe], relabelled and shuffled.
    ``etype``    element type code.
    ``n_vert``   number of vertices.
    ``perm``     int64 [n_vert]; new id of lattice vertex ``x`` is ``perm[x]``.
    ``dims``     lattice vertex counts per axis (before relabelling).
    ``elem_order`` int64 [n_elem]; row ``r`` of ``conn`` is lattice element
                 ``elem_order[r]``.
    """

    conn: np.ndarray
    etype: int
    n_vert: int
    perm: np.ndarray
    dims: tuple
    elem_order: np.ndarray
    name: str = ""

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def npe(self) -> int:
        return NODES_PER_ELEM[self.etype]


def _finish(conn_lattice, etype, n_vert, dims, rng, name, relabel=True, shuffle=True):
    conn_lattice = np.asarray(conn_lattice, dtype=np.int64)
    if relabel:
        perm = rng.permutation(n_vert).astype(np.int64)
    else:
        perm = np.arange(n_vert, dtype=np.int64)
    conn = perm[conn_lattice]
    f = conn.shape[0]
    if shuffle:
        order = rng.permutation(f).astype(np.int64)
    else:
        order = np.arange(f, dtype=np.int64)
    conn = np.ascontiguousarray(conn[order].astype(np.int32))
    return Mesh(conn=conn, etype=etype, n_vert=int(n_vert), perm=perm, dims=tuple(dims),
                elem_order=order, name=name)


def tri_grid(n: int, diag: str = "main", seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """Triangle grid of ``n x n`` vertices, two triangles per cell.

    Lattice vertex (i, j) has id ``i*n + j``.  ``diag='main'`` splits every
    cell along (i,j)-(i+1,j+1); ``diag='coin'`` draws one seeded coin per cell
    and uses the other diagonal (i,j+1)-(i+1,j) where it comes up 1.  Draw
    order from ``default_rng(seed)``: coins (if any), vertex permutation,
    element permutation.
    """
    if n < 2:
        raise ValueError("tri_grid needs n >= 2")
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    a = i * n + j
    b = i * n + j + 1
    c = (i + 1) * n + j
    d = (i + 1) * n + j + 1
    if diag == "main":
        flip = np.zeros(a.shape, dtype=bool)
    elif diag == "coin":
        flip = rng.integers(0, 2, size=a.shape[0]).astype(bool)
    else:
        raise ValueError(diag)
    t1 = np.where(flip[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(flip[:, None], np.stack([b, d, c], 1), np.stack([a, d, c], 1))
    conn = np.empty((2 * a.shape[0], 3), dtype=np.int64)
    conn[0::2] = t1
    conn[1::2] = t2
    return _finish(conn, TRI3, n * n, (n, n), rng, f"tri{n}_{diag}", relabel, shuffle)


def _cube_vertex_ids(m):
    """Lattice ids of the 8 corners of every cell of an m^3 cell cube.

    Vertex (x, y, z) has id ``(x*(m+1) + y)*(m+1) + z``.  Returns a dict
    keyed by the corner offset (dx, dy, dz).
    """
    s = m + 1
    x, y, z = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    x = x.ravel()
    y = y.ravel()
    z = z.ravel()
    out = {}
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                out[(dx, dy, dz)] = ((x + dx) * s + (y + dy)) * s + (z + dz)
    return out


def kuhn_tet_grid(m: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """Cube of ``m^3`` cells, each split into the 6 Kuhn tetrahedra.

    Every tet of a cell walks a monotone lattice path from corner (0,0,0) to
    (1,1,1), stepping along the axes in one of the 6 axis orders, so all six
    share the main diagonal.  Draw order: vertex permutation, element
    permutation.
    """
    if m < 1:
        raise ValueError("kuhn_tet_grid needs m >= 1")
    rng = np.random.default_rng(seed)
    corner = _cube_vertex_ids(m)
    axis_orders = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for order in axis_orders:
        p = [0, 0, 0]
        path = [corner[tuple(p)]]
        for ax in order:
            p[ax] = 1
            path.append(corner[tuple(p)])
        tets.append(np.stack(path, 1))
    conn = np.stack(tets, 1).reshape(-1, 4)
    s = m + 1
    return _finish(conn, TET4, s ** 3, (s, s, s), rng, f"kuhn{m}", relabel, shuffle)


def hex_grid(m: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """Cube of ``m^3`` hexahedral cells, VTK node order."""
    if m < 1:
        raise ValueError("hex_grid needs m >= 1")
    rng = np.random.default_rng(seed)
    corner = _cube_vertex_ids(m)
    vtk = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    conn = np.stack([corner[c] for c in vtk], 1)
    s = m + 1
    return _finish(conn, HEX8, s ** 3, (s, s, s), rng, f"hex{m}", relabel, shuffle)


def quad_grid(n: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """Quadrilateral grid of ``n x n`` vertices (lattice id ``i*n + j``), one
    quad per cell with its nodes around the cell."""
    if n < 2:
        raise ValueError("quad_grid needs n >= 2")
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    i, j = i.ravel(), j.ravel()
    conn = np.stack([i * n + j, (i + 1) * n + j, (i + 1) * n + j + 1, i * n + j + 1], 1)
    return _finish(conn, QUAD4, n * n, (n, n), rng, f"quad{n}", relabel, shuffle)


def wedge_grid(n: int, layers: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """The ``n x n`` vertex main-diagonal triangle grid extruded through
    ``layers`` layers: lattice vertex (i, j, k) has id ``(i*n + j)*(layers+1) + k``
    and every triangle of every layer is a wedge, its lower triangle first."""
    if n < 2 or layers < 1:
        raise ValueError("wedge_grid needs n >= 2 and layers >= 1")
    rng = np.random.default_rng(seed)
    i, j, k = np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(layers), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    L = layers + 1

    def vid(a, b, c):
        return (a * n + b) * L + c

    tris = [((0, 0), (0, 1), (1, 1)), ((0, 0), (1, 1), (1, 0))]
    wedges = []
    for t in tris:
        lower = [vid(i + di, j + dj, k) for di, dj in t]
        upper = [vid(i + di, j + dj, k + 1) for di, dj in t]
        wedges.append(np.stack(lower + upper, 1))
    conn = np.stack(wedges, 1).reshape(-1, 6)
    return _finish(conn, WEDGE6, n * n * L, (n, n, L), rng, f"wedge{n}x{layers}", relabel, shuffle)


# the 6 faces of a cell as quadrilaterals around the face, seen so that the
# pyramid's base and the cell centre give a VTK pyramid
_CELL_FACES = [
    [(0, 0, 0), (0, 1, 0), (1, 1, 0), (1, 0, 0)],
    [(0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
    [(0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)],
    [(0, 1, 0), (0, 1, 1), (1, 1, 1), (1, 1, 0)],
    [(0, 0, 0), (0, 0, 1), (0, 1, 1), (0, 1, 0)],
    [(1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1)],
]


def pyramid_grid(m: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> Mesh:
    """Cube of ``m^3`` cells, each cut into 6 pyramids: one per face, the
    face as base and a vertex at the cell centre as apex.  Lattice corners
    come first (as in ``hex_grid``), then the m^3 cell centres."""
    if m < 1:
        raise ValueError("pyramid_grid needs m >= 1")
    rng = np.random.default_rng(seed)
    corner = _cube_vertex_ids(m)
    s = m + 1
    centre = s ** 3 + np.arange(m ** 3)
    pyrs = [np.stack([corner[c] for c in face] + [centre], 1) for face in _CELL_FACES]
    conn = np.stack(pyrs, 1).reshape(-1, 5)
    return _finish(conn, PYRAMID5, s ** 3 + m ** 3, (s ** 3 + m ** 3,), rng, f"pyramid{m}", relabel, shuffle)


@dataclasses.dataclass
class MixedMesh:
    """A mesh whose elements carry their own types: ``conn`` int32 holds
    every element's ids back to back, ``etypes`` uint8 one code per element."""

    conn: np.ndarray
    etypes: np.ndarray
    n_vert: int
    name: str = ""

    @property
    def n_elem(self) -> int:
        return int(self.etypes.shape[0])

    def elem_off(self):
        npe = np.array([NODES_PER_ELEM[t] for t in range(6)], dtype=np.int64)[self.etypes.astype(np.int64)]
        off = np.zeros(self.n_elem + 1, dtype=np.int64)
        np.cumsum(npe, out=off[1:])
        return off


def _kuhn_cell_tets(corner_of):
    out = []
    for order in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
        p = [0, 0, 0]
        path = [corner_of(tuple(p))]
        for ax in order:
            p[ax] = 1
            path.append(corner_of(tuple(p)))
        out.append(path)
    return out


def hybrid_grid(m: int, seed: int = BASE_SEED, relabel=True, shuffle=True) -> MixedMesh:
    """Cube of ``m^3`` cells, each (by a seeded draw) one hexahedron, two
    wedges (cut along the plane through its (0,0,z)-(1,1,z) diagonals), six
    pyramids to a centre vertex, or six Kuhn tetrahedra.  Vertices: the
    lattice corners, then one centre per cell (used only by pyramid cells).
    Element order shuffled, vertex ids relabelled."""
    if m < 1:
        raise ValueError("hybrid_grid needs m >= 1")
    rng = np.random.default_rng(seed)
    s = m + 1
    kinds = rng.integers(0, 4, size=m ** 3)
    elems, types = [], []
    vtk_hex = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    cell = 0
    for x in range(m):
        for y in range(m):
            for z in range(m):
                def corner(c):
                    return ((x + c[0]) * s + (y + c[1])) * s + (z + c[2])
                kind = int(kinds[cell])
                if kind == 0:
                    elems.append([corner(c) for c in vtk_hex])
                    types.append(HEX8)
                elif kind == 1:
                    for tri in (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                        elems.append([corner((a, b, 0)) for a, b in tri] + [corner((a, b, 1)) for a, b in tri])
                        types.append(WEDGE6)
                elif kind == 2:
                    for face in _CELL_FACES:
                        elems.append([corner(c) for c in face] + [s ** 3 + cell])
                        types.append(PYRAMID5)
                else:
                    for t in _kuhn_cell_tets(corner):
                        elems.append(t)
                        types.append(TET4)
                cell += 1
    n_vert = s ** 3 + m ** 3
    perm = rng.permutation(n_vert) if relabel else np.arange(n_vert)
    order = rng.permutation(len(elems)) if shuffle else np.arange(len(elems))
    conn = np.concatenate([perm[np.asarray(elems[e])] for e in order]).astype(np.int32)
    etypes = np.asarray(types, dtype=np.uint8)[order]
    return MixedMesh(conn=np.ascontiguousarray(conn), etypes=etypes, n_vert=n_vert, name=f"hybrid{m}")


def random_mixed(n_elem: int, n_vert: int, seed: int, types=(0, 1, 2, 3, 4, 5)) -> MixedMesh:
    """Random element types (from ``types``) with ids uniform in [0, n_vert):
    degenerate and duplicate elements and unused vertices all occur."""
    rng = np.random.default_rng(seed)
    etypes = np.asarray(types, dtype=np.uint8)[rng.integers(0, len(types), size=n_elem)]
    n_ids = int(sum(NODES_PER_ELEM[int(t)] for t in etypes))
    conn = rng.integers(0, max(n_vert, 1), size=n_ids).astype(np.int32)
    return MixedMesh(conn=conn, etypes=etypes, n_vert=int(n_vert), name=f"mixed{n_elem}x{n_vert}")


def random_mesh(n_elem: int, n_vert: int, etype: int, seed: int) -> Mesh:
    """Unstructured random connectivity (ids uniform in [0, n_vert)).

    Repeated ids inside one element (degenerate elements), unused vertices and
    duplicate elements all occur; used for edge-case parity tests.
    """
    rng = np.random.default_rng(seed)
    npe = NODES_PER_ELEM[etype]
    conn = rng.integers(0, max(n_vert, 1), size=(n_elem, npe)).astype(np.int32)
    if n_vert == 0:
        conn = conn[:0]
    return Mesh(conn=np.ascontiguousarray(conn), etype=etype, n_vert=int(n_vert),
                perm=np.arange(n_vert), dims=(n_vert,), elem_order=np.arange(conn.shape[0]),
                name=f"random{TYPE_NAMES[etype]}_{n_elem}x{n_vert}")


# ---------------------------------------------------------------------------
# The workloads: a small structured triangle grid, a large coin-flip triangle
# surface, a Kuhn tetrahedral cube, a batch of mixed meshes and a Poisson
# request stream drawn from the batch's size distribution.
# ---------------------------------------------------------------------------

def tri64(seed=BASE_SEED + 0) -> Mesh:
    """64 x 64 vertex grid, main diagonals: 7938 triangles, 4096 vertices."""
    return tri_grid(64, "main", seed)


def tri2048(seed=BASE_SEED + 1) -> Mesh:
    """2048 x 2048 vertex grid, coin-flip diagonals: 8,380,418 triangles."""
    return tri_grid(2048, "coin", seed)


def kuhn96(seed=BASE_SEED + 2) -> Mesh:
    """96^3 cell Kuhn cube: 5,308,416 tets, 912,673 vertices."""
    return kuhn_tet_grid(96, seed)


@dataclasses.dataclass
class MeshSpec:
    etype: int
    size: int  # tri: vertices per side; tet/hex: cells per side
    seed: int

    def build(self) -> Mesh:
        if self.etype == TRI3:
            return tri_grid(self.size, "coin", self.seed)
        if self.etype == TET4:
            return kuhn_tet_grid(self.size, self.seed)
        return hex_grid(self.size, self.seed)

    @property
    def n_elem(self) -> int:
        if self.etype == TRI3:
            return 2 * (self.size - 1) ** 2
        if self.etype == TET4:
            return 6 * self.size ** 3
        return self.size ** 3

    @property
    def n_vert(self) -> int:
        if self.etype == TRI3:
            return self.size ** 2
        return (self.size + 1) ** 3


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_specs(n_mesh: int = 512, seed: int = BASE_SEED + 3,
                tri_range=(8, 512), cell_range=(4, 48), p_hex=0.10):
    """Size/type draw of the mixed batch.

    Per mesh: hex with probability ``p_hex``, otherwise triangle or Kuhn tet
    with equal probability.  Triangle grids have a log-uniform vertex side in
    ``tri_range``; tet and hex grids a log-uniform cell side in
    ``cell_range``.  Each mesh gets its own seed drawn from the batch seed.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_mesh):
        u = rng.uniform()
        if u < p_hex:
            et = HEX8
        elif u < p_hex + (1 - p_hex) / 2:
            et = TRI3
        else:
            et = TET4
        if et == TRI3:
            size = _log_uniform_int(rng, *tri_range)
        else:
            size = _log_uniform_int(rng, *cell_range)
        specs.append(MeshSpec(et, size, int(rng.integers(0, 2 ** 31 - 1))))
    return specs


def batch_meshes(n_mesh: int = 512, seed: int = BASE_SEED + 3, **kw):
    return [s.build() for s in batch_specs(n_mesh, seed, **kw)]


def poisson_arrivals(n_req: int, rate_per_s: float, seed: int = BASE_SEED + 4):
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_req)
    return np.cumsum(gaps)
