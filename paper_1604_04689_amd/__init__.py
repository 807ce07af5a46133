"""One-ring node and element neighbor lists of generic meshes on MI355X.

The compute path is the HIP library ``libmeshnbr.so`` (C ABI in
``include/mesh_neighbors.h``); this package holds its ctypes binding
(``binding``), the in-tree build script (``build``), seeded synthetic mesh
generators (``meshgen``), the autotuner (``autotune``) and the serving loop
(``serve``).
"""
from .binding import (HEX8, PYRAMID5, QUAD4, TET4, TRI3, WEDGE6, BatchBuild, Graph, MeshError,  # noqa: F401
                      MixedBuild, NeighborBuild, Options, Status, concat_conn, elem_neighbors, lib, make_options,
                      mixed_layout, mixed_neighbors, neighbors, neighbors_noalloc, node_neighbors, query, query_elem, query_node,
                      radix_launch_shape, radix_shapes, segment_table, status_string, timing_enable, timing_read,
                      timing_select, NODE_SORT_FULL_KEY, NODE_SORT_VERTEX_ROWS, NODE_SORT_EDGE_ROWS, NODE_SORT_ELEM_ROWS,
                      NODE_SORT_NAMES)
