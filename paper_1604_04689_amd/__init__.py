"""One-ring node and element neighbor lists of generic meshes on MI355X.

The compute path is the HIP library ``libmeshnbr.so`` (C ABI in
``include/mesh_neighbors.h``); this package holds its ctypes binding
(``binding``), the in-tree build script (``build``) and seeded synthetic
mesh generators (``meshgen``).
"""
from .binding import (HEX8, TET4, TRI3, MeshError, NeighborBuild, Status, elem_neighbors,  # noqa: F401
                      lib, node_neighbors, query_elem, query_node, status_string, timing_enable,
                      timing_read, radix_shapes, set_radix_shape, get_radix_shape,
                      BatchBuild, segment_table, concat_conn, set_node_sort, get_node_sort,
                      NODE_SORT_FULL_KEY, NODE_SORT_VERTEX_ROWS, NODE_SORT_EDGE_ROWS, Graph)
