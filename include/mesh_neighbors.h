/*
 * mesh_neighbors.h -- C ABI of the one-ring neighbor library (libmeshnbr.so).
 *
 * For every vertex of a mesh given as plain integer connectivity, the library
 * finds its one-ring neighboring nodes (vertices joined to it by an element
 * edge) and its one-ring neighboring elements (elements that contain it), as
 * defined in Sec. 1 of Mei et al., "A Parallel Solution to Finding Nodal
 * Neighbors in Generic Meshes", and returns each relation as a CSR matrix with
 * ascending, duplicate-free rows.  The method follows Sec. 2: form integer
 * pairs per element, sort them by their first entry, then derive counts and
 * first indices per vertex by segmented reduction and scan.  Everything runs
 * in HIP kernels on the device; inputs and outputs stay in device memory.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Ids are 0-based.  Element e is row e of the connectivity array, which is
 *    int32, row-major [n_elem][nodes_per_element] (for a mesh of one element
 *    type), or, for a mixed mesh, element e's ids are
 *    conn[elem_off[e] .. elem_off[e+1]).
 *  - Element types and their edges (pairs of node positions).  Node orders
 *    are those of VTK; the paper shows triangles and states that the method
 *    applies to meshes of any element type (Sec. 2.2, Sec. 4):
 *      MESH_TRI3     (3 nodes): (0,1) (1,2) (2,0)
 *      MESH_TET4     (4 nodes): all 6 pairs
 *      MESH_HEX8     (8 nodes, 0-1-2-3 bottom face, 4-7 the nodes above them):
 *                    (0,1)(1,2)(2,3)(3,0)(4,5)(5,6)(6,7)(7,4)(0,4)(1,5)(2,6)(3,7)
 *      MESH_QUAD4    (4 nodes around the face): (0,1)(1,2)(2,3)(3,0)
 *      MESH_WEDGE6   (6 nodes, triangle 0-1-2 and triangle 3-4-5 above it):
 *                    (0,1)(1,2)(2,0)(3,4)(4,5)(5,3)(0,3)(1,4)(2,5)
 *      MESH_PYRAMID5 (5 nodes, base 0-1-2-3 and apex 4):
 *                    (0,1)(1,2)(2,3)(3,0)(0,4)(1,4)(2,4)(3,4)
 *    Face and body diagonals are not edges.
 *  - Output CSR: row_ptr is int32 [n_vert + 1], row_ptr[0] = 0, and the
 *    neighbors of v are cols[row_ptr[v] .. row_ptr[v+1]) in ascending order.
 *    A vertex is never its own neighbor; a repeated id inside one element
 *    (a degenerate element) yields no self pair and lists that element once.
 *    Vertices used by no element get empty rows.  nnz = row_ptr[n_vert].
 *  - Every data pointer (conn, row_ptr, cols, workspace, the batched and
 *    mixed descriptor arrays) is a DEVICE pointer owned by the caller; the
 *    library allocates nothing and keeps no state between calls (apart from
 *    the fixed scratch array of mesh_neighbors_noalloc).  `opts`
 *    (host pointer, may be NULL) selects speed-only choices for that call
 *    alone.  `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *    asynchronous and stream-ordered; none synchronises the host except
 *    mesh_check and a bounded-memory build (chunk_keys, below), which waits
 *    once on its stream.
 *  - Argument errors are returned synchronously before anything is launched.
 *    Data errors found on the device (a vertex id outside [0, n_vert), more
 *    nnz than cols_capacity) are recorded in the workspace: the output is then
 *    unspecified but every access stays in bounds, and mesh_check reports it.
 *  - Calls are thread-safe; two calls may run concurrently only with
 *    distinct workspaces and outputs.
 */
#ifndef MESH_NEIGHBORS_H
#define MESH_NEIGHBORS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MESH_TRI3 = 0,
    MESH_TET4 = 1,
    MESH_HEX8 = 2,
    MESH_QUAD4 = 3,
    MESH_WEDGE6 = 4,
    MESH_PYRAMID5 = 5
} mesh_elem_type;

typedef enum {
    MESH_OK = 0,
    MESH_ERR_INVALID_ARG = 1,      /* null pointer, negative size, bad option  */
    MESH_ERR_UNSUPPORTED_TYPE = 2, /* element type code not listed above       */
    MESH_ERR_WORKSPACE = 3,        /* workspace smaller than the query says    */
    MESH_ERR_CAPACITY = 4,         /* nnz exceeded cols_capacity (device check)*/
    MESH_ERR_OVERFLOW = 5,         /* sizes beyond the int32 / pair-count range*/
    MESH_ERR_INDEX_RANGE = 6,      /* a connectivity id outside [0, n_vert)    */
    MESH_ERR_HIP = 7,              /* a HIP runtime call or launch failed       */
    MESH_ERR_INTERNAL = 8,         /* a device-side consistency guard tripped   */
    MESH_ERR_SCRATCH_LIMIT = 9,    /* mesh_neighbors_noalloc: the mesh needs more
                                      scratch than MESH_NOALLOC_SCRATCH_BYTES      */
    MESH_ERR_CHUNK = 10            /* bounded-memory build: one vertex bin holds
                                      more pairs than chunk_keys               */
} mesh_status;

/* ------------------------------------------------------------------------ */
/* Per-call options: speed only, never results.                             */
/* ------------------------------------------------------------------------ */

/* How the node relation orders its pairs.  All give the same bytes.
 *  FULL_KEY:     directed pairs packed as (u << b) | w, b = bits of n_vert - 1,
 *                LSD radix passes over all 2b bits, then one pass drops
 *                repeats and writes the CSR.
 *  VERTEX_ROWS:  the same pairs sorted by the bits of u only (the paper's sort
 *                by the first array, Sec. 2.2.1), then each row's neighbor ids
 *                deduplicated and ordered in LDS (rows over 256 pairs by a
 *                block each), counts scanned into row_ptr, rows gathered.
 *  EDGE_ROWS:    every element edge once, (min << b) | max, sorted by min and
 *                deduplicated per row as in VERTEX_ROWS (each vertex's higher
 *                neighbors and the unique edges); those edges transposed and
 *                sorted by max give each vertex's lower neighbors; a row is its
 *                lower neighbors followed by its higher ones.
 *  ELEM_ROWS:    the element relation first (the counting sort of (v, e) pairs
 *                by v, Sec. 2.2.2); row v of the node relation is then the
 *                set of edge-neighbors of v over the elements of its element
 *                row, gathered into LDS, deduplicated and ordered there (rows
 *                over the LDS limit by a block each from global memory).  Only
 *                the element pairs are sorted. */
typedef enum {
    MESH_NODE_SORT_FULL_KEY = 0,
    MESH_NODE_SORT_VERTEX_ROWS = 1,
    MESH_NODE_SORT_EDGE_ROWS = 2,
    MESH_NODE_SORT_ELEM_ROWS = 3
} mesh_node_sort;

/* Fields set to -1 take the library default (a rule built into the library,
 * the same for every call of the same sizes).  The workspace size depends on
 * the options: query and call with the same options. */
typedef struct {
    int32_t node_sort;    /* mesh_node_sort, or -1                               */
    int32_t radix_shape;  /* radix tile shape 0 .. mesh_radix_shape_count()-1, or -1 */
    int32_t digit_bits;   /* radix digit width: 8 or 11 bits per pass, or -1      */
    int32_t chunk_keys;   /* bounded-memory build: most pairs sorted at once, or
                             -1 / 0 for the whole mesh at once (see below)     */
    int32_t reserved[4];  /* 0                                                    */
} mesh_options;

/* Bounded-memory build (chunk_keys > 0).  The paper names the device memory
 * its pair arrays take as the limit of its method and leaves a leaner
 * variant to future work (Sec. 3.2.2, Sec. 4).  With chunk_keys set, a call
 * builds the relations one vertex range at a time: a histogram of the
 * (vertex, element) pairs over the top 11 bits of the vertex id is read back
 * (the call waits on its stream once, so it cannot be captured into a
 * graph), the host cuts [0, n_vert) at bin boundaries into ranges of at most
 * chunk_keys pairs and chunk_keys vertices, and each range compacts its own
 * pairs out of the connectivity (every range reads all of it), sorts them,
 * and writes its element rows, then derives its node rows, straight into the
 * outputs.  The workspace holds O(chunk_keys) words plus one 8-byte word per
 * 24576 connectivity slots, where a whole-mesh build takes 17 to 50 bytes per
 * slot.  Results are identical.
 * Applies to mesh_node_neighbors, mesh_elem_neighbors, mesh_neighbors (and
 * their queries and mesh_neighbors_noalloc) under the ELEM_ROWS node
 * algorithm (mesh_elem_neighbors takes any node_sort) with 8-bit digits;
 * other entry points (batches, mixed meshes, graph captures), other node
 * algorithms or digit_bits = 11 return MESH_ERR_INVALID_ARG, as does
 * chunk_keys below 4096 or below the vertices of one bin
 * (2^(bits of n_vert - 1) / 2^11).  A bin of more than chunk_keys pairs
 * returns MESH_ERR_CHUNK (synchronously, after the histogram; the outputs
 * are then unspecified). */

/* Options with every field set to -1 (the library defaults). */
mesh_options mesh_default_options(void);

/* ------------------------------------------------------------------------ */
/* Neighboring nodes (Sec. 2.1.1, 2.2.1).                                   */
/* ------------------------------------------------------------------------ */

/* Workspace size and a cols capacity that always suffices for
 * mesh_node_neighbors on a mesh of n_elem elements of type etype over n_vert
 * vertices, under `opts`.  The capacity is the number of directed edge pairs,
 * 2 * edges_per_element * n_elem (every pair distinct in the worst case).
 * Limits: n_vert <= 2^31 - 1; pairs <= 2^31 - 1 (else MESH_ERR_OVERFLOW). */
mesh_status mesh_node_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                      size_t* workspace_bytes, int64_t* cols_capacity);

/* One-ring neighboring nodes of every vertex.
 *   conn           device int32 [n_elem * npe], read only
 *   row_ptr        device int32 [n_vert + 1], written
 *   cols           device int32 [cols_capacity], first nnz entries written
 *   opts           host, may be NULL (defaults)
 *   workspace      device scratch of >= the queried size (256-byte aligned);
 *                  its first bytes carry the device error word that
 *                  mesh_check reads, so keep it until checked.
 * The pipeline is the one opts->node_sort names (see mesh_node_sort). */
mesh_status mesh_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Neighboring elements (Sec. 2.1.2, 2.2.2).                                */
/* ------------------------------------------------------------------------ */

/* Workspace size and sufficient cols capacity (npe * n_elem) for
 * mesh_elem_neighbors.  Limits: n_elem * npe <= 2^31 - 1. */
mesh_status mesh_elem_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                      size_t* workspace_bytes, int64_t* cols_capacity);

/* One-ring neighboring elements of every vertex.  Same arguments as
 * mesh_node_neighbors.  Pipeline: one (v, e) pair per node slot of every
 * element (the first occurrence of an id inside its element), sorted by v
 * with stable LSD counting-sort passes over the digits of v, the first pass
 * reading the connectivity itself; pairs enter in element order, so each row
 * comes out ascending.  The last pass writes cols and offers every row start
 * to row_ptr with an atomic minimum; empty rows take the next row's start. */
mesh_status mesh_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Both relations in one call.                                              */
/* ------------------------------------------------------------------------ */

/* Workspace size and both cols capacities for mesh_neighbors. */
mesh_status mesh_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                 size_t* workspace_bytes, int64_t* node_cols_capacity,
                                 int64_t* elem_cols_capacity);

/* The node and element relations of one mesh.  Output arguments as for the
 * two single-relation calls.  Under MESH_NODE_SORT_ELEM_ROWS the node
 * relation is derived from the element relation just written (so the element
 * pairs are sorted once for both); otherwise the two pipelines run one after
 * the other in the one workspace. */
mesh_status mesh_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                           int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                           int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                           const mesh_options* opts, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Both relations without a workspace argument.                             */
/* ------------------------------------------------------------------------ */

/* Size of the library's fixed device scratch array (64 MiB): enough for any
 * mesh whose mesh_neighbors_query workspace is at most this size, e.g. up to
 * about 1.2 M triangles or 0.97 M tetrahedra under the default options. */
#define MESH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc):
 * mesh_neighbors with the same arguments, results and argument checks, but
 * without a workspace.  Its scratch is a device array of
 * MESH_NOALLOC_SCRATCH_BYTES owned by the library: each GPU the library runs
 * on holds its own copy until the process ends.  The caller still passes the
 * inputs and the outputs (device memory it owns).  Nothing is allocated: no
 * hipMalloc, hipFree or allocating library routine is called, and launches
 * are never timed (mesh_timing_enable does not apply).  The first call on a
 * device looks up that device's copy of the array, with the device current.
 *   - A mesh whose workspace (mesh_neighbors_query with the same options)
 *     exceeds MESH_NOALLOC_SCRATCH_BYTES is refused with
 *     MESH_ERR_SCRATCH_LIMIT before anything is launched.  Under a pair
 *     budget (mesh_options.chunk_keys) the workspace no longer grows with
 *     the mesh, so much larger meshes fit; such a call waits on its stream
 *     once and so cannot be captured into a graph.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (each call sets everything that must start at a fixed
 *     value itself).  Calls that overlap on one GPU (other streams, other
 *     host threads) RACE on the array and give wrong results: serialise them.
 *   - mesh_check(NULL, stream) reports the data error of the last call on
 *     the current device, as mesh_check does for a workspace. */
mesh_status mesh_neighbors_noalloc(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                   int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                   int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                   const mesh_options* opts, void* stream);

/* ------------------------------------------------------------------------ */
/* Meshes with several element types.                                       */
/* ------------------------------------------------------------------------ */

/* A mesh whose elements have their own types: element e has type etypes[e]
 * (uint8, a mesh_elem_type) and ids conn[elem_off[e] .. elem_off[e+1]),
 * elem_off int32 [n_elem + 1] with elem_off[0] = 0 and
 * elem_off[e+1] - elem_off[e] = nodes of etypes[e].  n_ids = elem_off[n_elem]
 * (the slot count) and n_pairs = sum of 2 * edges of each element's type are
 * given by the caller for sizing.  Both relations are built; the node
 * relation always takes the ELEM_ROWS algorithm (opts->node_sort must be -1
 * or MESH_NODE_SORT_ELEM_ROWS).  An element whose type code is unknown or
 * whose offsets disagree with its type raises MESH_ERR_INDEX_RANGE on the
 * device and contributes nothing.  Limits: n_ids, n_pairs <= 2^31 - 1. */
mesh_status mesh_mixed_neighbors_query(int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert,
                                       const mesh_options* opts, size_t* workspace_bytes,
                                       int64_t* node_cols_capacity, int64_t* elem_cols_capacity);
mesh_status mesh_mixed_neighbors(const int32_t* conn, const int32_t* elem_off, const uint8_t* etypes,
                                 int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* ------------------------------------------------------------------------ */
/* Batches of independent meshes in one launch sequence.                    */
/* ------------------------------------------------------------------------ */

/* One mesh of a batch: a record in DEVICE memory, filled by the caller.  All
 * meshes share one int32 connectivity array; the ids inside a mesh are local
 * to it, in [0, n_vert).  Offsets are prefix sums over the meshes before it,
 * in order: pair_off of 2 * edges_per_element * n_elem, slot_off of
 * nodes_per_element * n_elem, vert_off of n_vert (so the meshes' vertex
 * ranges tile [0, total_vert) in order).  Meshes may mix types. */
typedef struct {
    int64_t conn_off;  /* index of the mesh's first id in the shared conn */
    int64_t n_elem;
    int64_t pair_off;  /* first directed edge pair of the mesh            */
    int64_t slot_off;  /* first (node, element) slot of the mesh          */
    int32_t vert_off;  /* first global vertex of the mesh                 */
    int32_t n_vert;
    int32_t etype;     /* mesh_elem_type                                  */
    int32_t reserved;  /* 0                                               */
} mesh_segment;

/* Neighboring nodes of every vertex of every mesh of a batch.
 *   segs         device mesh_segment [n_mesh]
 *   total_pairs  sum of 2 * edges_per_element * n_elem (the pair_off end)
 *   total_slots  sum of nodes_per_element * n_elem (the slot_off end)
 *   total_vert   sum of n_vert;  max_vert = largest n_vert of one mesh
 *   row_ptr      device int32 [total_vert + 1]: one CSR over all vertices,
 *                mesh m owning rows vert_off[m] .. vert_off[m] + n_vert[m]
 *   cols         device int32 [cols_capacity]; entries are LOCAL vertex ids
 * The slice row_ptr[vert_off .. vert_off + n_vert] - row_ptr[vert_off] with its
 * cols equals mesh_node_neighbors on that mesh alone.  Keys carry the global
 * vertex vert_off + u.  A record inconsistent with total_pairs, total_vert
 * or its own size (a key or vertex range outside the batch, an unknown type)
 * raises MESH_ERR_INDEX_RANGE on the device, and its pairs are dropped;
 * conn itself must cover every record (not checkable here). */
mesh_status mesh_batch_node_neighbors_query(int32_t n_mesh, int64_t total_pairs, int64_t total_slots,
                                            int32_t total_vert, int32_t max_vert, const mesh_options* opts,
                                            size_t* workspace_bytes, int64_t* cols_capacity);
mesh_status mesh_batch_node_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      void* stream);

/* Neighboring elements of every vertex of every mesh of a batch: as above,
 * with total_slots = sum of nodes_per_element * n_elem; cols hold element
 * ids LOCAL to the mesh.  Keys (vert_off + v) << 32 | e, sorted over the bits
 * of total_vert - 1. */
mesh_status mesh_batch_elem_neighbors_query(int32_t n_mesh, int64_t total_slots, int32_t total_vert,
                                            const mesh_options* opts, size_t* workspace_bytes,
                                            int64_t* cols_capacity);
mesh_status mesh_batch_elem_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_slots, int32_t total_vert, int32_t* row_ptr, int32_t* cols,
                                      int64_t cols_capacity, const mesh_options* opts, void* workspace,
                                      size_t workspace_bytes, void* stream);

/* Both relations of a batch in one call (as mesh_neighbors for one mesh). */
mesh_status mesh_batch_neighbors_query(int32_t n_mesh, int64_t total_pairs, int64_t total_slots,
                                       int32_t total_vert, int32_t max_vert, const mesh_options* opts,
                                       size_t* workspace_bytes, int64_t* node_cols_capacity,
                                       int64_t* elem_cols_capacity);
mesh_status mesh_batch_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                 int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* ------------------------------------------------------------------------ */
/* HIP graphs: one call's launch sequence, captured once, replayed cheaply. */
/* ------------------------------------------------------------------------ */

/* An instantiated HIP graph owned by the library (opaque). */
typedef struct mesh_graph_s* mesh_graph;

/* Each mesh_graph_* capture takes the arguments of the entry point of the
 * same name (without the stream), validates them exactly as that entry point
 * does (returning the same status), and records its whole launch sequence on
 * a private stream into *graph.  Nothing runs at capture time.  The graph
 * keeps the pointers, sizes and options it was captured with: every replay
 * reads the buffers' contents at that time (conn, and segs for batches, may
 * change between replays; their sizes may not) and rewrites the outputs and
 * the workspace, so a replay returns what an eager call on the same contents
 * returns, bit for bit.  The buffers must stay allocated while the graph
 * lives.  Launches being captured are not timed.  Returns MESH_ERR_HIP if
 * capture or instantiation fails; *graph is then NULL. */
mesh_status mesh_graph_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      mesh_graph* graph);
mesh_status mesh_graph_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      mesh_graph* graph);
mesh_status mesh_graph_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                 mesh_graph* graph);
mesh_status mesh_graph_batch_node_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                            int64_t total_pairs, int64_t total_slots, int32_t total_vert,
                                            int32_t max_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                            const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                            mesh_graph* graph);
mesh_status mesh_graph_batch_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                       int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                       int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                       int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                       const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                       mesh_graph* graph);
mesh_status mesh_graph_batch_elem_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                            int64_t total_slots, int32_t total_vert, int32_t* row_ptr,
                                            int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                            void* workspace, size_t workspace_bytes, mesh_graph* graph);

/* Enqueues one replay of `graph` on `stream` (asynchronous, like the eager
 * calls; read errors with mesh_check on the captured workspace).  Replays of
 * one graph on different streams must not overlap: they share its buffers. */
mesh_status mesh_graph_launch(mesh_graph graph, void* stream);

/* Frees the graph (NULL is accepted).  Replays already enqueued complete. */
mesh_status mesh_graph_destroy(mesh_graph graph);

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                             */
/* ------------------------------------------------------------------------ */

/* Synchronises `stream`, then returns the data error recorded in `workspace`
 * by the last call that used it: MESH_OK, MESH_ERR_INDEX_RANGE,
 * MESH_ERR_CAPACITY or MESH_ERR_INTERNAL (MESH_ERR_HIP if the sync fails).
 * workspace = NULL reads the fixed scratch of mesh_neighbors_noalloc on the
 * current device. */
mesh_status mesh_check(const void* workspace, void* stream);

/* Static, human-readable name of a status code. */
const char* mesh_status_string(mesh_status status);

/* Library ABI version, (major << 16) | minor. */
int32_t mesh_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Tuning information.                                                      */
/* ------------------------------------------------------------------------ */

/* The radix tile shapes built into the library (threads per block x keys per
 * thread), numbered 0 .. mesh_radix_shape_count() - 1, for
 * mesh_options.radix_shape.  Returns MESH_ERR_INVALID_ARG for an unknown
 * shape. */
int32_t mesh_radix_shape_count(void);
mesh_status mesh_radix_shape_info(int32_t shape, int32_t* block, int32_t* items);

/* The tile shape (block x items) and digit width that a radix pass over
 * n_keys keys actually launches with when the options ask for `shape` and
 * `digit_bits` (-1 for defaults): passes over 2^30 keys or more, and digit
 * widths that have no such shape, take the default shape of that width.
 * Every table sized by tiles of a pass uses this same shape. */
mesh_status mesh_radix_launch_shape(int32_t shape, int32_t digit_bits, int64_t n_keys, int32_t* block,
                                    int32_t* items, int32_t* bits);

/* ------------------------------------------------------------------------ */
/* Kernel timing (diagnostics, not part of the method).                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    char name[32];     /* kernel name, e.g. "radix_pass"               */
    int64_t launches;  /* timed launches since the last read           */
    double total_ms;   /* summed device duration of those launches     */
    double min_ms;
    double max_ms;
} mesh_kernel_time;

/* While enabled (a process-wide diagnostics switch that changes no result),
 * every kernel the library launches (or each one mesh_timing_select names)
 * is bracketed by HIP events recorded by the launch itself on the launch's
 * own stream (hipExtLaunchKernel), on the device current when the events
 * were first created.  Up to 65536 launches are recorded between reads;
 * later ones run untimed.  Always MESH_OK. */
mesh_status mesh_timing_enable(int32_t enable);

/* Restricts timing to the launches named in `names`, a comma-separated list
 * of launch names as mesh_timing_read reports them (e.g. "node_erows");
 * NULL or "" times every launch again.  Each timed launch costs the stream
 * a few microseconds (the events it records), so a caller timing a whole
 * step can time only the kernels it needs.  Process-wide, like
 * mesh_timing_enable.  MESH_ERR_INVALID_ARG if the list is longer than 1024
 * characters or holds more than 32 names (the selection is then unchanged). */
mesh_status mesh_timing_select(const char* names);

/* Waits for the recorded launches to finish, aggregates their durations per
 * kernel name into out[0 .. min(n, max_entries)) and clears the record.
 * Returns n, the number of distinct kernel names, or -1 if an event query
 * failed. out may be NULL to only clear. */
int32_t mesh_timing_read(mesh_kernel_time* out, int32_t max_entries);

#ifdef __cplusplus
}
#endif

#endif /* MESH_NEIGHBORS_H */
