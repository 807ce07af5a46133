/*
 * CPU oracle for one-ring neighbor finding.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, by the smoke check and by the benchmark's CPU-baseline
 * leg, never by the product path, and it shares no code with the HIP library.
 *
 * It writes out the plain serial definition the paper starts from (Sec. 1,
 * and the serial solution of Sec. 3.2.2): loop over the elements in order;
 * every pair of nodes joined by an element edge are one-ring neighboring
 * nodes of each other; every element is a one-ring neighboring element of
 * each node it contains.  Each vertex keeps its neighbors in an ordered set
 * (a sorted growable array with insert-if-absent), so the result holds no
 * repeated entries, which is how the serial solution stores them "without
 * redundant space" (Sec. 3.2.2).  Output is CSR: row_ptr[v]..row_ptr[v+1]
 * index the ascending neighbor ids of vertex v.
 *
 * Readings of the paper taken here (it is silent on them):
 *   - rows are ascending and free of duplicates;
 *   - a node is never its own neighbor (a repeated id inside a degenerate
 *     element yields no self pair) and an element is listed once per vertex;
 *   - neighboring nodes of a non-simplex element are those joined by one of
 *     its edges: 3 for a triangle, all 6 pairs of a tetrahedron, the 12 edges
 *     of a VTK-ordered hexahedron, the 4 sides of a quadrilateral, the 9 edges
 *     of a wedge, the 8 edges of a pyramid (the paper demonstrates triangles
 *     only, Sec. 2.2, and claims the method applies to arbitrary meshes,
 *     Sec. 2.2 and Sec. 4); a mesh may mix element types, each element
 *     contributing the edges of its own type;
 *   - ids are 0-based, element id = row of the connectivity array (for a
 *     mixed mesh, the element's index in its list of types).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- per-type element edge tables (node positions inside one element) --- */
static const int TRI_EDGES[3][2] = {{0, 1}, {1, 2}, {2, 0}};
static const int TET_EDGES[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
/* VTK hexahedron: bottom ring 0-1-2-3, top ring 4-5-6-7, verticals i-(i+4). */
static const int HEX_EDGES[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                                     {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
/* Quadrilateral: the four sides 0-1-2-3 (no diagonals). */
static const int QUAD_EDGES[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
/* VTK wedge: triangle 0-1-2, triangle 3-4-5 above it, verticals i-(i+3). */
static const int WEDGE_EDGES[9][2] = {{0, 1}, {1, 2}, {2, 0}, {3, 4}, {4, 5},
                                      {5, 3}, {0, 3}, {1, 4}, {2, 5}};
/* VTK pyramid: base ring 0-1-2-3, apex 4 joined to every base node. */
static const int PYR_EDGES[8][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {0, 4}, {1, 4}, {2, 4}, {3, 4}};

static int type_info(int32_t etype, int* npe, int* n_edges, const int (**edges)[2]) {
    switch (etype) {
        case 0: *npe = 3; *n_edges = 3; *edges = TRI_EDGES; return 0;
        case 1: *npe = 4; *n_edges = 6; *edges = TET_EDGES; return 0;
        case 2: *npe = 8; *n_edges = 12; *edges = HEX_EDGES; return 0;
        case 3: *npe = 4; *n_edges = 4; *edges = QUAD_EDGES; return 0;
        case 4: *npe = 6; *n_edges = 9; *edges = WEDGE_EDGES; return 0;
        case 5: *npe = 5; *n_edges = 8; *edges = PYR_EDGES; return 0;
        default: return -1;
    }
}

/* ---- ordered set of int32 (sorted array, insert if absent) -------------- */
typedef struct {
    int32_t* v;
    int32_t n, cap;
} ordered_set;

static int set_insert(ordered_set* s, int32_t x) {
    int32_t lo = 0, hi = s->n; /* first position with v[pos] >= x */
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (s->v[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo < s->n && s->v[lo] == x) return 0; /* already present */
    if (s->n == s->cap) {
        int32_t nc = s->cap ? 2 * s->cap : 8;
        int32_t* nv = (int32_t*)realloc(s->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        s->v = nv;
        s->cap = nc;
    }
    memmove(s->v + lo + 1, s->v + lo, (size_t)(s->n - lo) * sizeof(int32_t));
    s->v[lo] = x;
    s->n++;
    return 0;
}

static void free_sets(ordered_set* sets, int32_t n) {
    if (!sets) return;
    for (int32_t i = 0; i < n; ++i) free(sets[i].v);
    free(sets);
}

/* Concatenate the sets into CSR.  Returns nnz, or -3 if cols is too small or
 * nnz does not fit int32. */
static int64_t emit_csr(const ordered_set* sets, int32_t n_vert, int32_t* row_ptr,
                        int32_t* cols, int64_t cols_cap) {
    int64_t nnz = 0;
    for (int32_t v = 0; v < n_vert; ++v) nnz += sets[v].n;
    if (nnz > cols_cap || nnz > INT32_MAX) return -3;
    int64_t at = 0;
    row_ptr[0] = 0;
    for (int32_t v = 0; v < n_vert; ++v) {
        if (sets[v].n > 0) memcpy(cols + at, sets[v].v, (size_t)sets[v].n * sizeof(int32_t));
        at += sets[v].n;
        row_ptr[v + 1] = (int32_t)at;
    }
    return nnz;
}

/* Return codes shared by both entry points:
 *   >= 0  number of CSR entries written
 *   -1    invalid argument or unknown element type
 *   -2    a connectivity id lies outside [0, n_vert)
 *   -3    cols_cap too small (or nnz beyond int32)
 *   -4    out of host memory */

/* The node pairs of one element: both endpoints of every edge of its type
 * go into each other's set, except a self pair (Sec. 1; Sec. 2.1.1).
 * Returns 0, or -4 when out of memory. */
static int insert_element_nodes(ordered_set* sets, const int32_t* el, int n_edges, const int (*edges)[2]) {
    for (int k = 0; k < n_edges; ++k) {
        int32_t u = el[edges[k][0]], w = el[edges[k][1]];
        if (u == w) continue; /* no self pair */
        if (set_insert(&sets[u], w) || set_insert(&sets[w], u)) return -4;
    }
    return 0;
}

/* The element into the set of each of its nodes (Sec. 1; Sec. 2.1.2). */
static int insert_element_elem(ordered_set* sets, const int32_t* el, int npe, int32_t e) {
    for (int j = 0; j < npe; ++j) {
        if (set_insert(&sets[el[j]], e)) return -4;
    }
    return 0;
}

/* One-ring neighboring nodes of every vertex (Sec. 1; Sec. 2.1.1). */
int64_t oracle_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                              int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    int npe, n_edges;
    const int(*edges)[2];
    if (type_info(etype, &npe, &n_edges, &edges) != 0) return -1;
    if (n_elem < 0 || n_vert < 0 || (n_elem > 0 && !conn) || !row_ptr) return -1;
    for (int64_t i = 0; i < n_elem * npe; ++i)
        if (conn[i] < 0 || conn[i] >= n_vert) return -2;
    ordered_set* sets = (ordered_set*)calloc((size_t)n_vert + 1, sizeof(ordered_set));
    if (!sets) return -4;
    for (int64_t e = 0; e < n_elem; ++e) {
        if (insert_element_nodes(sets, conn + e * npe, n_edges, edges)) {
            free_sets(sets, n_vert);
            return -4;
        }
    }
    int64_t r = emit_csr(sets, n_vert, row_ptr, cols, cols_cap);
    free_sets(sets, n_vert);
    return r;
}

/* One-ring neighboring elements of every vertex (Sec. 1; Sec. 2.1.2). */
int64_t oracle_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                              int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    int npe, n_edges;
    const int(*edges)[2];
    if (type_info(etype, &npe, &n_edges, &edges) != 0) return -1;
    if (n_elem < 0 || n_vert < 0 || (n_elem > 0 && !conn) || !row_ptr) return -1;
    if (n_elem > INT32_MAX) return -1;
    for (int64_t i = 0; i < n_elem * npe; ++i)
        if (conn[i] < 0 || conn[i] >= n_vert) return -2;
    ordered_set* sets = (ordered_set*)calloc((size_t)n_vert + 1, sizeof(ordered_set));
    if (!sets) return -4;
    for (int64_t e = 0; e < n_elem; ++e) {
        if (insert_element_elem(sets, conn + e * npe, npe, (int32_t)e)) {
            free_sets(sets, n_vert);
            return -4;
        }
    }
    int64_t r = emit_csr(sets, n_vert, row_ptr, cols, cols_cap);
    free_sets(sets, n_vert);
    return r;
}

/* Meshes whose elements carry their own types: element e has type etypes[e]
 * and ids conn[elem_off[e] .. elem_off[e+1]).  relation 0: neighboring nodes,
 * 1: neighboring elements.  Beyond the codes above, -5: an element whose
 * offsets do not span its type's node count. */
static int64_t mixed_relation(int relation, const int32_t* conn, const int64_t* elem_off, const int32_t* etypes,
                              int64_t n_elem, int32_t n_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    if (n_elem < 0 || n_vert < 0 || n_elem > INT32_MAX || !row_ptr || (n_elem > 0 && (!elem_off || !etypes)))
        return -1;
    if (n_elem > 0 && elem_off[0] != 0) return -5;
    for (int64_t e = 0; e < n_elem; ++e) {
        int npe, n_edges;
        const int(*edges)[2];
        if (type_info(etypes[e], &npe, &n_edges, &edges) != 0) return -1;
        if (elem_off[e + 1] - elem_off[e] != npe) return -5;
    }
    for (int64_t i = 0; i < (n_elem > 0 ? elem_off[n_elem] : 0); ++i)
        if (conn[i] < 0 || conn[i] >= n_vert) return -2;
    ordered_set* sets = (ordered_set*)calloc((size_t)n_vert + 1, sizeof(ordered_set));
    if (!sets) return -4;
    for (int64_t e = 0; e < n_elem; ++e) {
        int npe, n_edges;
        const int(*edges)[2];
        type_info(etypes[e], &npe, &n_edges, &edges);
        const int32_t* el = conn + elem_off[e];
        int fail = relation == 0 ? insert_element_nodes(sets, el, n_edges, edges)
                                 : insert_element_elem(sets, el, npe, (int32_t)e);
        if (fail) {
            free_sets(sets, n_vert);
            return -4;
        }
    }
    int64_t r = emit_csr(sets, n_vert, row_ptr, cols, cols_cap);
    free_sets(sets, n_vert);
    return r;
}

int64_t oracle_mixed_node_neighbors(const int32_t* conn, const int64_t* elem_off, const int32_t* etypes,
                                    int64_t n_elem, int32_t n_vert, int32_t* row_ptr, int32_t* cols,
                                    int64_t cols_cap) {
    return mixed_relation(0, conn, elem_off, etypes, n_elem, n_vert, row_ptr, cols, cols_cap);
}

int64_t oracle_mixed_elem_neighbors(const int32_t* conn, const int64_t* elem_off, const int32_t* etypes,
                                    int64_t n_elem, int32_t n_vert, int32_t* row_ptr, int32_t* cols,
                                    int64_t cols_cap) {
    return mixed_relation(1, conn, elem_off, etypes, n_elem, n_vert, row_ptr, cols, cols_cap);
}

/* ---- all-cores variant (for the CPU baseline) ------------------------------
 * The same definition with T threads: thread t owns the vertices
 * [t V / T, (t+1) V / T), scans every element and inserts only into the sets
 * of the vertices it owns, so no set is shared.  Rows are then concatenated
 * in vertex order. */
typedef struct {
    int relation; /* 0 nodes, 1 elements */
    const int32_t* conn;
    int64_t n_elem;
    int npe, n_edges;
    const int (*edges)[2];
    int32_t v0, v1;
    ordered_set* sets; /* sets[v] for v in [v0, v1) */
    int status;
} mt_job;

static void* mt_worker(void* arg) {
    mt_job* j = (mt_job*)arg;
    for (int64_t e = 0; e < j->n_elem && !j->status; ++e) {
        const int32_t* el = j->conn + e * j->npe;
        if (j->relation == 0) {
            for (int k = 0; k < j->n_edges; ++k) {
                int32_t u = el[j->edges[k][0]], w = el[j->edges[k][1]];
                if (u == w) continue;
                if (u >= j->v0 && u < j->v1 && set_insert(&j->sets[u], w)) j->status = -4;
                if (w >= j->v0 && w < j->v1 && set_insert(&j->sets[w], u)) j->status = -4;
            }
        } else {
            for (int q = 0; q < j->npe; ++q) {
                int32_t v = el[q];
                if (v >= j->v0 && v < j->v1 && set_insert(&j->sets[v], (int32_t)e)) j->status = -4;
            }
        }
    }
    return NULL;
}

static int64_t relation_mt(int relation, const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                           int n_threads, int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    int npe, n_edges;
    const int(*edges)[2];
    if (type_info(etype, &npe, &n_edges, &edges) != 0) return -1;
    if (n_elem < 0 || n_vert < 0 || n_elem > INT32_MAX || (n_elem > 0 && !conn) || !row_ptr || n_threads < 1)
        return -1;
    for (int64_t i = 0; i < n_elem * npe; ++i)
        if (conn[i] < 0 || conn[i] >= n_vert) return -2;
    ordered_set* sets = (ordered_set*)calloc((size_t)n_vert + 1, sizeof(ordered_set));
    mt_job* jobs = (mt_job*)calloc((size_t)n_threads, sizeof(mt_job));
    pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!sets || !jobs || !th) {
        free(sets);
        free(jobs);
        free(th);
        return -4;
    }
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        mt_job* j = &jobs[t];
        j->relation = relation;
        j->conn = conn;
        j->n_elem = n_elem;
        j->npe = npe;
        j->n_edges = n_edges;
        j->edges = edges;
        j->v0 = (int32_t)((int64_t)n_vert * t / n_threads);
        j->v1 = (int32_t)((int64_t)n_vert * (t + 1) / n_threads);
        j->sets = sets;
        if (pthread_create(&th[t], NULL, mt_worker, j) != 0) {
            j->status = -4;
            break;
        }
        ++started;
    }
    int64_t r = 0;
    for (int t = 0; t < started; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].status) r = jobs[t].status;
    }
    if (started < n_threads) r = -4;
    if (r == 0) r = emit_csr(sets, n_vert, row_ptr, cols, cols_cap);
    free_sets(sets, n_vert);
    free(jobs);
    free(th);
    return r;
}

int64_t oracle_node_neighbors_mt(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert, int n_threads,
                                 int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    return relation_mt(0, conn, n_elem, etype, n_vert, n_threads, row_ptr, cols, cols_cap);
}

int64_t oracle_elem_neighbors_mt(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert, int n_threads,
                                 int32_t* row_ptr, int32_t* cols, int64_t cols_cap) {
    return relation_mt(1, conn, n_elem, etype, n_vert, n_threads, row_ptr, cols, cols_cap);
}
