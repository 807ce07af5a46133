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
 *     of a VTK-ordered hexahedron (the paper demonstrates triangles only,
 *     Sec. 2.2, and claims the method applies to arbitrary meshes);
 *   - ids are 0-based, element id = row of the connectivity array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- per-type element edge tables (node positions inside one element) --- */
static const int TRI_EDGES[3][2] = {{0, 1}, {1, 2}, {2, 0}};
static const int TET_EDGES[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
/* VTK hexahedron: bottom ring 0-1-2-3, top ring 4-5-6-7, verticals i-(i+4). */
static const int HEX_EDGES[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                                     {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

static int type_info(int32_t etype, int* npe, int* n_edges, const int (**edges)[2]) {
    switch (etype) {
        case 0: *npe = 3; *n_edges = 3; *edges = TRI_EDGES; return 0;
        case 1: *npe = 4; *n_edges = 6; *edges = TET_EDGES; return 0;
        case 2: *npe = 8; *n_edges = 12; *edges = HEX_EDGES; return 0;
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
        memcpy(cols + at, sets[v].v, (size_t)sets[v].n * sizeof(int32_t));
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
        const int32_t* el = conn + e * npe;
        for (int k = 0; k < n_edges; ++k) {
            int32_t u = el[edges[k][0]], w = el[edges[k][1]];
            if (u == w) continue; /* no self pair */
            if (set_insert(&sets[u], w) || set_insert(&sets[w], u)) {
                free_sets(sets, n_vert);
                return -4;
            }
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
        const int32_t* el = conn + e * npe;
        for (int j = 0; j < npe; ++j) {
            if (set_insert(&sets[el[j]], (int32_t)e)) {
                free_sets(sets, n_vert);
                return -4;
            }
        }
    }
    int64_t r = emit_csr(sets, n_vert, row_ptr, cols, cols_cap);
    free_sets(sets, n_vert);
    return r;
}
