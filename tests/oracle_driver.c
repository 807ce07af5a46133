/* Test driver: runs the oracle's entry points on meshes read from a binary
 * file, so that a test can run them in a build with the address and
 * undefined-behaviour sanitizers (a shared library loaded into Python cannot
 * carry them).  Input records, little-endian:
 *   int32 kind (0 one type, 1 mixed, 2 one type on 3 threads), int32 etype,
 *   int32 n_vert, int64 n_elem, int64 n_ids, int32 ids[n_ids], and for mixed
 *   int32 etypes[n_elem].
 * Output per record: for node then element relation, int64 r (the return
 * code), then when r >= 0: int32 row_ptr[n_vert + 1], int32 cols[r]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_node_neighbors(const int32_t*, int64_t, int32_t, int32_t, int32_t*, int32_t*, int64_t);
int64_t oracle_elem_neighbors(const int32_t*, int64_t, int32_t, int32_t, int32_t*, int32_t*, int64_t);
int64_t oracle_node_neighbors_mt(const int32_t*, int64_t, int32_t, int32_t, int, int32_t*, int32_t*, int64_t);
int64_t oracle_elem_neighbors_mt(const int32_t*, int64_t, int32_t, int32_t, int, int32_t*, int32_t*, int64_t);
int64_t oracle_mixed_node_neighbors(const int32_t*, const int64_t*, const int32_t*, int64_t, int32_t, int32_t*,
                                    int32_t*, int64_t);
int64_t oracle_mixed_elem_neighbors(const int32_t*, const int64_t*, const int32_t*, int64_t, int32_t, int32_t*,
                                    int32_t*, int64_t);

static const int NPE[6] = {3, 4, 8, 4, 6, 5};

static void emit(int64_t r, const int32_t* row_ptr, int32_t n_vert, const int32_t* cols) {
    fwrite(&r, sizeof r, 1, stdout);
    if (r >= 0) {
        fwrite(row_ptr, sizeof(int32_t), (size_t)n_vert + 1, stdout);
        fwrite(cols, sizeof(int32_t), (size_t)r, stdout);
    }
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t kind, etype, n_vert;
    int64_t n_elem, n_ids;
    while (fread(&kind, 4, 1, f) == 1) {
        if (fread(&etype, 4, 1, f) != 1 || fread(&n_vert, 4, 1, f) != 1 || fread(&n_elem, 8, 1, f) != 1 ||
            fread(&n_ids, 8, 1, f) != 1)
            return 3;
        int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_ids + 1));
        int32_t* types = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_elem + 1));
        int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_elem + 1));
        if (fread(ids, 4, (size_t)n_ids, f) != (size_t)n_ids) return 3;
        if (kind == 1 && fread(types, 4, (size_t)n_elem, f) != (size_t)n_elem) return 3;
        int64_t cap = 24 * n_elem + 1;
        int32_t* row_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n_vert + 1));
        int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        int64_t r;
        if (kind == 1) {
            off[0] = 0;
            for (int64_t e = 0; e < n_elem; ++e) off[e + 1] = off[e] + (types[e] >= 0 && types[e] < 6 ? NPE[types[e]] : 0);
            r = oracle_mixed_node_neighbors(ids, off, types, n_elem, n_vert, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
            r = oracle_mixed_elem_neighbors(ids, off, types, n_elem, n_vert, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
        } else if (kind == 2) {
            r = oracle_node_neighbors_mt(ids, n_elem, etype, n_vert, 3, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
            r = oracle_elem_neighbors_mt(ids, n_elem, etype, n_vert, 3, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
        } else {
            r = oracle_node_neighbors(ids, n_elem, etype, n_vert, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
            r = oracle_elem_neighbors(ids, n_elem, etype, n_vert, row_ptr, cols, cap);
            emit(r, row_ptr, n_vert, cols);
        }
        free(ids);
        free(types);
        free(off);
        free(row_ptr);
        free(cols);
    }
    fclose(f);
    return 0;
}
