// Element types and their edge tables: which node positions of an element are
// joined by an edge.  Two nodes joined by an edge are one-ring neighboring
// nodes of each other (paper Sec. 1, Sec. 2.1.1); the paper demonstrates
// triangles and states that the method applies to any element type.
#pragma once

#include <stdint.h>

namespace mnb {

enum ElemType : int32_t { TRI3 = 0, TET4 = 1, HEX8 = 2 };

template <int ET>
struct Elem;

// Triangle: its 3 edges.  Emitting each in both directions gives the six
// integer pairs per triangle of Sec. 2.2.1 (three in CCW and three in CW order).
template <>
struct Elem<TRI3> {
    static constexpr int NPE = 3, NE = 3;
    static constexpr int A[3] = {0, 1, 2};
    static constexpr int B[3] = {1, 2, 0};
};

// Tetrahedron: every pair of its 4 nodes.
template <>
struct Elem<TET4> {
    static constexpr int NPE = 4, NE = 6;
    static constexpr int A[6] = {0, 0, 0, 1, 1, 2};
    static constexpr int B[6] = {1, 2, 3, 2, 3, 3};
};

// Hexahedron in VTK node order (0-1-2-3 bottom face counter-clockwise, node
// i+4 above node i): bottom ring, top ring, 4 verticals.  Face and body
// diagonals are not edges.
template <>
struct Elem<HEX8> {
    static constexpr int NPE = 8, NE = 12;
    static constexpr int A[12] = {0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3};
    static constexpr int B[12] = {1, 2, 3, 0, 5, 6, 7, 4, 4, 5, 6, 7};
};

// The edge tables packed four bits per entry (entry k in bits 4k .. 4k+3),
// so a runtime edge index selects its two nodes with one shift each.
template <int N>
constexpr uint64_t pack_nibbles(const int (&t)[N]) {
    uint64_t r = 0;
    for (int i = 0; i < N; ++i) r |= (uint64_t)t[i] << (4 * i);
    return r;
}

template <int ET>
__device__ __forceinline__ void edge_nodes(int k, int* a, int* b) {
    constexpr uint64_t TA = pack_nibbles(Elem<ET>::A), TB = pack_nibbles(Elem<ET>::B);
    *a = (int)((TA >> (4 * k)) & 15u);
    *b = (int)((TB >> (4 * k)) & 15u);
}

// The ids of element e, read by one thread (consecutive threads read
// consecutive elements, so a wave's loads cover one contiguous span).
template <int ET>
__device__ __forceinline__ void load_elem_ids(const int32_t* __restrict__ conn, int64_t e,
                                              int32_t (&id)[Elem<ET>::NPE]) {
    const int32_t* el = conn + e * Elem<ET>::NPE;
#pragma unroll
    for (int j = 0; j < Elem<ET>::NPE; ++j) id[j] = el[j];
}

__host__ __device__ inline int nodes_per_elem(int32_t et) {
    return et == TRI3 ? 3 : et == TET4 ? 4 : et == HEX8 ? 8 : 0;
}

__host__ __device__ inline int edges_per_elem(int32_t et) {
    return et == TRI3 ? 3 : et == TET4 ? 6 : et == HEX8 ? 12 : 0;
}

}  // namespace mnb
