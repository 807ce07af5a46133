// Element types and their edge tables: which node positions of an element are
// joined by an edge.  Two nodes joined by an edge are one-ring neighboring
// nodes of each other (paper Sec. 1, Sec. 2.1.1); the paper demonstrates
// triangles and states that the method applies to any element type (Sec. 2.2,
// Sec. 4).  Node orders are those of VTK.
#pragma once

#include <stdint.h>

#include <utility>

namespace mnb {

enum ElemType : int32_t { TRI3 = 0, TET4 = 1, HEX8 = 2, QUAD4 = 3, WEDGE6 = 4, PYR5 = 5 };
constexpr int N_ELEM_TYPES = 6;
constexpr int MAX_NPE = 8;

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

// Hexahedron (0-1-2-3 bottom face, node i+4 above node i): bottom ring, top
// ring, 4 verticals.  Face and body diagonals are not edges.
template <>
struct Elem<HEX8> {
    static constexpr int NPE = 8, NE = 12;
    static constexpr int A[12] = {0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3};
    static constexpr int B[12] = {1, 2, 3, 0, 5, 6, 7, 4, 4, 5, 6, 7};
};

// Quadrilateral: the 4 sides; the diagonals are not edges.
template <>
struct Elem<QUAD4> {
    static constexpr int NPE = 4, NE = 4;
    static constexpr int A[4] = {0, 1, 2, 3};
    static constexpr int B[4] = {1, 2, 3, 0};
};

// Wedge (triangle 0-1-2, triangle 3-4-5 with node i+3 above node i): the two
// triangle rings and 3 verticals.
template <>
struct Elem<WEDGE6> {
    static constexpr int NPE = 6, NE = 9;
    static constexpr int A[9] = {0, 1, 2, 3, 4, 5, 0, 1, 2};
    static constexpr int B[9] = {1, 2, 0, 4, 5, 3, 3, 4, 5};
};

// Pyramid (quadrilateral base 0-1-2-3, apex 4): the base ring and 4 edges to
// the apex.
template <>
struct Elem<PYR5> {
    static constexpr int NPE = 5, NE = 8;
    static constexpr int A[8] = {0, 1, 2, 3, 0, 1, 2, 3};
    static constexpr int B[8] = {1, 2, 3, 0, 4, 4, 4, 4};
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

// Bit p' of adjacency(p) is set when positions p and p' share an edge.  Eight
// bits per position, packed into one 64-bit word per type.
template <int ET>
constexpr uint64_t adjacency_word() {
    uint64_t w = 0;
    for (int k = 0; k < Elem<ET>::NE; ++k) {
        const int a = Elem<ET>::A[k], b = Elem<ET>::B[k];
        w |= 1ull << (8 * a + b);
        w |= 1ull << (8 * b + a);
    }
    return w;
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
    switch (et) {
        case TRI3: return 3;
        case TET4: return 4;
        case HEX8: return 8;
        case QUAD4: return 4;
        case WEDGE6: return 6;
        case PYR5: return 5;
        default: return 0;
    }
}

__host__ __device__ inline int edges_per_elem(int32_t et) {
    switch (et) {
        case TRI3: return 3;
        case TET4: return 6;
        case HEX8: return 12;
        case QUAD4: return 4;
        case WEDGE6: return 9;
        case PYR5: return 8;
        default: return 0;
    }
}

// Adjacency word of a runtime type (0 for an unknown type).
__host__ __device__ inline uint64_t adjacency_of(int32_t et) {
    switch (et) {
        case TRI3: return adjacency_word<TRI3>();
        case TET4: return adjacency_word<TET4>();
        case HEX8: return adjacency_word<HEX8>();
        case QUAD4: return adjacency_word<QUAD4>();
        case WEDGE6: return adjacency_word<WEDGE6>();
        case PYR5: return adjacency_word<PYR5>();
        default: return 0;
    }
}

// Calls f(std::integral_constant<int, ET>{}) for the runtime type et (which
// the caller has validated).
template <class F>
__host__ __device__ inline decltype(auto) with_type(int32_t et, F&& f) {
    switch (et) {
        case TET4: return f(std::integral_constant<int, TET4>{});
        case HEX8: return f(std::integral_constant<int, HEX8>{});
        case QUAD4: return f(std::integral_constant<int, QUAD4>{});
        case WEDGE6: return f(std::integral_constant<int, WEDGE6>{});
        case PYR5: return f(std::integral_constant<int, PYR5>{});
        default: return f(std::integral_constant<int, TRI3>{});
    }
}

// Element index and position of slot loc of a mesh of nodes-per-element npe,
// with a constant divisor per type.
__device__ __forceinline__ uint32_t slot_elem(uint32_t loc, int npe) {
    switch (npe) {
        case 3: return loc / 3u;
        case 4: return loc >> 2;
        case 5: return loc / 5u;
        case 6: return loc / 6u;
        default: return loc >> 3;
    }
}

}  // namespace mnb
