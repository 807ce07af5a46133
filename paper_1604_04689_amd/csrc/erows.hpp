// Node relation through the element relation (the ELEM_ROWS node algorithm).
//
// Once the element relation is built (the (v, e) pairs counting-sorted by v,
// Sec. 2.2.2), row v of the node relation is the set of vertices joined to v
// by an edge of one of the elements in v's element row: the node pairs of
// Sec. 2.2.1 grouped by their first entry without sorting them, since the
// element sort already grouped every element by each of its nodes.  Each
// row's candidates (the edge-neighbors of v inside each of its elements,
// gathered from the connectivity) are deduplicated and ordered in LDS, which
// gives the ascending, duplicate-free rows of our reading of the serial
// solution (Sec. 3.2.2).  Every tile works alone: its rows' distinct values
// are staged within the rows' own candidate slots (packed back to back) with
// each row's count and offset, the counts are scanned into row_ptr, and the
// staged values gathered into cols.
//
//   erows_prep    per vertex: the first vertex whose element row starts in
//                 each tile of ER_TILE element-CSR entries; rows longer than
//                 ER_ROW_MAX entries listed
//   erows_long    one block per listed row: candidates to the stage, sorted
//                 and deduplicated there (block_sort_unique), count written
//   erows_tile    one block per tile: the rows that start in the tile,
//                 candidates into LDS hash tables spanning each row's own
//                 candidate slots, distinct values compacted and ordered by
//                 counting, written to the stage with the row counts and
//                 offsets (a batch: tiles sorted into lists by element type
//                 first, erows_classify, each list with its type's access)
//   erows_scan    counts -> row_ptr (decoupled look-back scan)
//   erows_gather  stage -> cols, coalesced
#pragma once

#include <climits>
#include <cstdio>

#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "rows.hpp"

namespace mnb {

constexpr int ER_BLOCK = 256;
constexpr int ER_TILE = 1024;    // element-CSR entries whose rows one block owns
constexpr int ER_ROW_MAX = 256;  // longest element row (entries) handled in LDS
constexpr int ER_SPAN = ER_TILE + ER_ROW_MAX;
constexpr int ER_EPT = ER_SPAN / ER_BLOCK;  // entry positions per thread
constexpr int ER_LONG_GRID = 256;
constexpr int ER_PREP_BLOCK = 256;
constexpr uint32_t CAND_NONE = SLOT_EMPTY;
constexpr int TK_EROWS = 12;  // ticket slot of erows_tile in the workspace header
static_assert(ER_SPAN % ER_BLOCK == 0, "whole positions per thread");
static_assert(ER_TILE % 32 == 0 && ER_TILE / 32 <= WAVE, "row-start bitmap words, scanned by one wave");
static_assert(ER_BLOCK == LONG_BLOCK, "long rows share block_sort_unique");

// The edge-neighbors of vertex v inside one element with ids[0 .. npe) and
// adjacency word adj (bit 8p + q: positions p and q share an edge).  Slot s
// stands for position s before pv, the first position holding v, and for
// position s + 1 from there on; it holds that position's id when the
// position is joined by an edge to some position holding v and its id is
// another vertex in [0, n_vert), else CAND_NONE.  Returns false if v is not
// in the element.
template <int NPE>
__device__ __forceinline__ bool elem_cands(const int32_t (&ids)[NPE], int npe, uint64_t adj, int32_t v,
                                           int32_t n_vert, uint32_t (&c)[NPE - 1]) {
    uint32_t vmask = 0;
#pragma unroll
    for (int p = 0; p < NPE; ++p) vmask |= (uint32_t)(p < npe && ids[p] == v) << p;
    const int pv = vmask ? __builtin_ctz(vmask) : NPE;
#pragma unroll
    for (int s = 0; s < NPE - 1; ++s) {
        const bool after = s >= pv;
        const int q = s + (after ? 1 : 0);
        const int32_t w = after ? ids[s + 1] : ids[s];
        const bool ok = q < npe && w != v && (uint32_t)w < (uint32_t)n_vert && ((adj >> (8 * q)) & vmask) != 0;
        c[s] = ok ? (uint32_t)w : CAND_NONE;
    }
    return vmask != 0;
}

// Element access.  The candidates of one element-CSR entry (row vertex v,
// element e) come in three steps, so that a thread can issue the loads of all
// its entries before it waits for any of them (the gathers from conn are
// random accesses; one round trip per entry would leave the kernel waiting on
// memory latency):
//   locate(ctx, v, e, in) -> Loc   where e's ids are and its type (loads only
//                                  what that needs: nothing for one element
//                                  type, the offsets for mixed types, the
//                                  segment record for a batch)
//   fetch(loc, ids)                the ids (loads only where loc.ok)
//   cands(loc, ids, v, c, bad)     the candidates; *bad when the entry is in a
//                                  row but e is not an element or v not in it
// `in` is false for positions outside every short row: no loads, no
// candidates, no error.

// A mesh of one type: element e's ids at conn + e * NPE.  Row index r stands
// for vertex r + v0 (v0 = 0 unless the rows are one vertex range of a
// bounded-memory build).
template <int ET>
struct UniformRows {
    static constexpr int NPE = Elem<ET>::NPE;
    static constexpr int S = NPE - 1;
    static constexpr int IDS = NPE;
    static constexpr bool kCtx = false;
    const int32_t* __restrict__ conn;
    int64_t n_elem;
    int32_t n_vert;
    int32_t v0 = 0;
    struct Loc {
        uint32_t e;
        bool ok, bad;
    };
    __device__ __forceinline__ int32_t ctx(int32_t) const { return 0; }
    __device__ __forceinline__ int32_t ctx_from(int32_t, int32_t) const { return 0; }
    __device__ __forceinline__ Loc locate(int32_t, int32_t, int32_t e, bool in) const {
        const bool valid = (uint64_t)(uint32_t)e < (uint64_t)n_elem;
        return Loc{(uint32_t)e, in && valid, in && !valid};
    }
    __device__ __forceinline__ void fetch(const Loc& l, int32_t (&ids)[IDS]) const {
        if (l.ok) {
            const int32_t* el = conn + (size_t)l.e * NPE;
#pragma unroll
            for (int j = 0; j < NPE; ++j) ids[j] = el[j];
        } else {
#pragma unroll
            for (int j = 0; j < NPE; ++j) ids[j] = -1;
        }
    }
    __device__ __forceinline__ void cands(const Loc& l, const int32_t (&ids)[IDS], int32_t v, uint32_t (&c)[S],
                                          bool* bad) const {
        *bad |= l.bad;
        if (!l.ok) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            return;
        }
        *bad |= !elem_cands<NPE>(ids, NPE, adjacency_word<ET>(), v + v0, n_vert, c);
    }
};

// Candidates from up to MAX_NPE ids of an element of runtime type et.
__device__ __forceinline__ bool runtime_cands(const int32_t (&ids)[MAX_NPE], int32_t et, int32_t v, int32_t n_vert,
                                              uint32_t (&c)[MAX_NPE - 1]) {
    return elem_cands<MAX_NPE>(ids, nodes_per_elem(et), adjacency_of(et), v, n_vert, c);
}

// Up to MAX_NPE ids at el, the first npe of them loaded (the rest -1).
__device__ __forceinline__ void fetch_runtime(const int32_t* __restrict__ el, int npe, bool ok,
                                              int32_t (&ids)[MAX_NPE]) {
#pragma unroll
    for (int j = 0; j < MAX_NPE; ++j) ids[j] = -1;
    if (ok) {
#pragma unroll
        for (int j = 0; j < MAX_NPE; ++j)
            if (j < npe) ids[j] = el[j];
    }
}

// A mesh whose elements carry their own types: element e has type etypes[e]
// and ids conn[elem_off[e] .. elem_off[e+1]).
struct MixedRows {
    static constexpr int S = MAX_NPE - 1;
    static constexpr int IDS = MAX_NPE;
    static constexpr bool kCtx = false;
    const int32_t* __restrict__ conn;
    const int32_t* __restrict__ elem_off;
    const uint8_t* __restrict__ etypes;
    int64_t n_elem, n_ids;
    int32_t n_vert;
    struct Loc {
        int32_t a, et;
        bool ok, bad;
    };
    __device__ __forceinline__ int32_t ctx(int32_t) const { return 0; }
    __device__ __forceinline__ int32_t ctx_from(int32_t, int32_t) const { return 0; }
    __device__ __forceinline__ Loc locate(int32_t, int32_t, int32_t e, bool in) const {
        Loc l{0, 0, false, false};
        if (!in) return l;
        bool ok = (uint64_t)(uint32_t)e < (uint64_t)n_elem;
        if (ok) {
            l.a = elem_off[e];
            const int32_t b = elem_off[e + 1];
            l.et = etypes[e];
            const int npe = nodes_per_elem(l.et);
            ok = npe > 0 && l.a >= 0 && b - l.a == npe && (int64_t)b <= n_ids;
        }
        l.ok = ok;
        l.bad = !ok;
        return l;
    }
    __device__ __forceinline__ void fetch(const Loc& l, int32_t (&ids)[IDS]) const {
        fetch_runtime(conn + (l.ok ? l.a : 0), nodes_per_elem(l.et), l.ok, ids);
    }
    __device__ __forceinline__ void cands(const Loc& l, const int32_t (&ids)[IDS], int32_t v, uint32_t (&c)[S],
                                          bool* bad) const {
        *bad |= l.bad;
        if (!l.ok) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            return;
        }
        *bad |= !runtime_cands(ids, l.et, v, n_vert, c);
    }
};

// The mesh of global vertex v in a batch: the last segment with vert_off <=
// v (vert_off non-decreasing), by binary search.
__device__ __forceinline__ int32_t batch_mesh_of(const mesh_segment* __restrict__ segs, int32_t n_mesh, int32_t v) {
    int lo = 0, hi = n_mesh - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].vert_off <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
// The mesh of v >= the first vertex of mesh m0: walk forward from m0 (a
// tile's rows span few meshes, so this is a step or two, not a search).
__device__ __forceinline__ int32_t batch_mesh_from(const mesh_segment* __restrict__ segs, int32_t n_mesh, int32_t m0,
                                                   int32_t v) {
    int32_t m = m0 < 0 ? 0 : m0;
    while (m + 1 < n_mesh && segs[m + 1].vert_off <= v) ++m;
    return m;
}

// A batch: row vertex v is global; its mesh is the last segment with
// vert_off <= v, its element ids are local to that mesh and so are the
// candidates.  ctx(v) is the mesh index.  Any element type per mesh.
struct BatchRows {
    static constexpr int S = MAX_NPE - 1;
    static constexpr int IDS = MAX_NPE;
    static constexpr bool kCtx = true;
    const int32_t* __restrict__ conn;
    const mesh_segment* __restrict__ segs;
    int32_t n_mesh;
    struct Loc {
        int64_t off;  // first id of the element in conn
        int32_t et, vl, nv;
        bool ok, bad;
    };
    __device__ __forceinline__ int32_t ctx(int32_t v) const { return batch_mesh_of(segs, n_mesh, v); }
    __device__ __forceinline__ int32_t ctx_from(int32_t m0, int32_t v) const {
        return batch_mesh_from(segs, n_mesh, m0, v);
    }
    __device__ __forceinline__ Loc locate(int32_t m, int32_t v, int32_t e, bool in) const {
        Loc l{0, 0, 0, 0, false, false};
        if (!in) return l;
        const mesh_segment& sg = segs[m];
        const int npe = nodes_per_elem(sg.etype);
        l.et = sg.etype;
        l.vl = v - sg.vert_off;
        l.nv = sg.n_vert;
        l.ok = npe > 0 && (uint64_t)(uint32_t)e < (uint64_t)sg.n_elem && l.vl >= 0 && l.vl < sg.n_vert;
        l.bad = !l.ok;
        l.off = l.ok ? sg.conn_off + (int64_t)e * npe : 0;
        return l;
    }
    __device__ __forceinline__ void fetch(const Loc& l, int32_t (&ids)[IDS]) const {
        fetch_runtime(conn + l.off, nodes_per_elem(l.et), l.ok, ids);
    }
    __device__ __forceinline__ void cands(const Loc& l, const int32_t (&ids)[IDS], int32_t, uint32_t (&c)[S],
                                          bool* bad) const {
        *bad |= l.bad;
        if (!l.ok) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            return;
        }
        *bad |= !runtime_cands(ids, l.et, l.vl, l.nv, c);
    }
};

// A batch whose rows (those of one tile) all belong to meshes of element type
// ET: the same access as BatchRows with the type's own candidate slots (S =
// npe - 1 instead of the largest type's), so a tile of triangles or
// tetrahedra keeps its registers and LDS tables to its own size.  An entry of
// a mesh of another type is an error (the tile lists never send one here).
template <int ET>
struct BatchTypedRows {
    static constexpr int NPE = Elem<ET>::NPE;
    static constexpr int S = NPE - 1;
    static constexpr int IDS = NPE;
    static constexpr bool kCtx = true;
    const int32_t* __restrict__ conn;
    const mesh_segment* __restrict__ segs;
    int32_t n_mesh;
    struct Loc {
        int64_t off;
        int32_t vl, nv;
        bool ok, bad;
    };
    __device__ __forceinline__ int32_t ctx(int32_t v) const { return batch_mesh_of(segs, n_mesh, v); }
    __device__ __forceinline__ int32_t ctx_from(int32_t m0, int32_t v) const {
        return batch_mesh_from(segs, n_mesh, m0, v);
    }
    __device__ __forceinline__ Loc locate(int32_t m, int32_t v, int32_t e, bool in) const {
        Loc l{0, 0, 0, false, false};
        if (!in) return l;
        const mesh_segment& sg = segs[m];
        l.vl = v - sg.vert_off;
        l.nv = sg.n_vert;
        l.ok = sg.etype == ET && (uint64_t)(uint32_t)e < (uint64_t)sg.n_elem && l.vl >= 0 && l.vl < sg.n_vert;
        l.bad = !l.ok;
        l.off = l.ok ? sg.conn_off + (int64_t)e * NPE : 0;
        return l;
    }
    __device__ __forceinline__ void fetch(const Loc& l, int32_t (&ids)[IDS]) const {
        if (l.ok) {
            const int32_t* el = conn + l.off;
#pragma unroll
            for (int j = 0; j < NPE; ++j) ids[j] = el[j];
        } else {
#pragma unroll
            for (int j = 0; j < NPE; ++j) ids[j] = -1;
        }
    }
    __device__ __forceinline__ void cands(const Loc& l, const int32_t (&ids)[IDS], int32_t, uint32_t (&c)[S],
                                          bool* bad) const {
        *bad |= l.bad;
        if (!l.ok) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            return;
        }
        *bad |= !elem_cands<NPE>(ids, NPE, adjacency_word<ET>(), l.vl, l.nv, c);
    }
};

// All three steps for one entry (long rows, one entry per thread at a time).
template <class Acc>
__device__ __forceinline__ void entry_cands(const Acc& acc, int32_t cx, int32_t v, int32_t e, bool in,
                                            uint32_t (&c)[Acc::S], bool* bad) {
    const typename Acc::Loc l = acc.locate(cx, v, e, in);
    int32_t ids[Acc::IDS];
    acc.fetch(l, ids);
    acc.cands(l, ids, v, c, bad);
}

// Element row length of vertex v, 0 (and *bad) when the row pointers are not
// a valid CSR there.
__device__ __forceinline__ int32_t erow_len(const int32_t* __restrict__ erp, int32_t v, int64_t q, int32_t* a,
                                            bool* bad) {
    const int32_t x = erp[v], y = erp[v + 1];
    if (x < 0 || y < x || (int64_t)y > q) {
        *bad = true;
        *a = 0;
        return 0;
    }
    *a = x;
    return y - x;
}

// Distinct count of long row v (written by erows_long), never more than the
// row's candidate slots (an invalid element CSR aside, it never is).
__device__ __forceinline__ int64_t long_count(const int32_t* __restrict__ ldeg, int32_t v, int32_t len, int slots) {
    return tmin<int64_t>((uint32_t)ldeg[v], (int64_t)slots * len);
}

// erp[n_vert] clamped to the host's bound of the element nnz.
__device__ __forceinline__ int64_t erow_total(const int32_t* __restrict__ erp, int32_t n_vert, int64_t q_bound) {
    const int64_t q = erp[n_vert];
    return q < 0 ? 0 : (q > q_bound ? q_bound : q);
}

// tile_first[t] = first vertex v (in [0, n_vert], n_vert standing for "none")
// whose element row starts at or after t * ER_TILE, and tile_ctx[t] its
// accessor context (the mesh of v in a batch; found once per tile here)
// whose element row starts at or after t * ER_TILE; rows longer than
// ER_ROW_MAX entries go to the long list.  One thread per v in [0, n_vert].
template <class Acc>
__global__ __launch_bounds__(ER_PREP_BLOCK) void erows_prep_kernel(Acc acc, const int32_t* __restrict__ erp,
                                                                         int32_t n_vert, int64_t q_bound,
                                                                         int32_t* __restrict__ tile_first,
                                                                         int32_t* __restrict__ tile_ctx,
                                                                         int64_t n_tiles_bound,
                                                                         int32_t* __restrict__ long_list,
                                                                         int64_t long_cap, uint32_t* long_count,
                                                                         uint32_t* err) {
    const int64_t v = (int64_t)blockIdx.x * ER_PREP_BLOCK + threadIdx.x;
    if (v > n_vert) return;
    const int64_t q = erow_total(erp, n_vert, q_bound);
    const int64_t prev = v > 0 ? tmin<int64_t>(tmax<int64_t>(erp[v - 1], -1), q) : -1;
    const int64_t cur = v < n_vert ? tmin<int64_t>(tmax<int64_t>(erp[v], 0), q) : q;
    // tiles t with prev < t * ER_TILE <= cur
    const int64_t t0 = (prev + ER_TILE) / ER_TILE, t1 = tmin<int64_t>(cur / ER_TILE, n_tiles_bound - 1);
    if (t0 <= t1) {
        const int32_t cx = Acc::kCtx && v < n_vert ? acc.ctx((int32_t)v) : 0;
        for (int64_t t = t0; t <= t1; ++t) {
            tile_first[t] = (int32_t)v;
            tile_ctx[t] = cx;
        }
    }
    if (v < n_vert) {
        int32_t a;
        bool bad = false;
        const int32_t len = erow_len(erp, (int32_t)v, q, &a, &bad);
        if (bad) set_error(err, ERR_INTERNAL);
        if (len > ER_ROW_MAX) {
            const uint32_t slot = atomicAdd(long_count, 1u);
            if ((int64_t)slot < long_cap) long_list[slot] = (int32_t)v;
            else set_error(err, ERR_INTERNAL);
        }
    }
}

// Long rows: one block per listed row.  Its candidates go to
// temp[S * a .. S * (a + len)) (CAND_NONE as INT_MAX, which never is an id),
// are sorted and deduplicated there; ldeg[v] = the distinct count.
template <class Acc>
__global__ __launch_bounds__(ER_BLOCK) void erows_long_kernel(Acc acc, const int32_t* __restrict__ erp,
                                                             const int32_t* __restrict__ ecols, int32_t n_vert,
                                                             int64_t q_bound, int64_t ecap,
                                                             const int32_t* __restrict__ long_list,
                                                             int64_t long_cap, const uint32_t* long_count,
                                                             int32_t* __restrict__ ldeg,
                                                             int16_t* __restrict__ soff, int32_t* temp,
                                                             uint32_t* err) {
    constexpr int S = Acc::S;
    __shared__ int32_t s[LONG_LDS];
    __shared__ uint32_t s_wcnt[LONG_BLOCK / WAVE];
    const int tid = threadIdx.x;
    const int64_t n_long = tmin<int64_t>(*long_count, long_cap);
    const int64_t q = erow_total(erp, n_vert, q_bound);
    const int64_t qe = tmin<int64_t>(q, ecap);
    bool bad = false;
    for (int64_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const int32_t v = long_list[li];
        int32_t a;
        const int32_t len = erow_len(erp, v, q, &a, &bad);
        const int32_t cx = acc.ctx(v);
        int32_t* x = temp + (int64_t)S * a;
        for (int64_t i = tid; i < len; i += ER_BLOCK) {
            const int64_t p = a + i;
            uint32_t c[S];
            entry_cands(acc, cx, v, p < qe ? ecols[p] : 0, p < qe, c, &bad);
#pragma unroll
            for (int k = 0; k < S; ++k) x[S * i + k] = c[k] == CAND_NONE ? INT_MAX : (int32_t)c[k];
        }
        __threadfence_block();
        __syncthreads();
        const int64_t cnt = block_sort_unique(x, (int64_t)S * len, s, s_wcnt);
        if (tid == 0) {
            ldeg[v] = (int32_t)cnt;
            soff[v] = 0;
        }
        __syncthreads();
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// The node rows from the element CSR, one tile of ER_TILE entries per block,
// independently of every other tile.  A block owns the vertices whose element
// row starts in its tile.  Entry position r of the tile (0 <= r < ER_SPAN,
// entry base + r) sits in register slot r / ER_BLOCK of thread r % ER_BLOCK,
// with its S candidates.  Row v's distinct values go, ascending, to
// stage[P * a .. P * a + cnt[v]) (a = the row's first entry, P = stage_slots
// >= S: the S candidate slots per entry always have room), and cnt[v] is written for every owned
// vertex except the long rows (erows_long writes theirs).
//
// The work of a tile is a chain of memory round trips and barriers, kept
// short: the element ids of the first ER_TILE + WAVE positions are loaded,
// and for an accessor that needs no row context their connectivity gathered,
// while the owned rows are being listed; every candidate is offered to its
// row's table in one round of LDS atomics (the few that collide probe on).
// With no offset to wait for, no tile waits for another.
template <class Acc>
__device__ __forceinline__ void erows_tile_body(const Acc& acc, const int32_t* __restrict__ erp,
                                                const int32_t* __restrict__ ecols, int32_t n_vert, int64_t q_bound,
                                                int64_t ecap, const int32_t* __restrict__ tile_first,
                                                const int32_t* __restrict__ tile_ctx, int32_t* __restrict__ cnt,
                                                int16_t* __restrict__ soff, int32_t* __restrict__ stage,
                                                int stage_slots, uint32_t* err, int64_t t) {
    constexpr int S = Acc::S;
    constexpr int CAP = ER_SPAN * S;
    constexpr int WAVES = ER_BLOCK / WAVE;
    constexpr bool kEarly = !Acc::kCtx;  // ids gathered before the rows are known
    static_assert(CAP < INT16_MAX, "16-bit dense indices");
    // per-row hash tables over each row's own candidate slots; once every
    // insertion is done, the same words hold the distinct values, dense, in
    // slot order (each row's values contiguous); 4 words of padding for the
    // unrolled rank loop
    __shared__ uint32_t s_tab[CAP + 4];
    __shared__ int16_t s_ra[ER_TILE];    // short row k: first entry, relative to the tile base
    __shared__ int16_t s_rlen[ER_TILE];  // entries
    __shared__ int16_t s_rds[ER_TILE];   // dense range of its distinct values
    __shared__ int16_t s_rde[ER_TILE];
    __shared__ int32_t s_rv[ER_TILE];    // vertex
    __shared__ int32_t s_rctx[Acc::kCtx ? ER_TILE : 1];
    __shared__ uint32_t s_wtot[ER_EPT][WAVES];
    __shared__ uint32_t s_tmp[WAVES];
    // row starts as a bitmap: bit j of word w (.x) set where a short row
    // starts at entry 32w + j; .y the short rows starting in earlier words
    __shared__ uint2 s_rmap[ER_TILE / 32];

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t q = erow_total(erp, n_vert, q_bound);
    const int64_t n_tiles = q / ER_TILE + 1;
    if (t >= n_tiles) return;  // owns nothing
    for (int i = tid; i < CAP + 4; i += ER_BLOCK) s_tab[i] = SLOT_EMPTY;
    for (int i = tid; i < ER_TILE / 32; i += ER_BLOCK) s_rmap[i].x = 0;
    const int64_t base = t * ER_TILE;
    const bool last_tile = t == n_tiles - 1;
    const int64_t qe = tmin<int64_t>(q, ecap);
    const int64_t in_end = tmin<int64_t>(qe - base, ER_SPAN);  // entry positions that can be read
    bool bad = false;

    // ---- element ids of every readable position; for the positions below
    // ER_TILE + WAVE (the first halo slots hold the rest of the tile's last
    // row, which almost always runs past ER_TILE and is seldom longer than a
    // wave's worth of entries) their elements' ids too, owned row or not
    int32_t ent[ER_EPT];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int r = i * ER_BLOCK + tid;
        ent[i] = r < in_end ? ecols[base + r] : 0;
    }
    int32_t v_first = tile_first[t];
    int32_t v_end = last_tile ? n_vert : tile_first[t + 1];
    v_first = tmin<int32_t>(tmax<int32_t>(v_first, 0), n_vert);
    v_end = tmin<int32_t>(tmax<int32_t>(v_end, v_first), n_vert);
    const int32_t ctx0 = Acc::kCtx ? tile_ctx[t] : 0;
    auto early = [&](int i) { return kEarly && i * ER_BLOCK + tid < ER_TILE + WAVE; };
    typename Acc::Loc loc[ER_EPT];
    int32_t ids[ER_EPT][Acc::IDS];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        if (early(i)) {
            const int r = i * ER_BLOCK + tid;
            loc[i] = acc.locate(0, 0, ent[i], r < in_end);
            acc.fetch(loc[i], ids[i]);
        }
    }

    // ---- the owned vertices' rows: short non-empty rows listed in LDS; empty
    // rows get their count (0) here
    int32_t nrows = 0;
    for (int32_t c0 = v_first; c0 < v_end; c0 += ER_BLOCK) {
        const int32_t v = c0 + tid;
        int32_t a = 0, len = 0;
        if (v < v_end) len = erow_len(erp, v, q, &a, &bad);
        if (len > 0 && (a < base || a >= base + ER_TILE)) {  // not owned: only on an invalid CSR
            bad = true;
            len = 0;
        }
        if (v < v_end && len == 0) {
            cnt[v] = 0;
            soff[v] = 0;
        }
        const bool is_short = len > 0 && len <= ER_ROW_MAX;
        uint32_t total;
        const uint32_t k = (uint32_t)nrows + block_exclusive_sum<ER_BLOCK>((uint32_t)is_short, s_tmp, &total);
        if (is_short && k < (uint32_t)ER_TILE) {
            s_ra[k] = (int16_t)(a - base);
            s_rlen[k] = (int16_t)len;
            s_rv[k] = v;
            atomicOr(&s_rmap[(a - base) >> 5].x, 1u << ((a - base) & 31));
            s_rds[k] = 0;
            s_rde[k] = 0;
            if constexpr (Acc::kCtx) s_rctx[k] = acc.ctx_from(ctx0, v);
        }
        nrows += (int32_t)total;
    }
    if (nrows > ER_TILE) {  // distinct row starts in the tile: only on an invalid CSR
        bad = true;
        nrows = ER_TILE;
    }
    __syncthreads();
    if (tid < WAVE) {
        const uint32_t c = lane < ER_TILE / 32 ? (uint32_t)__popc(s_rmap[lane].x) : 0u;
        const uint32_t inc = wave_inclusive_sum(c);
        if (lane < ER_TILE / 32) s_rmap[lane].y = inc - c;
    }
    // the short rows' values go to the stage back to back from the first
    // short row's slots on (the gather then reads them densely), unless a
    // long row lies between two of them (its values take its own slots)
    bool gap = false;
    for (int k = 1 + tid; k < nrows; k += ER_BLOCK) gap |= s_ra[k - 1] + s_rlen[k - 1] != s_ra[k];
    const bool dense = !__syncthreads_or(gap);

    // ---- the row of every position (the last short row starting at or
    // before it: the row starts counted in the bitmap up to it; past the
    // tile, the last row), then the ids not gathered yet, then the candidates
    uint32_t cand[ER_EPT][S];
    int32_t rowk[ER_EPT];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int r = i * ER_BLOCK + tid;
        int lo = nrows - 1;
        if (r < ER_TILE) {
            const uint2 m = s_rmap[r >> 5];
            lo = tmin<int>((int)m.y + __popc(m.x & (0xffffffffu >> (31 - (r & 31)))) - 1, lo);
        }
        const int lk = lo < 0 ? 0 : lo;
        const bool in = lo >= 0 && s_ra[lk] <= r && r < s_ra[lk] + s_rlen[lk] && r < in_end;
        rowk[i] = in ? lo : -1;
    }
    int32_t rv[ER_EPT];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int k = rowk[i] >= 0 ? rowk[i] : 0;
        rv[i] = s_rv[k];
        if (!early(i)) loc[i] = acc.locate(Acc::kCtx ? s_rctx[k] : 0, rv[i], ent[i], rowk[i] >= 0);
    }
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i)
        if (!early(i)) acc.fetch(loc[i], ids[i]);
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        // a position outside every owned row contributes nothing (its early
        // gather, if any, is dropped; a bad element there is not ours to report)
        if (rowk[i] < 0) loc[i] = acc.locate(0, 0, 0, false);
        acc.cands(loc[i], ids[i], rv[i], cand[i], &bad);
    }

    // ---- offer every candidate to its row's table (open addressing over the
    // row's own slots): one round of atomics for all of them, then linear
    // probing for the few whose first slot held another value.  The insertion
    // that fills an empty slot keeps the value.
    uint64_t kept = 0;
    {
        uint32_t old[ER_EPT][S];
#pragma unroll
        for (int i = 0; i < ER_EPT; ++i) {
            const int k = rowk[i] >= 0 ? rowk[i] : 0;
            const uint32_t t0 = (uint32_t)S * (uint32_t)s_ra[k];
            const uint32_t len = (uint32_t)S * (uint32_t)s_rlen[k];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const uint32_t w = cand[i][s];
                old[i][s] = w;  // settled unless offered below
                if (rowk[i] >= 0 && w != CAND_NONE)
                    old[i][s] = atomicCAS(&s_tab[t0 + (uint32_t)(((uint64_t)(w * 2654435761u) * len) >> 32)],
                                          SLOT_EMPTY, w);
            }
        }
#pragma unroll
        for (int i = 0; i < ER_EPT; ++i) {
            const int k = rowk[i] >= 0 ? rowk[i] : 0;
            const uint32_t t0 = (uint32_t)S * (uint32_t)s_ra[k];
            const uint32_t len = (uint32_t)S * (uint32_t)s_rlen[k];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const uint32_t w = cand[i][s];
                if (rowk[i] < 0 || w == CAND_NONE) continue;
                if (old[i][s] == SLOT_EMPTY) {
                    kept |= 1ull << (i * S + s);
                    continue;
                }
                if (old[i][s] == w) continue;
                uint32_t h = (uint32_t)(((uint64_t)(w * 2654435761u) * len) >> 32);
                for (uint32_t probe = 1; probe < len; ++probe) {
                    h = h + 1 == len ? 0 : h + 1;
                    const uint32_t o = atomicCAS(&s_tab[t0 + h], SLOT_EMPTY, w);
                    if (o == SLOT_EMPTY) {
                        kept |= 1ull << (i * S + s);
                        break;
                    }
                    if (o == w) break;
                }
            }
        }
    }
    // ---- dense list of the kept values in slot order (entry order, then
    // slot); each row's distinct values [rds, rde)
    uint32_t excl[ER_EPT];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const uint32_t c = (uint32_t)__popcll((kept >> (i * S)) & ((1ull << S) - 1));
        const uint32_t incl = wave_inclusive_sum(c);
        excl[i] = incl - c;
        if (lane == WAVE - 1) s_wtot[i][wid] = incl;
    }
    __syncthreads();  // every insertion is done: the tables may be overwritten
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        uint32_t off = excl[i];
#pragma unroll
        for (int ii = 0; ii < ER_EPT; ++ii)
#pragma unroll
            for (int w = 0; w < WAVES; ++w) off += (ii < i || (ii == i && w < wid)) ? s_wtot[ii][w] : 0u;
        excl[i] = off;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int r = i * ER_BLOCK + tid;
        const int k = rowk[i];
        uint32_t d = excl[i];
        if (k >= 0 && r == s_ra[k]) s_rds[k] = (int16_t)d;
#pragma unroll
        for (int s = 0; s < S; ++s)
            if ((kept >> (i * S + s)) & 1ull) s_tab[d++] = cand[i][s];
        // the row's last entry that can be read closes its range
        if (k >= 0 && r == tmin<int64_t>(s_ra[k] + s_rlen[k], in_end) - 1) s_rde[k] = (int16_t)d;
    }
    __syncthreads();

    // ---- counts of the short rows, and each kept value to its place: the
    // number of its row's distinct values below it
    // (dense: row k's values at P * (base + s_ra[0]) + s_rds[k], P =
    // stage_slots; soff[v] = that minus P * (row start), the gather's offset;
    // the rows' values fit the rows' own slots, S <= P per entry)
    for (int k = tid; k < nrows; k += ER_BLOCK) {
        cnt[s_rv[k]] = tmax<int32_t>(s_rde[k] - s_rds[k], 0);
        soff[s_rv[k]] = dense ? (int16_t)(s_rds[k] - stage_slots * (s_ra[k] - s_ra[0])) : (int16_t)0;
    }
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        if (rowk[i] < 0) continue;
        const int k = rowk[i];
        const int ds = s_rds[k], de = s_rde[k];
        int32_t* row = dense ? stage + (int64_t)stage_slots * (base + s_ra[0]) + ds
                             : stage + (int64_t)stage_slots * (base + s_ra[k]);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (!((kept >> (i * S + s)) & 1ull)) continue;
            const uint32_t w = cand[i][s];
            int n = 0;
            for (int x = ds; x < de; x += 4) {  // padding past de reads SLOT_EMPTY or other rows' values
                const uint32_t a0 = s_tab[x], a1 = s_tab[x + 1], a2 = s_tab[x + 2], a3 = s_tab[x + 3];
                n += (a0 < w) + (x + 1 < de && a1 < w) + (x + 2 < de && a2 < w) + (x + 3 < de && a3 < w);
            }
            row[n] = (int32_t)w;  // n < distinct count <= S * (row entries)
        }
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// One tile per block: tile blockIdx.x.
template <class Acc>
__global__ __launch_bounds__(ER_BLOCK) void erows_tile_kernel(Acc acc, const int32_t* __restrict__ erp,
                                                             const int32_t* __restrict__ ecols, int32_t n_vert,
                                                             int64_t q_bound, int64_t ecap,
                                                             const int32_t* __restrict__ tile_first,
                                                             const int32_t* __restrict__ tile_ctx,
                                                             int32_t* __restrict__ cnt, int16_t* __restrict__ soff,
                                                             int32_t* __restrict__ stage, uint32_t* err) {
    erows_tile_body(acc, erp, ecols, n_vert, q_bound, ecap, tile_first, tile_ctx, cnt, soff, stage, Acc::S, err,
                    (int64_t)blockIdx.x);
}

// The tiles of a list (list[0 .. *count)), the blocks taking them in turn.
template <class Acc>
__global__ __launch_bounds__(ER_BLOCK) void erows_tile_list_kernel(Acc acc, const int32_t* __restrict__ erp,
                                                                  const int32_t* __restrict__ ecols, int32_t n_vert,
                                                                  int64_t q_bound, int64_t ecap,
                                                                  const int32_t* __restrict__ tile_first,
                                                                  const int32_t* __restrict__ tile_ctx,
                                                                  int32_t* __restrict__ cnt,
                                                                  int16_t* __restrict__ soff,
                                                                  int32_t* __restrict__ stage, int stage_slots,
                                                                  uint32_t* err, const int32_t* __restrict__ list,
                                                                  const uint32_t* count) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        erows_tile_body(acc, erp, ecols, n_vert, q_bound, ecap, tile_first, tile_ctx, cnt, soff, stage, stage_slots,
                        err, (int64_t)list[i]);
        __syncthreads();  // the next tile rewrites the LDS tables
    }
}

// cols[row_ptr[v] + i] = stage[S * erp[v] + soff[v] + i] for i < cnt[v] =
// row_ptr[v+1] - row_ptr[v].  A block covers EG_BLOCK consecutive vertices;
// their output range is contiguous, so consecutive threads take consecutive outputs
// (coalesced writes), each finding its row by a fixed-step binary search over
// the block's row starts in LDS, four outputs per thread at a time.
constexpr int EG_BLOCK = 256;
constexpr int EG_UNROLL = 4;

static __global__ __launch_bounds__(EG_BLOCK) void erows_gather_kernel(const int32_t* __restrict__ row_ptr,
                                                                      const int32_t* __restrict__ erp,
                                                                      const int16_t* __restrict__ soff, int slots,
                                                                      const int32_t* __restrict__ stage,
                                                                      int32_t n_vert, int64_t q_bound,
                                                                      int32_t* __restrict__ cols, int64_t cols_cap,
                                                                      uint32_t* err) {
    __shared__ int32_t s_start[EG_BLOCK + 1];
    __shared__ int64_t s_src[EG_BLOCK];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * EG_BLOCK;
    const int nv = (int)tmin<int64_t>(EG_BLOCK, (int64_t)n_vert - v0);
    bool bad = false;
    if (tid < nv) {
        const int32_t a = erp[v0 + tid], b = erp[v0 + tid + 1];
        const int32_t r0 = row_ptr[v0 + tid], r1 = row_ptr[v0 + tid + 1];
        const int32_t so = soff[v0 + tid];
        // a row holds at most its candidate slots, inside the element CSR;
        // its values start at or before its own slots (packed rows move down)
        const bool ok = a >= 0 && b >= a && (int64_t)b <= q_bound && r1 - r0 >= 0 &&
                        (int64_t)(r1 - r0) <= (int64_t)slots * (b - a) && so <= 0 && (int64_t)slots * a + so >= 0;
        bad |= !ok;
        s_start[tid] = r0;
        s_src[tid] = ok ? (int64_t)slots * a + so : -1;
    }
    if (tid == 0) s_start[nv] = row_ptr[v0 + nv];
    for (int i = nv + 1 + tid; i <= EG_BLOCK; i += EG_BLOCK) s_start[i] = INT32_MAX;  // past the last row
    __syncthreads();
    const int64_t a = s_start[0], e = s_start[nv];
    if (e > cols_cap || e < a) {
        if (tid == 0) set_error(err, e > cols_cap ? ERR_CAPACITY : ERR_INTERNAL);
        return;
    }
    for (int64_t i0 = a + tid; i0 < e; i0 += (int64_t)EG_BLOCK * EG_UNROLL) {
        int lo[EG_UNROLL];
#pragma unroll
        for (int u = 0; u < EG_UNROLL; ++u) lo[u] = 0;
#pragma unroll
        for (int step = EG_BLOCK / 2; step >= 1; step >>= 1)  // last row whose start <= i
#pragma unroll
            for (int u = 0; u < EG_UNROLL; ++u) {
                const int64_t i = i0 + (int64_t)u * EG_BLOCK;
                if ((int64_t)s_start[lo[u] + step] <= i) lo[u] += step;
            }
#pragma unroll
        for (int u = 0; u < EG_UNROLL; ++u) {
            const int64_t i = i0 + (int64_t)u * EG_BLOCK;
            if (i < e) {
                const int64_t src = s_src[lo[u]];
                if (src >= 0) cols[i] = stage[src + (i - s_start[lo[u]])];
            }
        }
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// Buffers of the stage (inside the workspace): tile_first and tile_ctx
// (n_tiles_bound + 1 ints each), the long-row list and its counter (zero on
// entry), cnt (n_vert + 1 ints: each row's distinct count, then the scan's
// input), soff (n_vert + 1 int16: where each row's values start in the stage,
// relative to its own slots), stage (S * q_bound ints, free memory: it may
// alias dead buffers), the scan's look-back words (zero on entry) and ticket.
struct ErowsBufs {
    int32_t* tile_first;
    int32_t* tile_ctx;
    int32_t* long_list;
    int64_t long_cap;
    uint32_t* long_count;
    int32_t* cnt;
    int16_t* soff;  // per row: where its values start in the stage, relative to stage_slots * (row start)
    int32_t* stage;
    uint64_t* scan_lb;
    uint32_t* scan_ticket;
    uint32_t* err;
};

inline int64_t erows_tiles_bound(int64_t q_bound) { return q_bound / ER_TILE + 1; }
inline int64_t erows_scan_tiles(int32_t n_vert) { return ceil_div((int64_t)n_vert + 1, SCAN_TILE); }
struct ErowsPlan;
ErowsBufs erows_bufs(const ErowsPlan& er, char* ws, uint32_t* err, uint32_t* ticket);
inline int64_t erows_long_cap(int64_t q_bound) { return q_bound / (ER_ROW_MAX + 1) + 1; }

// The stage: rows' counts and values (prep, long rows, tiles), counts scanned
// into row_ptr, values gathered into cols.
// scan_base: the row starts are offset by *scan_base (read on the device;
// null: none), for rows that continue a CSR written by earlier calls.
template <class Acc>
hipError_t launch_erows(const char* tag, const Acc& acc, const int32_t* erp, const int32_t* ecols, int64_t ecap,
                        int32_t n_vert, int64_t q_bound, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                        const ErowsBufs& b, hipStream_t s, const int32_t* scan_base = nullptr) {
    const int64_t n_tiles = erows_tiles_bound(q_bound);
    char name[48];
    snprintf(name, sizeof name, "%s_erows_prep", tag);
    hipError_t e = launch(name, erows_prep_kernel<Acc>, dim3((unsigned)ceil_div((int64_t)n_vert + 1, ER_PREP_BLOCK)),
                          dim3(ER_PREP_BLOCK), s, acc, erp, n_vert, q_bound, b.tile_first, b.tile_ctx, n_tiles,
                          b.long_list,
                          erows_long_cap(q_bound), b.long_count, b.err);
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_long", tag);
        e = launch(name, erows_long_kernel<Acc>, dim3(ER_LONG_GRID), dim3(ER_BLOCK), s, acc, erp, ecols, n_vert,
                   q_bound, ecap, (const int32_t*)b.long_list, erows_long_cap(q_bound), (const uint32_t*)b.long_count,
                   b.cnt, b.soff, b.stage, b.err);
    }
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows", tag);
        e = launch(name, erows_tile_kernel<Acc>, dim3((unsigned)n_tiles), dim3(ER_BLOCK), s, acc, erp, ecols,
                   n_vert, q_bound, ecap, (const int32_t*)b.tile_first, (const int32_t*)b.tile_ctx, b.cnt, b.soff,
                   b.stage, b.err);
    }
    if (e == hipSuccess && n_vert == 0) e = fill_i32(row_ptr, 1, 0, s);
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_scan", tag);
        e = launch(name, scan_i32_kernel, dim3((unsigned)ceil_div((int64_t)n_vert, SCAN_TILE)), dim3(SCAN_BLOCK), s,
                   (const int32_t*)b.cnt, (int64_t)n_vert, row_ptr, b.scan_lb, b.scan_ticket, b.err, scan_base);
    }
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_gather", tag);
        e = launch(name, erows_gather_kernel, dim3((unsigned)ceil_div((int64_t)n_vert, EG_BLOCK)), dim3(EG_BLOCK), s,
                   (const int32_t*)row_ptr, erp, (const int16_t*)b.soff, Acc::S, (const int32_t*)b.stage, n_vert,
                   q_bound, cols, cols_cap, b.err);
    }
    return e;
}

// Tile lists of a batch by element type: list k (k < N_ELEM_TYPES) holds the
// tiles whose owned rows all belong to meshes of type k, list N_ELEM_TYPES
// the rest (rows of several types, or a segment record with an unknown
// type).  Tiles that own no row are left out (their block would write
// nothing).  One thread per tile; lists[k * stride + i], counts[k].
constexpr int ER_LISTS = N_ELEM_TYPES + 1;
constexpr int ER_CLASSIFY_BLOCK = 256;
constexpr int ER_LIST_GRID = 2048;  // blocks of each list launch (each takes tiles in turn)
static __global__ __launch_bounds__(ER_CLASSIFY_BLOCK) void erows_classify_kernel(
    const int32_t* __restrict__ erp, int32_t n_vert, int64_t q_bound, const int32_t* __restrict__ tile_first,
    const int32_t* __restrict__ tile_ctx, const mesh_segment* __restrict__ segs, int32_t n_mesh,
    int32_t* __restrict__ lists, int64_t stride, uint32_t* counts) {
    const int64_t t = (int64_t)blockIdx.x * ER_CLASSIFY_BLOCK + threadIdx.x;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t n_tiles = erow_total(erp, n_vert, q_bound) / ER_TILE + 1;
    int k = -1;  // the tile's list, -1 for none
    if (t < n_tiles && n_mesh > 0) {
        // the owned vertices, clamped as erows_tile_body clamps them
        int32_t v_first = tile_first[t];
        int32_t v_end = t == n_tiles - 1 ? n_vert : tile_first[t + 1];
        v_first = tmin<int32_t>(tmax<int32_t>(v_first, 0), n_vert);
        v_end = tmin<int32_t>(tmax<int32_t>(v_end, v_first), n_vert);
        if (v_end > v_first) {
            const int32_t m0 = tmin<int32_t>(tmax<int32_t>(tile_ctx[t], 0), n_mesh - 1);
            const int32_t m1 = batch_mesh_from(segs, n_mesh, m0, v_end - 1);
            k = segs[m0].etype;
            for (int32_t m = m0 + 1; m <= m1 && k < N_ELEM_TYPES; ++m)
                if (segs[m].etype != k) k = N_ELEM_TYPES;
            if (k < 0 || k > N_ELEM_TYPES) k = N_ELEM_TYPES;
        }
    }
    // one counter atomic per (wave, list): most tiles go to one or two lists,
    // and one atomic per tile on the same word queues them all behind it
    const uint64_t lt = (1ull << lane) - 1;
    for (int kk = 0; kk < ER_LISTS; ++kk) {
        const uint64_t m = __ballot(k == kk);
        if (!m) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&counts[kk], (uint32_t)__popcll(m));
        base = __shfl(base, leader, WAVE);
        if (k == kk) {
            const uint32_t i = base + (uint32_t)__popcll(m & lt);
            if ((int64_t)i < stride) lists[kk * stride + i] = (int32_t)t;
        }
    }
}

// The stage for a batch: as launch_erows, with the tiles sorted into lists by
// the element type of their rows' meshes and each list run with that type's
// accessor (the rest with BatchRows).  lists: ER_LISTS * stride ints
// (stride >= the tile bound); counts: ER_LISTS words, zero on entry.
inline hipError_t launch_erows_batch(const char* tag, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                     const int32_t* erp, const int32_t* ecols, int64_t ecap, int32_t n_vert,
                                     int64_t q_bound, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                                     const ErowsBufs& b, int32_t* lists, int64_t stride, uint32_t* counts,
                                     hipStream_t s) {
    const BatchRows any{conn, segs, n_mesh};
    const int64_t n_tiles = erows_tiles_bound(q_bound);
    if (stride < n_tiles) return hipErrorInvalidValue;
    char name[48];
    snprintf(name, sizeof name, "%s_erows_prep", tag);
    hipError_t e = launch(name, erows_prep_kernel<BatchRows>,
                          dim3((unsigned)ceil_div((int64_t)n_vert + 1, ER_PREP_BLOCK)), dim3(ER_PREP_BLOCK), s, any,
                          erp, n_vert, q_bound, b.tile_first, b.tile_ctx, n_tiles, b.long_list,
                          erows_long_cap(q_bound), b.long_count, b.err);
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_long", tag);
        e = launch(name, erows_long_kernel<BatchRows>, dim3(ER_LONG_GRID), dim3(ER_BLOCK), s, any, erp, ecols, n_vert,
                   q_bound, ecap, (const int32_t*)b.long_list, erows_long_cap(q_bound), (const uint32_t*)b.long_count,
                   b.cnt, b.soff, b.stage, b.err);
    }
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_classify", tag);
        e = launch(name, erows_classify_kernel, dim3((unsigned)ceil_div(n_tiles, ER_CLASSIFY_BLOCK)),
                   dim3(ER_CLASSIFY_BLOCK), s, erp, n_vert, q_bound, (const int32_t*)b.tile_first,
                   (const int32_t*)b.tile_ctx, segs, n_mesh, lists, stride, counts);
    }
    snprintf(name, sizeof name, "%s_erows", tag);
    const dim3 grid((unsigned)tmin<int64_t>(n_tiles, ER_LIST_GRID));
    auto run_list = [&](auto acc, int k) {
        return launch(name, erows_tile_list_kernel<decltype(acc)>, grid, dim3(ER_BLOCK), s, acc, erp, ecols, n_vert,
                      q_bound, ecap, (const int32_t*)b.tile_first, (const int32_t*)b.tile_ctx, b.cnt, b.soff,
                      b.stage, (int)BatchRows::S, b.err, (const int32_t*)(lists + k * stride), (const uint32_t*)(counts + k));
    };
    for (int k = 0; k < N_ELEM_TYPES && e == hipSuccess; ++k)
        e = with_type(k, [&](auto et) {
            constexpr int ET = decltype(et)::value;
            return run_list(BatchTypedRows<ET>{conn, segs, n_mesh}, ET);
        });
    if (e == hipSuccess) e = run_list(any, N_ELEM_TYPES);
    if (e == hipSuccess && n_vert == 0) e = fill_i32(row_ptr, 1, 0, s);
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_scan", tag);
        e = launch(name, scan_i32_kernel, dim3((unsigned)ceil_div((int64_t)n_vert, SCAN_TILE)), dim3(SCAN_BLOCK), s,
                   (const int32_t*)b.cnt, (int64_t)n_vert, row_ptr, b.scan_lb, b.scan_ticket, b.err,
                   (const int32_t*)nullptr);
    }
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_gather", tag);
        e = launch(name, erows_gather_kernel, dim3((unsigned)ceil_div((int64_t)n_vert, EG_BLOCK)), dim3(EG_BLOCK), s,
                   (const int32_t*)row_ptr, erp, (const int16_t*)b.soff, (int)BatchRows::S, (const int32_t*)b.stage,
                   n_vert, q_bound, cols, cols_cap, b.err);
    }
    return e;
}

}  // namespace mnb
