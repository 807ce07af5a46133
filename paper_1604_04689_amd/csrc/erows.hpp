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
// solution (Sec. 3.2.2); counts become row starts by a decoupled look-back
// across tiles.
//
//   erows_prep   per vertex: the first vertex whose element row starts in
//                each tile of ER_TILE element-CSR entries; rows longer than
//                ER_ROW_MAX entries listed
//   erows_long   one block per listed row: candidates to global memory,
//                sorted and deduplicated there (block_sort_unique)
//   erows_tile   one block per tile, in tile order by ticket: the rows that
//                start in the tile, candidates into LDS hash tables spanning
//                each row's own candidate slots, distinct values compacted,
//                counts scanned (long rows' counts from erows_long), tile
//                offset by look-back, rows written to cols
#pragma once

#include <climits>
#include <cstdio>

#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "elements.hpp"
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

// Element access of a mesh of one type: element e's ids at conn + e * NPE.
template <int ET>
struct UniformRows {
    static constexpr int NPE = Elem<ET>::NPE;
    static constexpr int S = NPE - 1;
    static constexpr bool kCtx = false;
    const int32_t* __restrict__ conn;
    int64_t n_elem;
    int32_t n_vert;
    __device__ __forceinline__ int32_t ctx(int32_t) const { return 0; }
    // candidates of row vertex v in element e (as listed in v's element row);
    // *bad: e is not an element, or v is not in it
    __device__ __forceinline__ void cands(int32_t, int32_t v, int32_t e, uint32_t (&c)[S], bool* bad) const {
        if ((uint64_t)(uint32_t)e >= (uint64_t)n_elem) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            *bad = true;
            return;
        }
        int32_t ids[NPE];
        const int32_t* el = conn + (int64_t)e * NPE;
#pragma unroll
        for (int j = 0; j < NPE; ++j) ids[j] = el[j];
        *bad |= !elem_cands<NPE>(ids, NPE, adjacency_word<ET>(), v, n_vert, c);
    }
};

// Up to 8 ids of an element of runtime type `et` at el, and the candidates.
__device__ __forceinline__ bool runtime_cands(const int32_t* __restrict__ el, int32_t et, int32_t v, int32_t n_vert,
                                              uint32_t (&c)[MAX_NPE - 1]) {
    const int npe = nodes_per_elem(et);
    int32_t ids[MAX_NPE];
#pragma unroll
    for (int j = 0; j < MAX_NPE; ++j) ids[j] = j < npe ? el[j] : -1;
    return elem_cands<MAX_NPE>(ids, npe, adjacency_of(et), v, n_vert, c);
}

// Element access of a mesh whose elements carry their own types:
// element e has type etypes[e] and ids conn[elem_off[e] .. elem_off[e+1]).
struct MixedRows {
    static constexpr int S = MAX_NPE - 1;
    static constexpr bool kCtx = false;
    const int32_t* __restrict__ conn;
    const int32_t* __restrict__ elem_off;
    const uint8_t* __restrict__ etypes;
    int64_t n_elem, n_ids;
    int32_t n_vert;
    __device__ __forceinline__ int32_t ctx(int32_t) const { return 0; }
    __device__ __forceinline__ void cands(int32_t, int32_t v, int32_t e, uint32_t (&c)[S], bool* bad) const {
        bool ok = (uint64_t)(uint32_t)e < (uint64_t)n_elem;
        int32_t a = 0, et = 0;
        if (ok) {
            a = elem_off[e];
            const int32_t b = elem_off[e + 1];
            et = etypes[e];
            const int npe = nodes_per_elem(et);
            ok = npe > 0 && a >= 0 && b - a == npe && (int64_t)b <= n_ids;
        }
        if (!ok) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            *bad = true;
            return;
        }
        *bad |= !runtime_cands(conn + a, et, v, n_vert, c);
    }
};

// Element access of a batch: row vertex v is global; its mesh is the last
// segment with vert_off <= v (vert_off non-decreasing), its element ids are
// local to that mesh and so are the candidates.  ctx(v) is the mesh index.
struct BatchRows {
    static constexpr int S = MAX_NPE - 1;
    static constexpr bool kCtx = true;
    const int32_t* __restrict__ conn;
    const mesh_segment* __restrict__ segs;
    int32_t n_mesh;
    __device__ __forceinline__ int32_t ctx(int32_t v) const {
        int lo = 0, hi = n_mesh - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].vert_off <= v) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ void cands(int32_t m, int32_t v, int32_t e, uint32_t (&c)[S], bool* bad) const {
        const mesh_segment& sg = segs[m];
        const int npe = nodes_per_elem(sg.etype);
        const int32_t vl = v - sg.vert_off;
        if (npe == 0 || (uint64_t)(uint32_t)e >= (uint64_t)sg.n_elem || vl < 0 || vl >= sg.n_vert) {
#pragma unroll
            for (int s = 0; s < S; ++s) c[s] = CAND_NONE;
            *bad = true;
            return;
        }
        *bad |= !runtime_cands(conn + sg.conn_off + (int64_t)e * npe, sg.etype, vl, sg.n_vert, c);
    }
};

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
// whose element row starts at or after t * ER_TILE; rows longer than
// ER_ROW_MAX entries go to the long list.  One thread per v in [0, n_vert].
static __global__ __launch_bounds__(ER_PREP_BLOCK) void erows_prep_kernel(const int32_t* __restrict__ erp,
                                                                         int32_t n_vert, int64_t q_bound,
                                                                         int32_t* __restrict__ tile_first,
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
    for (int64_t t = t0; t <= t1; ++t) tile_first[t] = (int32_t)v;
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
                                                             int32_t* __restrict__ ldeg, int32_t* temp,
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
            if (p < qe) {
                acc.cands(cx, v, ecols[p], c, &bad);
            } else {
#pragma unroll
                for (int k = 0; k < S; ++k) c[k] = CAND_NONE;
            }
#pragma unroll
            for (int k = 0; k < S; ++k) x[S * i + k] = c[k] == CAND_NONE ? INT_MAX : (int32_t)c[k];
        }
        __threadfence_block();
        __syncthreads();
        const int64_t cnt = block_sort_unique(x, (int64_t)S * len, s, s_wcnt);
        if (tid == 0) ldeg[v] = (int32_t)cnt;
        __syncthreads();
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// The node CSR from the element CSR, one tile of ER_TILE entries per block.
// A block owns the vertices whose element row starts in its tile (tiles are
// taken by ticket, in order, for the look-back).  Entry position r of the
// tile (0 <= r < ER_SPAN, entry base + r) sits in register slot r / ER_BLOCK
// of thread r % ER_BLOCK, with its S candidates.
template <class Acc>
__global__ __launch_bounds__(ER_BLOCK) void erows_tile_kernel(Acc acc, const int32_t* __restrict__ erp,
                                                             const int32_t* __restrict__ ecols, int32_t n_vert,
                                                             int64_t q_bound, int64_t ecap,
                                                             const int32_t* __restrict__ tile_first,
                                                             const int32_t* __restrict__ ldeg,
                                                             const int32_t* __restrict__ temp,
                                                             int32_t* __restrict__ row_ptr,
                                                             int32_t* __restrict__ cols, int64_t cols_cap,
                                                             uint64_t* lookback, uint32_t* ticket, uint32_t* err) {
    constexpr int S = Acc::S;
    constexpr int CAP = ER_SPAN * S;
    constexpr int WAVES = ER_BLOCK / WAVE;
    constexpr int MAX_LONG = 64;  // long rows copied per chunk of owned vertices
    static_assert(CAP < INT16_MAX, "16-bit dense indices");
    // per-row hash tables over each row's own candidate slots; once every
    // insertion is done, the same words hold the distinct values, dense, in
    // slot order (each row's values contiguous)
    __shared__ uint32_t s_tab[CAP];
    __shared__ int16_t s_ra[ER_TILE];    // short row k: first entry, relative to the tile base
    __shared__ int16_t s_rlen[ER_TILE];  // entries
    __shared__ int16_t s_rds[ER_TILE];   // dense range of its distinct values
    __shared__ int16_t s_rde[ER_TILE];
    __shared__ int32_t s_rv[ER_TILE];    // vertex
    __shared__ int32_t s_roff[ER_TILE];  // offset of the row in the tile's output
    __shared__ int32_t s_rctx[Acc::kCtx ? ER_TILE : 1];
    __shared__ uint32_t s_wtot[ER_EPT][WAVES];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ int64_t s_tmp64[WAVES];
    __shared__ int32_t s_lv[MAX_LONG];   // long rows of a chunk: vertex, count, output offset
    __shared__ int64_t s_lcnt[MAX_LONG];
    __shared__ int64_t s_loff[MAX_LONG];
    __shared__ uint32_t s_nlong;
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_longsum;
    __shared__ uint64_t s_prefix;

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t q = erow_total(erp, n_vert, q_bound);
    const int64_t n_tiles = q / ER_TILE + 1;
    if ((int64_t)blockIdx.x >= n_tiles) return;  // owns nothing: takes no ticket
    if (tid == 0) {
        s_tile = atomicAdd(ticket, 1u);
        s_longsum = 0;
    }
    for (int i = tid; i < CAP; i += ER_BLOCK) s_tab[i] = SLOT_EMPTY;
    __syncthreads();
    const int64_t t = s_tile;
    const int64_t base = t * ER_TILE;
    const bool last_tile = t == n_tiles - 1;
    const int64_t qe = tmin<int64_t>(q, ecap);
    const int64_t in_end = tmin<int64_t>(qe - base, ER_SPAN);  // entry positions that can be read
    int32_t v_first = tile_first[t];
    int32_t v_end = last_tile ? n_vert : tile_first[t + 1];
    v_first = tmin<int32_t>(tmax<int32_t>(v_first, 0), n_vert);
    v_end = tmin<int32_t>(tmax<int32_t>(v_end, v_first), n_vert);
    bool bad = false;

    // ---- the owned vertices' rows: short non-empty rows listed in LDS;
    // long rows' distinct counts summed
    int32_t nrows = 0;
    for (int32_t c0 = v_first; c0 < v_end; c0 += ER_BLOCK) {
        const int32_t v = c0 + tid;
        int32_t a = 0, len = 0;
        if (v < v_end) len = erow_len(erp, v, q, &a, &bad);
        if (len > 0 && (a < base || a >= base + ER_TILE)) {  // not owned: only on an invalid CSR
            bad = true;
            len = 0;
        }
        const bool is_short = len > 0 && len <= ER_ROW_MAX;
        if (len > ER_ROW_MAX) atomicAdd(&s_longsum, (unsigned long long)long_count(ldeg, v, len, S));
        uint32_t total;
        const uint32_t k = (uint32_t)nrows + block_exclusive_sum<ER_BLOCK>((uint32_t)is_short, s_tmp, &total);
        if (is_short && k < (uint32_t)ER_TILE) {
            s_ra[k] = (int16_t)(a - base);
            s_rlen[k] = (int16_t)len;
            s_rv[k] = v;
            s_rds[k] = 0;
            s_rde[k] = 0;
            if constexpr (Acc::kCtx) s_rctx[k] = acc.ctx(v);
        }
        nrows += (int32_t)total;
    }
    if (nrows > ER_TILE) {  // distinct row starts in the tile: only on an invalid CSR
        bad = true;
        nrows = ER_TILE;
    }
    __syncthreads();

    // ---- candidates of every entry of a short row (element ids first, all
    // loads in flight, then the gathers)
    uint32_t cand[ER_EPT][S];
    int32_t rowk[ER_EPT];
    int32_t ent[ER_EPT];
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int r = i * ER_BLOCK + tid;
        int lo = 0, hi = nrows - 1;  // last short row starting at or before r
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_ra[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const bool in = nrows > 0 && s_ra[lo] <= r && r < s_ra[lo] + s_rlen[lo] && r < in_end;
        rowk[i] = in ? lo : -1;
        ent[i] = in ? ecols[base + r] : 0;
    }
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        if (rowk[i] >= 0) {
            const int k = rowk[i];
            acc.cands(Acc::kCtx ? s_rctx[k] : 0, s_rv[k], ent[i], cand[i], &bad);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) cand[i][s] = CAND_NONE;
        }
    }

    // ---- insert every candidate into its row's table (linear probing over
    // the row's own slots); the insertion that fills an empty slot keeps the
    // value
    uint64_t kept = 0;
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        if (rowk[i] < 0) continue;
        const int k = rowk[i];
        const uint32_t t0 = (uint32_t)S * (uint32_t)s_ra[k];
        const uint32_t len = (uint32_t)S * (uint32_t)s_rlen[k];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const uint32_t w = cand[i][s];
            if (w == CAND_NONE) continue;
            uint32_t h = (uint32_t)(((uint64_t)(w * 2654435761u) * len) >> 32);
            for (uint32_t probe = 0; probe < len; ++probe) {
                const uint32_t old = atomicCAS(&s_tab[t0 + h], SLOT_EMPTY, w);
                if (old == SLOT_EMPTY) {
                    kept |= 1ull << (i * S + s);
                    break;
                }
                if (old == w) break;
                h = h + 1 == len ? 0 : h + 1;
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

    // ---- the tile's output count, its offset by look-back
    int64_t mine = 0;
    for (int k = tid; k < nrows; k += ER_BLOCK) mine += tmax<int32_t>(s_rde[k] - s_rds[k], 0);
    int64_t tile_total;
    (void)block_exclusive_sum<ER_BLOCK, int64_t>(mine, s_tmp64, &tile_total);
    tile_total += (int64_t)s_longsum;
    if (wid == 0) {
        if (lane == 0) lb_store(lookback + t, (t == 0 ? LB_INC : LB_AGG) | (uint64_t)tile_total);
        const uint64_t before = wave_lookback_prefix(lookback, (uint32_t)t, (uint64_t)tile_total, err);
        if (lane == 0) s_prefix = before;
    }
    __syncthreads();
    const int64_t g0 = (int64_t)s_prefix;
    if (last_tile && tid == 0) row_ptr[n_vert] = (int32_t)(g0 + tile_total);

    // ---- row starts of the owned vertices; long rows copied from temp
    int64_t carry = 0;
    int32_t kk = 0;
    for (int32_t c0 = v_first; c0 < v_end; c0 += ER_BLOCK) {
        const int32_t v = c0 + tid;
        int32_t a = 0, len = 0;
        if (v < v_end) len = erow_len(erp, v, q, &a, &bad);
        if (len > 0 && (a < base || a >= base + ER_TILE)) len = 0;
        const bool is_short = len > 0 && len <= ER_ROW_MAX;
        const bool is_long = len > ER_ROW_MAX;
        uint32_t n_short;
        const uint32_t k = (uint32_t)kk + block_exclusive_sum<ER_BLOCK>((uint32_t)is_short, s_tmp, &n_short);
        int64_t cnt = 0;
        if (is_short && k < (uint32_t)ER_TILE) cnt = tmax<int32_t>(s_rde[k] - s_rds[k], 0);
        if (is_long) cnt = long_count(ldeg, v, len, S);
        int64_t chunk_total;
        const int64_t off = carry + block_exclusive_sum<ER_BLOCK, int64_t>(cnt, s_tmp64, &chunk_total);
        if (tid == 0) s_nlong = 0;
        __syncthreads();
        if (v < v_end) row_ptr[v] = (int32_t)(g0 + off);
        if (is_short && k < (uint32_t)ER_TILE) s_roff[k] = (int32_t)off;
        if (is_long) {
            const uint32_t slot = atomicAdd(&s_nlong, 1u);
            if (slot < (uint32_t)MAX_LONG) {
                s_lv[slot] = v;
                s_lcnt[slot] = cnt;
                s_loff[slot] = off;
            }
        }
        __syncthreads();
        const int n_long = (int)tmin<uint32_t>(s_nlong, (uint32_t)MAX_LONG);
        if (s_nlong > (uint32_t)MAX_LONG) bad = true;  // only on an invalid CSR
        for (int li = 0; li < n_long; ++li) {
            const int32_t lv = s_lv[li];
            const int64_t dst = g0 + s_loff[li];
            const int64_t n = s_lcnt[li];  // at most the row's candidate slots
            const int32_t* src = temp + (int64_t)S * erp[lv];
            if (dst + n > cols_cap) {
                if (tid == 0) set_error(err, ERR_CAPACITY);
                continue;
            }
            for (int64_t x = tid; x < n; x += ER_BLOCK) cols[dst + x] = src[x];
        }
        carry += chunk_total;
        kk += (int32_t)n_short;
        __syncthreads();
    }

    // ---- short rows' values: a value's place is the number of its row's
    // distinct values below it
    bool full = false;
#pragma unroll
    for (int i = 0; i < ER_EPT; ++i) {
        const int k = rowk[i];
        if (k < 0) continue;
        const int ds = s_rds[k], de = s_rde[k];
        const int64_t row0 = g0 + s_roff[k];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (!((kept >> (i * S + s)) & 1ull)) continue;
            const uint32_t w = cand[i][s];
            int below = 0;
            for (int x = ds; x < de; ++x) below += s_tab[x] < w ? 1 : 0;
            const int64_t dst = row0 + below;
            if (dst < cols_cap) cols[dst] = (int32_t)w;
            else full = true;
        }
    }
    if (full) set_error(err, ERR_CAPACITY);
    if (bad) set_error(err, ERR_INTERNAL);
}

// Buffers of the stage (inside the workspace): n_tiles_bound look-back words
// (zero on entry), tile_first (n_tiles_bound + 1 ints), the long-row list and
// its counter (zero on entry), ldeg (n_vert ints), temp (S * q_bound ints,
// free memory: it may alias dead buffers).
struct ErowsBufs {
    uint64_t* lookback;
    int32_t* tile_first;
    int32_t* long_list;
    int64_t long_cap;
    uint32_t* long_count;
    int32_t* ldeg;
    int32_t* temp;
    uint32_t* ticket;
    uint32_t* err;
};

inline int64_t erows_tiles_bound(int64_t q_bound) { return q_bound / ER_TILE + 1; }
struct ErowsPlan;
ErowsBufs erows_bufs(const ErowsPlan& er, char* ws, uint32_t* err, uint32_t* ticket);
inline int64_t erows_long_cap(int64_t q_bound) { return q_bound / (ER_ROW_MAX + 1) + 1; }

template <class Acc>
hipError_t launch_erows(const char* tag, const Acc& acc, const int32_t* erp, const int32_t* ecols, int64_t ecap,
                        int32_t n_vert, int64_t q_bound, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                        const ErowsBufs& b, hipStream_t s) {
    const int64_t n_tiles = erows_tiles_bound(q_bound);
    char name[48];
    snprintf(name, sizeof name, "%s_erows_prep", tag);
    hipError_t e = launch(name, erows_prep_kernel, dim3((unsigned)ceil_div((int64_t)n_vert + 1, ER_PREP_BLOCK)),
                          dim3(ER_PREP_BLOCK), s, erp, n_vert, q_bound, b.tile_first, n_tiles, b.long_list,
                          erows_long_cap(q_bound), b.long_count, b.err);
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows_long", tag);
        e = launch(name, erows_long_kernel<Acc>, dim3(ER_LONG_GRID), dim3(ER_BLOCK), s, acc, erp, ecols, n_vert,
                   q_bound, ecap, (const int32_t*)b.long_list, erows_long_cap(q_bound), (const uint32_t*)b.long_count,
                   b.ldeg, b.temp, b.err);
    }
    if (e == hipSuccess) {
        snprintf(name, sizeof name, "%s_erows", tag);
        e = launch(name, erows_tile_kernel<Acc>, dim3((unsigned)n_tiles), dim3(ER_BLOCK), s, acc, erp, ecols,
                   n_vert, q_bound, ecap, (const int32_t*)b.tile_first, (const int32_t*)b.ldeg,
                   (const int32_t*)b.temp, row_ptr, cols, cols_cap, b.lookback, b.ticket, b.err);
    }
    return e;
}

}  // namespace mnb
