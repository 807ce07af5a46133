// One-ring neighboring nodes (paper Sec. 2.1.1 and 2.2.1).
//
// The paper forms two integer pairs per triangle edge (both directions), sorts
// the pairs by their first entry, and derives per vertex the count and first
// index of its neighbors by segmented reduction and scan.  Four algorithms
// with identical output (mesh_node_sort):
//
//   FULL_KEY     each directed pair (u, w) packed into one 64-bit key
//                (u << b) | w, b = bits of a vertex id, the whole key sorted
//                (node_hist, radix_pass x p, the first pass generating the
//                keys from conn), then unique_csr drops repeats and writes
//                cols and the row starts;
//   VERTEX_ROWS  the same keys sorted by u only, rows deduplicated in LDS
//                (rows.hpp);
//   EDGE_ROWS    each element edge once as (min << b) | max sorted by min,
//                rows deduplicated, unique edges transposed and sorted by max,
//                lower and higher neighbours merged (edges.hpp);
//   ELEM_ROWS    the element relation (elem_path.hip), then each node row
//                gathered from the elements of the vertex's element row and
//                deduplicated in LDS (erows.hpp).
#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "csr.hpp"
#include "edges.hpp"
#include "erows.hpp"
#include "radix.hpp"
#include "rows.hpp"

namespace mnb {

constexpr int MAX_PASS = 8;  // 2b <= 62 key bits

constexpr int NH_BLOCK = 512;
constexpr int NH_UNROLL = 4;      // elements per thread in flight
constexpr int NH_GRID_MAX = 1024;

// ---------------------------------------------------------------------------
// Directed edge pairs of the elements, generated on the fly from the
// connectivity.  Key index i: element e = i / (2*NE), edge k and direction
// from the remainder; both directions of every edge (the six pairs per
// triangle of Sec. 2.2.1).  A self pair (repeated id in a degenerate element)
// or a pair touching an id outside [0, n_vert) yields KEY_NONE, which sorts
// after every real key and is dropped by unique_csr.
// ---------------------------------------------------------------------------
// Key of directed pair r (edge r / 2, direction r % 2) of the element whose
// ids start at el.
template <int ET>
__device__ __forceinline__ uint64_t elem_pair_key(const int32_t* el, int r, int32_t n_vert, uint32_t b) {
    int pa, pb;
    edge_nodes<ET>(r >> 1, &pa, &pb);
    const int32_t x = el[pa], y = el[pb];
    const int32_t u = (r & 1) ? y : x;
    const int32_t w = (r & 1) ? x : y;
    const bool edge = (uint32_t)u < (uint32_t)n_vert && (uint32_t)w < (uint32_t)n_vert && u != w;
    return edge ? ((uint64_t)u << b) | (uint64_t)w : KEY_NONE;
}

// Canonical key of edge k of the element whose ids start at el: the edge once,
// (min << b) | max, for the edge-rows algorithm.
template <int ET>
__device__ __forceinline__ uint64_t elem_canon_key(const int32_t* el, int k, int32_t n_vert, uint32_t b) {
    int pa, pb;
    edge_nodes<ET>(k, &pa, &pb);
    const int32_t x = el[pa], y = el[pb];
    const bool edge = (uint32_t)x < (uint32_t)n_vert && (uint32_t)y < (uint32_t)n_vert && x != y;
    const uint32_t lo = (uint32_t)(x < y ? x : y), hi = (uint32_t)(x < y ? y : x);
    return edge ? ((uint64_t)lo << b) | (uint64_t)hi : KEY_NONE;
}

// Key i of the node relation: directed pairs (2 per edge), or with CANON the
// edges once each.
template <int ET, bool CANON>
__device__ __forceinline__ uint64_t node_key_at(const int32_t* el, int r, int32_t n_vert, uint32_t b) {
    if constexpr (CANON) return elem_canon_key<ET>(el, r, n_vert, b);
    else return elem_pair_key<ET>(el, r, n_vert, b);
}

template <int ET, bool CANON>
__device__ __forceinline__ uint64_t node_pair_key(const int32_t* __restrict__ conn, int64_t i, int32_t n_vert,
                                                  uint32_t b) {
    constexpr uint32_t KPE = (CANON ? 1 : 2) * Elem<ET>::NE;
    const uint32_t ii = (uint32_t)i;  // pair indices stay below 2^31
    const uint32_t e = ii / KPE;
    return node_key_at<ET, CANON>(conn + (size_t)e * Elem<ET>::NPE, (int)(ii - e * KPE), n_vert, b);
}

// Pair keys of the single-mesh node relation.  A radix tile first copies the
// connectivity of the elements its pairs come from into LDS with coalesced
// loads (stage), then builds every key from there (load_staged).
template <int ET, bool CANON = false>
struct NodePairSrc {
    const int32_t* __restrict__ conn;
    int32_t n_vert;
    uint32_t b;
    static constexpr bool kSkipNone = false;
    static constexpr bool kStaged = true;
    static constexpr uint32_t KPE = (CANON ? 1 : 2) * Elem<ET>::NE;  // keys per element
    static constexpr int NPE = Elem<ET>::NPE;

    __device__ __forceinline__ uint64_t load(int64_t i) const {
        return node_pair_key<ET, CANON>(conn, i, n_vert, b);
    }

    // ids of the tile's elements to s[0 ..): at most (TILE / KPE + 2) * NPE words
    template <int BLOCK, int TILE>
    __device__ __forceinline__ void stage(int64_t tile_base, int64_t n, int32_t* s, int tid) const {
        constexpr int MAXC = (TILE / (int)KPE + 2) * NPE;
        constexpr int PER = (MAXC + BLOCK - 1) / BLOCK;
        static_assert(MAXC <= 2 * TILE, "staged ids fit the key staging area");
        const uint32_t e0 = (uint32_t)tile_base / KPE;
        const uint32_t e1 = ((uint32_t)tmin<int64_t>(tile_base + TILE, n) - 1u) / KPE;
        const int cnt = (int)(e1 - e0 + 1u) * NPE;
        const int32_t* src = conn + (size_t)e0 * NPE;
        int32_t v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            v[q] = i < cnt ? src[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            if (i < cnt) s[i] = v[q];
        }
    }
    struct Header {};
    __device__ __forceinline__ bool staged(const int32_t*) const { return true; }
    __device__ __forceinline__ Header header(const int32_t*) const { return {}; }
    __device__ __forceinline__ uint64_t load_staged(Header, int64_t i, int64_t tile_base, const int32_t* s) const {
        const uint32_t ii = (uint32_t)i;
        const uint32_t e = ii / KPE;
        const uint32_t e0 = (uint32_t)tile_base / KPE;
        return node_key_at<ET, CANON>(s + (e - e0) * NPE, (int)(ii - e * KPE), n_vert, b);
    }
};

// ---------------------------------------------------------------------------
// node_hist: the digit histograms of every radix pass over all pair keys,
// read from the connectivity (the keys themselves are generated again by the
// first radix pass).  A thread takes whole elements, HIST_UNROLL of them in
// flight at once; each block accumulates in LDS and flushes once with global
// atomics.  Raises ERR_INDEX_RANGE.
// ---------------------------------------------------------------------------
template <int ET, bool CANON>
__global__ __launch_bounds__(NH_BLOCK) void node_hist_kernel(const int32_t* __restrict__ conn, int64_t n_elem,
                                                            int32_t n_vert, uint32_t b, uint32_t shift0, int n_pass,
                                                            uint32_t last_bits, uint32_t* __restrict__ hist,
                                                            uint32_t* err) {
    using E = Elem<ET>;
    constexpr int NPE = E::NPE;
    __shared__ uint32_t s_hist[MAX_PASS * RADIX];
    const int tid = threadIdx.x;
    for (int i = tid; i < n_pass * RADIX; i += NH_BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool bad_seen = false;
    const int64_t stride = (int64_t)gridDim.x * NH_BLOCK;
    for (int64_t e0 = (int64_t)blockIdx.x * NH_BLOCK + tid; e0 < n_elem; e0 += stride * NH_UNROLL) {
        int32_t id[NH_UNROLL][NPE];
#pragma unroll
        for (int u = 0; u < NH_UNROLL; ++u) {  // all loads in flight first
            const int64_t e = e0 + u * stride;
            if (e < n_elem) load_elem_ids<ET>(conn, e, id[u]);
        }
#pragma unroll
        for (int u = 0; u < NH_UNROLL; ++u) {
            if (e0 + u * stride >= n_elem) continue;
            bool ok[NPE];
#pragma unroll
            for (int j = 0; j < NPE; ++j) {
                ok[j] = (uint32_t)id[u][j] < (uint32_t)n_vert;
                bad_seen |= !ok[j];
            }
#pragma unroll
            for (int k = 0; k < E::NE; ++k) {
                const int32_t x = id[u][E::A[k]], y = id[u][E::B[k]];
                const bool edge = ok[E::A[k]] && ok[E::B[k]] && x != y;
                const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
                const uint64_t k0 = !edge ? KEY_NONE
                                          : CANON ? ((uint64_t)lo << b) | (uint64_t)hi : ((uint64_t)x << b) | (uint64_t)y;
                const uint64_t k1 = edge ? ((uint64_t)y << b) | (uint64_t)x : KEY_NONE;
                for (int p = 0; p < n_pass; ++p) {
                    const uint32_t mask = (p == n_pass - 1) ? ((1u << last_bits) - 1) : (RADIX - 1);
                    atomicAdd(&s_hist[p * RADIX + ((uint32_t)(k0 >> (shift0 + p * RBITS)) & mask)], 1u);
                    if (!CANON) atomicAdd(&s_hist[p * RADIX + ((uint32_t)(k1 >> (shift0 + p * RBITS)) & mask)], 1u);
                }
            }
        }
    }
    if (bad_seen) set_error(err, ERR_INDEX_RANGE);
    __syncthreads();
    for (int i = tid; i < n_pass * RADIX; i += NH_BLOCK) {
        const uint32_t v = s_hist[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool plan_node(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, bool internal_elem, NodePlan* p) {
    const int ne = edges_per_elem(etype);
    if (ne == 0 || n_elem < 0 || n_vert < 0) return false;
    *p = NodePlan{};
    p->opts = o;
    p->mode = o.node_sort;
    p->n_elem = n_elem;
    p->etype = etype;
    p->n_vert = n_vert;
    p->n_pairs = 2 * (int64_t)ne * n_elem;
    p->n_edges = (int64_t)ne * n_elem;
    p->id_bits = id_bits_for(n_vert);
    if (p->mode == NS_ELEM_ROWS) {
        // the element relation first (its own plan from offset 0, header
        // included); its key buffers are dead once it has run, and hold the
        // long rows' candidates when they are large enough
        if (!plan_elem(n_elem, etype, n_vert, o, &p->ep)) return false;
        size_t off = p->ep.total;
        p->internal_elem = internal_elem;
        if (internal_elem) {
            p->off_erp = off;
            off += align_up(((size_t)n_vert + 1) * sizeof(int32_t));
            p->off_ecols = off;
            off += align_up((size_t)p->ep.n_slots * sizeof(int32_t));
        }
        off = plan_erows(p->ep.n_slots, nodes_per_elem(etype) - 1, n_vert, off, p->ep.off_keys0,
                         p->ep.off_bmin - p->ep.off_keys0, &p->er);
        p->zero_bytes = p->ep.zero_bytes;
        p->total = off;
        return true;
    }
    const bool full = p->mode == NS_FULL_KEY, edges = p->mode == NS_EDGE_ROWS;
    // full-key: passes over all 2b key bits; vertex-rows and edge-rows: over
    // the bits of the high part (a vertex id) above the low b bits, one more
    // than a vertex id needs when n_vert is a power of two, so that KEY_NONE
    // (all ones, still taking part in these sorts) ties with no real vertex
    p->sort_bits = full ? 2 * p->id_bits : bits_for_count((int64_t)n_vert + 1);
    p->pp = plan_passes(p->sort_bits, RBITS);  // the node sorts take 8-bit digits
    p->n_keys = edges ? p->n_edges : p->n_pairs;
    p->n_tiles = ceil_div(p->n_keys, min_radix_tile());  // look-back room for any tile shape
    p->n_utiles = ceil_div(p->n_pairs, UNIQ_TILE);
    p->long_cap = p->n_keys / (ROW_SHORT + 1) + 1;
    size_t off = HEADER_BYTES;
    p->off_hist = off;
    off += align_up(MAX_PASS * RADIX * sizeof(uint32_t));
    if (edges) {
        p->off_hist2 = off;
        off += align_up(MAX_KH_PASS * RADIX * sizeof(uint32_t));
    }
    p->off_ulb = off;  // unique/CSR look-back (full key) or the row-count scan's (rows)
    off += align_up((size_t)(full ? p->n_utiles : ceil_div((int64_t)n_vert + 1, SCAN_TILE)) * sizeof(uint64_t));
    p->off_lb0 = off;
    off += align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t));
    p->zero_bytes = off;  // header, histograms, CSR/scan look-back, pass-0 look-back
    p->off_lb1 = off;
    off += align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t));
    // key buffers: the sort ping-pongs n_keys keys.  Edge-rows then needs,
    // in the buffer the sort ended in, room for the transposed edges'
    // ping-pong (2 x n_edges keys); the other one holds the row values and
    // the higher neighbours (2 x n_edges ints).
    const size_t kb = align_up((size_t)p->n_keys * sizeof(uint64_t));
    const bool sorted_in_1 = ((p->pp.n_pass - 1) & 1) != 0;
    p->off_keys0 = off;
    off += edges && !sorted_in_1 ? 2 * kb : kb;
    p->off_keys1 = off;
    off += edges && sorted_in_1 ? 2 * kb : kb;
    if (!full) {
        p->off_deg = off;  // distinct neighbors per vertex
        off += align_up((size_t)n_vert * sizeof(int32_t));
        p->off_src = off;  // first key index of each row
        off += align_up((size_t)n_vert * sizeof(int64_t));
        p->off_long = off;
        off += align_up((size_t)p->long_cap * sizeof(int64_t));
    }
    if (edges) {
        p->off_up = off;
        off += align_up(((size_t)n_vert + 1) * sizeof(int32_t));
        p->off_low = off;
        off += align_up(((size_t)n_vert + 1) * sizeof(int32_t));
        p->off_bmin = off;  // block minima of the lower-group fill
        off += align_up((size_t)ceil_div((int64_t)n_vert + 1, (int64_t)RF_TILE) * sizeof(int32_t));
    }
    p->total = off;
    return true;
}

template <int ET>
static hipError_t node_pipeline(const NodePlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                                int64_t cols_capacity, char* w, hipStream_t s) {
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    uint32_t* tickets = hdr + HDR_TICKET0;
    uint32_t* hist = (uint32_t*)(w + p.off_hist);
    uint64_t* ulb = (uint64_t*)(w + p.off_ulb);
    uint64_t* lb[2] = {(uint64_t*)(w + p.off_lb0), (uint64_t*)(w + p.off_lb1)};
    uint64_t* kb[2] = {(uint64_t*)(w + p.off_keys0), (uint64_t*)(w + p.off_keys1)};
    const int shape = p.opts.shape;
    const bool rows = p.mode == NS_VERTEX_ROWS, edges = p.mode == NS_EDGE_ROWS;
    const PassPlan& pp = p.pp;
    const int n_pass = pp.n_pass;
    const uint32_t shift0 = rows || edges ? p.id_bits : 0;
    const int64_t n_keys = p.n_keys;
    const int grid = (int)tmin<int64_t>(ceil_div(p.n_elem, NH_BLOCK), NH_GRID_MAX);
    const uint32_t last_bits = pp.width[n_pass - 1];
    // (the caller has cleared the row degrees and, for edge-rows, set the
    // lower-group starts to INT32_MAX, with the workspace header)
    hipError_t e = edges ? launch("node_hist", node_hist_kernel<ET, true>, dim3(grid), dim3(NH_BLOCK), s, conn, p.n_elem,
                           p.n_vert, p.id_bits, shift0, n_pass, last_bits, hist, err)
                  : launch("node_hist", node_hist_kernel<ET, false>, dim3(grid), dim3(NH_BLOCK), s, conn, p.n_elem,
                           p.n_vert, p.id_bits, shift0, n_pass, last_bits, hist, err);
    if (e != hipSuccess) return e;
    if ((rows || edges) && p.n_vert == 0) return fill_i32(row_ptr, 1, 0, s);  // every id is out of range
    for (int pass = 0; pass < n_pass && e == hipSuccess; ++pass) {
        const uint32_t shift = shift0 + pp.shift[pass];
        const uint32_t bits = pp.width[pass];
        uint64_t* out = kb[pass & 1];
        // edge-rows: the last pass also clears the look-back slots of the
        // first pass over the transposed edges
        uint64_t* lb_next = pass + 1 < n_pass || edges ? lb[(pass + 1) & 1] : nullptr;
        if (pass == 0)
            e = edges ? launch_radix_pass("node_radix_first", shape, NodePairSrc<ET, true>{conn, p.n_vert, p.id_bits},
                                          out, n_keys, shift, bits, hist, lb[0], lb_next, tickets + 0, err, s)
                      : launch_radix_pass("node_radix_first", shape, NodePairSrc<ET, false>{conn, p.n_vert, p.id_bits},
                                          out, n_keys, shift, bits, hist, lb[0], lb_next, tickets + 0, err, s);
        else
            e = launch_radix_pass("node_radix", shape, KeyArraySrc{kb[(pass - 1) & 1]}, out, n_keys, shift, bits,
                                  hist + pass * RADIX, lb[pass & 1], lb_next, tickets + pass, err, s);
    }
    if (e != hipSuccess) return e;
    const uint64_t* sorted = kb[(n_pass - 1) & 1];
    if (!rows && !edges)
        return launch_unique_csr("node_unique_csr", sorted, p.n_pairs, (const uint32_t*)nullptr, p.id_bits,
                                 p.n_vert, cols, cols_capacity, row_ptr, ulb, tickets + (N_TICKETS - 1), err, s);
    // vertex-rows mode: canonical rows into the free key buffer, then scan and gather
    RowsStage r{sorted, n_keys, p.id_bits, p.n_vert, (int32_t*)(w + p.off_deg), (int64_t*)(w + p.off_src),
                (int32_t*)kb[n_pass & 1], (int64_t*)(w + p.off_long), p.long_cap, hdr + HDR_LONG_COUNT,
                ulb, tickets + (N_TICKETS - 2), err};
    if (rows) return launch_rows_stage(false, r, row_ptr, cols, cols_capacity, s);

    // edge-rows mode: the rows stage over the canonical keys gives each
    // vertex's higher neighbours; their scan is up_ptr (up_ptr[V] = E)
    int32_t* up_ptr = (int32_t*)(w + p.off_up);
    int32_t* low_ptr = (int32_t*)(w + p.off_low);
    e = launch_rows_dedup(r, up_ptr, s);
    if (e != hipSuccess) return e;
    // transposed edges (w << b) | v: ping-pong halves of the sorted buffer (free
    // now, sized for 2 x n_edges keys); w alone after the row values in the
    // other buffer
    EdgeStage g{up_ptr, r.deg, r.src, r.temp, p.n_vert, p.id_bits, nullptr, 0, p.n_edges,
                {kb[(n_pass - 1) & 1], kb[(n_pass - 1) & 1] + p.n_edges}, (int32_t*)kb[n_pass & 1] + p.n_edges,
                (uint32_t*)(w + p.off_hist2), {lb[0], lb[1]}, n_pass & 1, tickets + 8, shape, pp,
                low_ptr, (int32_t*)(w + p.off_bmin), err};
    e = launch_edge_stage(g, row_ptr, cols, cols_capacity, s);
    return e;
}

hipError_t run_node(const NodePlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                    void* ws, hipStream_t s, bool keep_err, const int32_t* elem_row_ptr, const int32_t* elem_cols,
                    int64_t elem_cap) {
    char* w = (char*)ws;
    if (p.mode == NS_ELEM_ROWS) {
        // the element relation into the caller's outputs, or the workspace
        int32_t* erp = p.internal_elem ? (int32_t*)(w + p.off_erp) : const_cast<int32_t*>(elem_row_ptr);
        int32_t* ecols = p.internal_elem ? (int32_t*)(w + p.off_ecols) : const_cast<int32_t*>(elem_cols);
        const int64_t ecap = p.internal_elem ? p.ep.n_slots : elem_cap;
        const FillRegion extra{w + p.er.off_lb, p.er.lb_words, 0u};
        hipError_t e = run_elem(p.ep, conn, erp, ecols, ecap, ws, s, keep_err, &extra);
        if (e != hipSuccess) return e;
        if (p.ep.n_slots == 0) return fill_i32(row_ptr, (int64_t)p.n_vert + 1, 0, s);
        uint32_t* hdr = (uint32_t*)w;
        return run_erows_uniform(p.etype, p.er, conn, p.n_elem, p.n_vert, erp, ecols, ecap, row_ptr, cols,
                                 cols_capacity, w, hdr + HDR_ERR, hdr + HDR_TICKET0 + TK_EROWS, s);
    }
    const int mode = p.mode;
    FillRegion fill[3] = {header_fill(ws, p.zero_bytes, keep_err)};
    int n_fill = 1;
    if (p.n_pairs > 0 && mode != NS_FULL_KEY) fill[n_fill++] = {w + p.off_deg, p.n_vert, 0u};
    if (p.n_pairs > 0 && mode == NS_EDGE_ROWS) fill[n_fill++] = {w + p.off_low, (int64_t)p.n_vert + 1, (uint32_t)INT32_MAX};
    hipError_t e = fill_regions(fill, n_fill, s);
    if (e != hipSuccess) return e;
    if (p.n_pairs == 0) return fill_i32(row_ptr, (int64_t)p.n_vert + 1, 0, s);
    return with_type(p.etype, [&](auto et) {
        return node_pipeline<decltype(et)::value>(p, conn, row_ptr, cols, cols_capacity, w, s);
    });
}

}  // namespace mnb
