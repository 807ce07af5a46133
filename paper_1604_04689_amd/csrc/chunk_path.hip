// Bounded-memory build: the relations of one mesh one vertex range at a time.
//
// The paper's method keeps every pair of the mesh in device memory at once,
// and the paper names that footprint as its limit, leaving a leaner design to
// future work (Sec. 3.2.2, Sec. 4).  Here the vertices are cut into ranges
// whose pairs fit a fixed budget, and each range runs the element sort of
// Sec. 2.2.2 on its own pairs only: rows of different vertices never share a
// pair, so a range's rows are final as soon as its sort ends, and the ranges
// are written one after the other at their place in the outputs.
//
//   fill            header, the first row start of each output
//   chunk_coarse    conn -> pairs per bin of the top vertex bits (block
//                   partials, then summed); read back with one wait
//   (host)          ranges of whole bins, at most cap pairs and cap vertices
//   per range [v0, v1), its pairs starting at element-CSR entry ebase:
//     fill            header (error word kept), histograms, look-back words,
//                     the range's row starts
//     chunk_compact   conn -> the range's (u << 32) | e keys, u = v - v0, in
//                     connectivity order (a stable compaction: tile offsets
//                     by a decoupled look-back over one count)
//     chunk_hist      digit histograms of the range's passes over its keys
//     radix passes    stable, by the digits of u; the last writes the
//                     element columns at ebase and the range's row starts
//     rowptr_fill     row starts of the range's empty rows
//     chunk_rows      element row starts + ebase -> the caller's row_ptr
//     erows stage     the range's node rows from its element rows (the
//                     ELEM_ROWS stage), their starts continuing the previous
//                     range's last one on the device
#include <vector>

#include "edges.hpp"
#include "elem.hpp"
#include "erows.hpp"

namespace mnb {

// Stable compaction of one range's keys.  Tile t (by ticket) covers
// connectivity slots [t * CC_TILE, (t + 1) * CC_TILE); item j of thread x is
// slot t * CC_TILE + j * CC_BLOCK + x, so (item, wave, lane) order is slot
// order.  A key's place is the number of the range's keys in earlier slots:
// the tile's own by ballots and a scan of the per-(item, wave) counts, the
// earlier tiles' by a decoupled look-back over one running count.  Their
// number goes to *pair_count.  (Counting the digit histograms here too was
// measured slower: every tile adding its few hundred digit counts to the same
// global words queued those atomics behind each other.)
constexpr int CC_BLOCK = 512;
// Tiles are large, so the chain of look-back status words is short (9% faster
// than 8192-slot tiles on MI355X); a slot keeps only its id and one validity
// bit in registers, and its key is rebuilt when it is written.
constexpr int CC_ITEMS = 48;
constexpr int CC_TILE = CC_BLOCK * CC_ITEMS;
constexpr int TK_COMPACT = 4;  // ticket slot in the workspace header (after the passes')
constexpr int CHUNK_HIST_GRID = 128;  // blocks of the range's histogram kernel (each adds its counts once)

template <int ET>
__global__ __launch_bounds__(CC_BLOCK) void chunk_compact_kernel(ElemPairSrc<ET> src, int64_t n_slots,
                                                                 uint64_t* __restrict__ keys, int64_t keys_cap,
                                                                 uint64_t* lookback, uint32_t* ticket,
                                                                 uint32_t* pair_count, uint32_t* err) {
    constexpr int NPE = ElemPairSrc<ET>::NPE;
    constexpr int WAVES = CC_BLOCK / WAVE;
    constexpr int PARTS = CC_ITEMS * WAVES;
    constexpr int PER_LANE = PARTS / WAVE;  // (item, wave) counts each lane of the scanning wave takes
    static_assert(PARTS % WAVE == 0 && CC_ITEMS <= 64, "whole counts per lane; one mask bit per item");
    __shared__ uint32_t s_cnt[PARTS];  // count of (item j, wave w) at j * WAVES + w, then its offset
    __shared__ uint32_t s_tile, s_total;
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t first = (int64_t)tile * CC_TILE;
    // every slot's id first (all loads in flight); a slot takes part when its
    // id lies in the window and first occurs there in its element (the few
    // such slots read their element's earlier ids)
    int32_t id[CC_ITEMS];
#pragma unroll
    for (int j = 0; j < CC_ITEMS; ++j) {
        const int64_t i = first + j * CC_BLOCK + tid;
        id[j] = i < n_slots ? src.conn[i] : src.v_lo - 1;
    }
    uint64_t valid = 0;
#pragma unroll
    for (int j = 0; j < CC_ITEMS; ++j) {
        if ((uint32_t)(id[j] - src.v_lo) < (uint32_t)src.n_vert) {
            const uint32_t s = (uint32_t)(first + j * CC_BLOCK + tid);  // slot indices stay below 2^31
            const uint32_t e = s / NPE;
            if (first_occurrence<NPE>(src.conn, e, (int)(s - e * NPE), id[j])) valid |= 1ull << j;
        }
    }
#pragma unroll
    for (int j = 0; j < CC_ITEMS; ++j) {
        const uint64_t b = __ballot((valid >> j) & 1ull);
        if (lane == 0) s_cnt[j * WAVES + wid] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (wid == 0) {
        uint32_t c[PER_LANE], sum = 0;
#pragma unroll
        for (int k = 0; k < PER_LANE; ++k) {
            c[k] = s_cnt[PER_LANE * lane + k];
            sum += c[k];
        }
        const uint32_t incl = wave_inclusive_sum(sum);
        uint32_t run = incl - sum;
#pragma unroll
        for (int k = 0; k < PER_LANE; ++k) {
            s_cnt[PER_LANE * lane + k] = run;
            run += c[k];
        }
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        if (lane == 0) lb_store(lookback + tile, (tile == 0 ? LB_INC : LB_AGG) | (uint64_t)total);
        const uint64_t before = wave_lookback_prefix(lookback, tile, total, err);
        if (lane == 0) {
            s_prefix = before;
            s_total = total;
        }
    }
    __syncthreads();
    const uint64_t prefix = s_prefix;
    const uint64_t lt = (1ull << lane) - 1;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < CC_ITEMS; ++j) {
        const uint64_t b = __ballot((valid >> j) & 1ull);
        if (!((valid >> j) & 1ull)) continue;
        const uint64_t dst = prefix + s_cnt[j * WAVES + wid] + (uint64_t)__popcll(b & lt);
        const uint32_t e = (uint32_t)(first + j * CC_BLOCK + tid) / NPE;
        if (dst < (uint64_t)keys_cap) keys[dst] = ((uint64_t)(uint32_t)(id[j] - src.v_lo) << 32) | (uint64_t)e;
        else bad = true;
    }
    if (bad) set_error(err, ERR_INTERNAL);
    if (tid == 0 && s_total) atomicAdd(pair_count, s_total);
}

// dst[i] = src[i] + add for i < n.
constexpr int CR_BLOCK = 256;
static __global__ __launch_bounds__(CR_BLOCK) void chunk_rows_kernel(int32_t* __restrict__ dst,
                                                                    const int32_t* __restrict__ src, int64_t n,
                                                                    int32_t add) {
    const int64_t i = (int64_t)blockIdx.x * CR_BLOCK + threadIdx.x;
    if (i < n) dst[i] = src[i] + add;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool plan_chunked(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, bool node, bool elem_out,
                  ChunkPlan* p) {
    const int npe = nodes_per_elem(etype);
    if (npe == 0 || n_elem < 0 || n_vert < 0 || o.chunk_keys < CHUNK_MIN_KEYS) return false;
    // the node relation through the element rows only, 8-bit digits only
    if (node && o.node_sort != NS_ELEM_ROWS) return false;
    if (o.digit_bits == WBITS) return false;
    *p = ChunkPlan{};
    p->opts = o;
    p->n_elem = n_elem;
    p->etype = etype;
    p->n_vert = n_vert;
    p->n_slots = (int64_t)npe * n_elem;
    p->cap = o.chunk_keys;
    p->node = node;
    p->elem_out = elem_out;
    const uint32_t id_bits = id_bits_for(n_vert);
    p->coarse_bits = id_bits < (uint32_t)WBITS ? id_bits : (uint32_t)WBITS;
    p->coarse_shift = id_bits - p->coarse_bits;
    if (((int64_t)1 << p->coarse_shift) > p->cap) return false;  // one bin's vertices fit a range
    const int64_t cap = p->cap;

    size_t off = HEADER_BYTES;
    p->off_hist = off;
    off += align_up((size_t)MAX_EPASS * RADIX * sizeof(uint32_t));
    if (node) {  // the node stage's scan look-back: cleared with the header
        p->er.n_entries = cap;
        p->er.slots = npe - 1;
        p->er.n_tiles = erows_tiles_bound(cap);
        p->er.long_cap = erows_long_cap(cap);
        p->er.off_lb = off;
        p->er.lb_words = erows_scan_tiles((int32_t)cap) * 2;
        off += align_up((size_t)p->er.lb_words * sizeof(uint32_t));
    }
    // the compaction's look-back (one word per tile of CC_TILE slots) and
    // the first pass's, both cleared per range with the header; every pass
    // clears the next one's
    p->off_clb = off;
    off += align_up((size_t)ceil_div(p->n_slots, (int64_t)CC_TILE) * sizeof(uint64_t));
    p->off_lb0 = off;
    off += align_up(radix_lookback_bytes(cap, false));
    p->zero_bytes = off;
    p->off_lb1 = off;
    off += align_up(radix_lookback_bytes(cap, false));
    p->off_keys0 = off;
    off += align_up((size_t)cap * sizeof(uint64_t));
    p->off_keys1 = off;
    off += align_up((size_t)cap * sizeof(uint64_t));
    const size_t keys_end = off;
    p->off_bmin = off;
    off += align_up((size_t)ceil_div(cap + 1, (int64_t)RF_TILE) * sizeof(int32_t));
    p->off_erp = off;
    off += align_up(((size_t)cap + 1) * sizeof(int32_t));
    if (node && !elem_out) {
        p->off_ecols = off;
        off += align_up((size_t)cap * sizeof(int32_t));
    }
    p->off_bins = off;
    off += align_up((size_t)WRADIX * sizeof(uint32_t));
    // the coarse histogram's block partials are dead before the first range:
    // they share the key buffers when those are large enough
    const size_t part_bytes = (size_t)HIST_GRID_WIDE * WRADIX * sizeof(uint32_t);
    if (part_bytes <= keys_end - p->off_keys0) {
        p->off_part = p->off_keys0;
    } else {
        p->off_part = off;
        off += align_up(part_bytes);
    }
    if (node) {
        ErowsPlan& er = p->er;
        er.off_tf = off;
        off += align_up(((size_t)er.n_tiles + 1) * sizeof(int32_t));
        er.off_tc = off;
        off += align_up(((size_t)er.n_tiles + 1) * sizeof(int32_t));
        er.off_list = off;
        off += align_up((size_t)er.long_cap * sizeof(int32_t));
        er.off_deg = off;
        off += align_up(((size_t)cap + 1) * sizeof(int32_t));
        er.off_soff = off;
        off += align_up(((size_t)cap + 1) * sizeof(int16_t));
        er.temp_bytes = (size_t)er.slots * (size_t)cap * sizeof(int32_t);
        if (er.temp_bytes <= keys_end - p->off_keys0) {  // the keys are dead once a range's rows are written
            er.off_temp = p->off_keys0;
        } else {
            er.off_temp = off;
            off += align_up(er.temp_bytes);
        }
    }
    p->total = off;
    return true;
}

namespace {

struct Range {
    int32_t v0, v1;
    int64_t ebase, count;
};

// Ranges of whole bins (bin b holds the vertices [b << shift, (b + 1) << shift)),
// each of at most cap pairs and cap vertices, covering [0, n_vert).  false:
// one bin holds more than cap pairs.
bool cut_ranges(const uint32_t* bins, uint32_t coarse_bits, uint32_t shift, int32_t n_vert, int64_t cap,
                std::vector<Range>* out) {
    out->clear();
    const int64_t width = (int64_t)1 << shift;
    const int64_t n_bins = (int64_t)1 << coarse_bits;
    int64_t v0 = 0, count = 0, ebase = 0;
    for (int64_t b = 0; b < n_bins && b * width < n_vert; ++b) {
        const int64_t bv0 = b * width, bv1 = bv0 + width < n_vert ? bv0 + width : n_vert;
        const int64_t c = bins[b];
        if (c > cap) return false;
        if (bv0 > v0 && (count + c > cap || bv1 - v0 > cap)) {
            out->push_back(Range{(int32_t)v0, (int32_t)bv0, ebase, count});
            ebase += count;
            v0 = bv0;
            count = 0;
        }
        count += c;
    }
    if (v0 < n_vert) out->push_back(Range{(int32_t)v0, n_vert, ebase, count});
    return true;
}

template <int ET>
hipError_t run_range(const ChunkPlan& p, const Range& r, const int32_t* conn, int32_t* node_row_ptr,
                     int32_t* node_cols, int64_t node_cap, int32_t* elem_row_ptr, int32_t* elem_cols,
                     int64_t elem_cap, char* w, hipStream_t s) {
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    uint32_t* count = hdr + HDR_KEY_COUNT;
    uint32_t* hist = (uint32_t*)(w + p.off_hist);
    const int32_t nv = r.v1 - r.v0;
    int32_t* erp = (int32_t*)(w + p.off_erp);
    const FillRegion fill[2] = {header_fill(w, p.zero_bytes, /*keep_err=*/true),
                                {erp, (int64_t)nv + 1, r.count == 0 ? 0u : (uint32_t)INT32_MAX}};
    hipError_t e = fill_regions(fill, 2, s);
    if (e != hipSuccess) return e;

    // the range's element columns: in the caller's output at ebase, or in the
    // workspace for a node-only call
    int32_t* ecols;
    int64_t ecap;
    if (p.elem_out) {
        ecols = elem_cols ? elem_cols + r.ebase : nullptr;
        ecap = elem_cols && elem_cap > r.ebase ? elem_cap - r.ebase : 0;
    } else {
        ecols = (int32_t*)(w + p.off_ecols);
        ecap = r.count;
    }
    if (r.count > 0) {
        const PassPlan pp = plan_passes(id_bits_for(nv), RBITS);
        uint64_t* lb[2] = {(uint64_t*)(w + p.off_lb0), (uint64_t*)(w + p.off_lb1)};
        uint64_t* kb[2] = {(uint64_t*)(w + p.off_keys0), (uint64_t*)(w + p.off_keys1)};
        e = launch("chunk_compact", chunk_compact_kernel<ET>, dim3((unsigned)ceil_div(p.n_slots, CC_TILE)),
                   dim3(CC_BLOCK), s, ElemPairSrc<ET>{conn, nv, r.v0}, p.n_slots, kb[0], p.cap,
                   (uint64_t*)(w + p.off_clb), hdr + HDR_TICKET0 + TK_COMPACT, count, err);
        if (e == hipSuccess)
            e = launch("chunk_hist", key_hist_kernel,
                       dim3((unsigned)tmin<int64_t>(ceil_div(r.count, 4 * KH_BLOCK), CHUNK_HIST_GRID)), dim3(KH_BLOCK),
                       s, (const uint64_t*)kb[0], (const int32_t*)count, 32u, pp.n_pass, pp.width[pp.n_pass - 1],
                       hist);
        // every pass over the range's keys: pass q reads kb[q & 1] and clears
        // the look-back words of pass q + 1; the last writes the CSR
        const CsrOut csr{ecols, erp, ecols ? ecap : 0, 32u, 0xffffffffull};
        for (int q = 0; q < pp.n_pass && e == hipSuccess; ++q) {
            const bool last = q + 1 == pp.n_pass;
            const uint32_t shift = 32 + pp.shift[q], bits = pp.width[q];
            const CountedKeySrc src{kb[q & 1], count};
            uint32_t* ticket = hdr + HDR_TICKET0 + TK_PASS0 + q;
            if (last)
                e = launch_radix_pass("chunk_elem_radix", p.opts.shape, src, csr, r.count, shift, bits,
                                      hist + q * RADIX, lb[q & 1], nullptr, ticket, err, s);
            else
                e = launch_radix_pass("chunk_elem_radix", p.opts.shape, src, KeyOut{kb[(q + 1) & 1]}, r.count,
                                      shift, bits, hist + q * RADIX, lb[q & 1], lb[(q + 1) & 1], ticket, err, s);
        }
        if (e == hipSuccess)
            e = launch_rowptr_fill("chunk_elem_row_fill", erp, nv, count, (int32_t*)(w + p.off_bmin), s);
        if (e != hipSuccess) return e;
    }
    if (p.elem_out) {
        e = launch("chunk_rows", chunk_rows_kernel, dim3((unsigned)ceil_div((int64_t)nv + 1, CR_BLOCK)),
                   dim3(CR_BLOCK), s, elem_row_ptr + r.v0, (const int32_t*)erp, (int64_t)nv + 1, (int32_t)r.ebase);
        if (e != hipSuccess) return e;
    }
    if (!p.node) return hipSuccess;
    const ErowsBufs b = erows_bufs(p.er, w, err, hdr + HDR_TICKET0 + TK_EROWS);
    int32_t* rp = node_row_ptr + r.v0;  // rp[0]: the previous range's end, the base of this one's starts
    return launch_erows("chunk_node", UniformRows<ET>{conn, p.n_elem, p.n_vert, r.v0}, erp, ecols,
                        ecols ? ecap : 0, nv, r.count, rp, node_cols, node_cap, b, s, rp);
}

}  // namespace

mesh_status run_chunked(const ChunkPlan& p, const int32_t* conn, int32_t* node_row_ptr, int32_t* node_cols,
                        int64_t node_cap, int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cap, void* ws,
                        hipStream_t s) {
    char* w = (char*)ws;
    uint32_t* hdr = (uint32_t*)w;
    if (p.n_slots == 0) {  // no pairs: every row empty
        hipError_t e = zero_words(ws, HEADER_BYTES, s);
        if (e == hipSuccess && p.node) e = fill_i32(node_row_ptr, (int64_t)p.n_vert + 1, 0, s);
        if (e == hipSuccess && p.elem_out) e = fill_i32(elem_row_ptr, (int64_t)p.n_vert + 1, 0, s);
        return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
    }
    FillRegion fill[3] = {header_fill(ws, HEADER_BYTES, false)};
    int n_fill = 1;
    if (p.node) fill[n_fill++] = {node_row_ptr, 1, 0u};
    if (p.elem_out) fill[n_fill++] = {elem_row_ptr, 1, 0u};
    hipError_t e = fill_regions(fill, n_fill, s);
    if (e != hipSuccess) return MESH_ERR_HIP;

    // pairs per bin of the top vertex bits
    uint32_t* bins = (uint32_t*)(w + p.off_bins);
    e = with_type(p.etype, [&](auto et) {
        constexpr int ET = decltype(et)::value;
        DigitPlan dp{};
        dp.n_pass = 1;
        dp.shift[0] = p.coarse_shift;
        dp.mask[0] = (1u << p.coarse_bits) - 1;
        const int grid = (int)tmin<int64_t>(ceil_div(p.n_elem, HIST_BLOCK), HIST_GRID_WIDE);
        hipError_t x = launch("chunk_coarse", elem_hist_kernel<ET, WRADIX>, dim3(grid), dim3(HIST_BLOCK), s, conn,
                              p.n_elem, p.n_vert, 0, p.n_vert, dp, (uint32_t*)(w + p.off_part),
                              hdr + HDR_KEY_COUNT, hdr + HDR_ERR);
        if (x == hipSuccess)
            x = launch("chunk_coarse_sum", hist_sum_kernel, dim3((unsigned)ceil_div(WRADIX, HSUM_BLOCK)),
                       dim3(HSUM_BLOCK), s, (const uint32_t*)(w + p.off_part), grid, WRADIX, bins);
        return x;
    });
    if (e != hipSuccess) return MESH_ERR_HIP;
    const int64_t n_bins = (int64_t)1 << p.coarse_bits;
    std::vector<uint32_t> h_bins((size_t)n_bins);
    uint32_t h_hdr[HDR_KEY_COUNT + 1];
    e = hipMemcpyAsync(h_bins.data(), bins, (size_t)n_bins * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_hdr, hdr, sizeof h_hdr, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return MESH_ERR_HIP;
    uint64_t total = 0;
    for (uint32_t c : h_bins) total += c;
    if (total != h_hdr[HDR_KEY_COUNT]) return MESH_ERR_INTERNAL;

    std::vector<Range> ranges;
    if (!cut_ranges(h_bins.data(), p.coarse_bits, p.coarse_shift, p.n_vert, p.cap, &ranges)) return MESH_ERR_CHUNK;
    e = with_type(p.etype, [&](auto et) {
        constexpr int ET = decltype(et)::value;
        hipError_t x = hipSuccess;
        for (size_t i = 0; i < ranges.size() && x == hipSuccess; ++i)
            x = run_range<ET>(p, ranges[i], conn, node_row_ptr, node_cols, node_cap, elem_row_ptr, elem_cols,
                              elem_cap, w, s);
        return x;
    });
    return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

}  // namespace mnb
