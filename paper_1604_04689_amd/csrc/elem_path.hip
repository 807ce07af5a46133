// One-ring neighboring elements (paper Sec. 2.1.2 and 2.2.2).
//
// The paper forms one (node, element) pair per node of every element and
// sorts the pairs by node.  Here each pair is the 64-bit key (v << 32) | e,
// generated straight from the connectivity by the first pass, and the keys
// are sorted by the bits of v only: a stable LSD radix sort over those bits,
// i.e. one counting sort per digit of the vertex id.  Pairs enter in element
// order and every pass is stable, so each vertex's elements come out
// ascending without a per-row sort.  A repeated id inside an element (a
// degenerate element) yields its pair once.  The last pass writes cols = e
// and offers each row start to row_ptr with an atomic minimum; a suffix
// minimum gives empty rows the next row's start.
//
// (A counting sort with one global atomic counter per vertex was measured
// first: on this GPU each device-scope atomic is a memory-side transaction,
// and the atomic count + scatter of a 25M-pair mesh took 3.5 ms.)
//
//   elem_hist        conn -> histograms of the vertex digits of every pass,
//                    and the number of pairs that take part
//   radix_pass x q   (v << 32 | e) keys, stable, by the digits of v; the last
//                    one writes cols and the row starts (CsrOut)
//   rowptr_fill      row starts of empty rows
#include "elem.hpp"

namespace mnb {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool plan_elem_slots(int64_t n_slots, int32_t n_vert, const Opts& o, ElemPlan* p) {
    if (n_slots < 0 || n_vert < 0) return false;
    p->opts = o;
    p->n_vert = n_vert;
    p->n_slots = n_slots;
    p->id_bits = id_bits_for(n_vert);
    int db = o.digit_bits < 0 ? default_elem_digit_bits(p->id_bits, n_slots) : o.digit_bits;
    if (n_slots >= LB32_MAX_KEYS) db = RBITS;  // the wide pass has 32-bit look-back words only
    p->pp = plan_passes(p->id_bits, db);
    p->n_tiles = ceil_div(p->n_slots, min_radix_tile());
    const size_t lb_bytes = align_up(radix_lookback_bytes(p->n_slots, p->pp.wide));
    size_t off = HEADER_BYTES;
    p->off_hist = off;
    off += align_up((size_t)MAX_EPASS * p->pp.hist_stride() * sizeof(uint32_t));
    p->off_lb0 = off;
    off += lb_bytes;
    p->zero_bytes = off;  // header, histograms, pass-0 look-back
    p->off_lb1 = off;
    off += p->pp.n_pass > 1 ? lb_bytes : 0;
    p->off_keys0 = off;
    off += align_up((size_t)p->n_slots * sizeof(uint64_t));
    p->off_keys1 = off;
    off += p->pp.n_pass > 1 ? align_up((size_t)p->n_slots * sizeof(uint64_t)) : 0;
    p->off_bmin = off;
    off += align_up((size_t)ceil_div((int64_t)n_vert + 1, (int64_t)RF_TILE) * sizeof(int32_t));
    if (p->pp.wide) {  // block partials of the wide histograms
        p->off_part = off;
        off += align_up((size_t)HIST_GRID_WIDE * p->pp.n_pass * WRADIX * sizeof(uint32_t));
    }
    p->total = off;
    return true;
}

bool plan_elem(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, ElemPlan* p, size_t) {
    const int npe = nodes_per_elem(etype);
    if (npe == 0 || n_elem < 0 || n_vert < 0) return false;
    *p = ElemPlan{};
    if (!plan_elem_slots((int64_t)npe * n_elem, n_vert, o, p)) return false;
    p->n_elem = n_elem;
    p->etype = etype;
    return true;
}

template <int ET>
static hipError_t elem_pipeline(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                                int64_t cols_cap, char* w, hipStream_t s) {
    uint32_t* hdr = (uint32_t*)w;
    const int grid = (int)tmin<int64_t>(ceil_div(p.n_elem, HIST_BLOCK), HIST_GRID_MAX);
    const DigitPlan dp = digit_plan(p.pp);
    hipError_t e;
    if (p.pp.wide) {
        const int n_words = dp.n_pass * WRADIX;
        const int wgrid = (int)tmin<int64_t>(grid, HIST_GRID_WIDE);
        uint32_t* part = (uint32_t*)(w + p.off_part);
        e = launch("elem_hist", elem_hist_kernel<ET, WRADIX>, dim3(wgrid), dim3(HIST_BLOCK), s, conn, p.n_elem, p.n_vert,
                   0, p.n_vert, dp, part, hdr + HDR_KEY_COUNT, hdr + HDR_ERR);
        if (e == hipSuccess)
            e = launch("hist_sum", hist_sum_kernel, dim3((unsigned)ceil_div(n_words, HSUM_BLOCK)), dim3(HSUM_BLOCK), s,
                       (const uint32_t*)part, wgrid, n_words, (uint32_t*)(w + p.off_hist));
    } else {
        e = launch("elem_hist", elem_hist_kernel<ET, RADIX>, dim3(grid), dim3(HIST_BLOCK), s, conn, p.n_elem, p.n_vert,
                   0, p.n_vert, dp, (uint32_t*)(w + p.off_hist), hdr + HDR_KEY_COUNT, hdr + HDR_ERR);
    }
    if (e != hipSuccess) return e;
    return elem_passes(p, ElemPairSrc<ET>{conn, p.n_vert}, row_ptr, cols, cols_cap, w, s);
}

hipError_t run_elem(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                    void* ws, hipStream_t s, bool keep_err, const FillRegion* extra) {
    FillRegion fill[3] = {header_fill(ws, p.zero_bytes, keep_err),
                          {row_ptr, (int64_t)p.n_vert + 1, p.n_slots == 0 ? 0u : (uint32_t)INT32_MAX}};
    int n_fill = 2;
    if (extra) fill[n_fill++] = *extra;
    hipError_t e = fill_regions(fill, n_fill, s);
    if (e != hipSuccess || p.n_slots == 0) return e;
    return with_type(p.etype, [&](auto et) {
        return elem_pipeline<decltype(et)::value>(p, conn, row_ptr, cols, cols_capacity, (char*)ws, s);
    });
}

}  // namespace mnb
