// Meshes whose elements carry their own types (the paper's claim that the
// method applies to meshes of any element type, Sec. 2.2 and Sec. 4, taken to
// meshes that mix them).  Element e has type etypes[e] and ids
// conn[elem_off[e] .. elem_off[e+1]).
//
//   mixed_map     slot -> element for every well-formed element (others are
//                 reported and left out)
//   mixed_hist    digit histograms of the (v, e) pairs, the pair count
//   radix_pass x q  the element relation's counting-sort passes by v, the
//                 first reading the pairs through the map, the last writing
//                 the element CSR
//   erows_*       the node relation from the element relation (ELEM_ROWS)
#include "elem.hpp"
#include "erows.hpp"
#include "internal.hpp"

namespace mnb {

constexpr int MX_BLOCK = 256;
constexpr int MX_GRID_MAX = 2048;

// map[s] = e for the slots s of every element e whose type is known and
// whose offsets span exactly its node count inside [0, n_ids); the map holds
// -1 beforehand.  Other elements raise ERR_INDEX_RANGE.
static __global__ __launch_bounds__(MX_BLOCK) void mixed_map_kernel(const int32_t* __restrict__ elem_off,
                                                                   const uint8_t* __restrict__ etypes,
                                                                   int64_t n_elem, int64_t n_ids,
                                                                   int32_t* __restrict__ map, uint32_t* err) {
    const int64_t e = (int64_t)blockIdx.x * MX_BLOCK + threadIdx.x;
    if (e >= n_elem) return;
    const int32_t a = elem_off[e], b = elem_off[e + 1];
    const int npe = nodes_per_elem(etypes[e]);
    if (npe == 0 || a < 0 || b - a != npe || (int64_t)b > n_ids) {
        set_error(err, ERR_INDEX_RANGE);
        return;
    }
    for (int j = 0; j < npe; ++j) map[a + j] = (int32_t)e;
}

// (vertex, element) pair of slot s: (v << 32) | e, or KEY_NONE for a slot of
// no well-formed element, an id outside [0, n_vert), or an id repeated
// earlier inside its element.
struct MixedElemPairSrc {
    const int32_t* __restrict__ conn;
    const int32_t* __restrict__ map;
    const int32_t* __restrict__ elem_off;
    int32_t n_vert;
    static constexpr bool kSkipNone = true;
    __device__ __forceinline__ uint64_t make(int64_t s, bool* bad) const {
        const int32_t e = map[s];
        if (e < 0) return KEY_NONE;
        const int32_t v = conn[s];
        if ((uint32_t)v >= (uint32_t)n_vert) {
            *bad = true;
            return KEY_NONE;
        }
        const int64_t a = elem_off[e];  // s lies in [a, a + npe): the map says so
#pragma unroll
        for (int j = 0; j < MAX_NPE - 1; ++j)
            if (a + j < s && conn[a + j] == v) return KEY_NONE;
        return ((uint64_t)(uint32_t)v << 32) | (uint64_t)(uint32_t)e;
    }
    __device__ __forceinline__ uint64_t load(int64_t s) const {
        bool bad = false;
        return make(s, &bad);
    }
};

// Digit histograms of v over the pairs that take part (pass q at
// hist[q * HR ..]), and their number.
template <int HR>
static __global__ __launch_bounds__(MX_BLOCK) void mixed_hist_kernel(MixedElemPairSrc src, int64_t n_ids, DigitPlan dp,
                                                                    uint32_t* __restrict__ hist, uint32_t* pair_count,
                                                                    uint32_t* err) {
    __shared__ uint32_t s_hist[hist_passes(HR) * HR];
    __shared__ uint32_t s_pairs;
    const int tid = threadIdx.x;
    const int n_pass = dp.n_pass;
    if (tid == 0) s_pairs = 0;
    for (int i = tid; i < n_pass * HR; i += MX_BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool bad = false;
    uint32_t pairs = 0;
    for (int64_t s = (int64_t)blockIdx.x * MX_BLOCK + tid; s < n_ids; s += (int64_t)gridDim.x * MX_BLOCK) {
        const uint64_t k = src.make(s, &bad);
        if (k == KEY_NONE) continue;
        ++pairs;
        const uint32_t v = (uint32_t)(k >> 32);
        for (int p = 0; p < n_pass; ++p) atomicAdd(&s_hist[p * HR + ((v >> dp.shift[p]) & dp.mask[p])], 1u);
    }
    if (bad) set_error(err, ERR_INDEX_RANGE);
    if (pairs) atomicAdd(&s_pairs, pairs);
    __syncthreads();
    if (tid == 0 && s_pairs) atomicAdd(pair_count, s_pairs);
    flush_hist<HR>(s_hist, n_pass * HR, hist, tid, MX_BLOCK);
}

bool plan_mixed(int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert, const Opts& o, MixedPlan* p) {
    if (n_elem < 0 || n_ids < 0 || n_pairs < 0 || n_vert < 0) return false;
    *p = MixedPlan{};
    p->opts = o;
    p->n_elem = n_elem;
    p->n_ids = n_ids;
    p->n_pairs = n_pairs;
    p->n_vert = n_vert;
    if (!plan_elem_slots(n_ids, n_vert, o, &p->ep)) return false;
    size_t off = p->ep.total;
    p->off_map = off;
    off += align_up((size_t)n_ids * sizeof(int32_t));
    off = plan_erows(n_ids, MAX_NPE - 1, n_vert, off, p->ep.off_keys0, p->ep.off_bmin - p->ep.off_keys0, &p->er);
    p->zero_bytes = p->ep.zero_bytes;
    p->total = off;
    return true;
}

hipError_t run_mixed(const MixedPlan& p, const int32_t* conn, const int32_t* elem_off, const uint8_t* etypes,
                     int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cap, int32_t* elem_row_ptr,
                     int32_t* elem_cols, int64_t elem_cap, void* ws, hipStream_t s) {
    char* w = (char*)ws;
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    int32_t* map = (int32_t*)(w + p.off_map);
    const FillRegion fill[4] = {{ws, (int64_t)(p.zero_bytes / 4), 0u},
                                {elem_row_ptr, (int64_t)p.n_vert + 1, p.n_ids == 0 ? 0u : (uint32_t)INT32_MAX},
                                {w + p.er.off_lb, p.er.lb_words, 0u},
                                {map, p.n_ids, 0xffffffffu}};
    hipError_t e = fill_regions(fill, 4, s);
    if (e != hipSuccess) return e;
    if (p.n_ids == 0 || p.n_elem == 0) {
        e = fill_i32(elem_row_ptr, (int64_t)p.n_vert + 1, 0, s);
        if (e == hipSuccess) e = fill_i32(node_row_ptr, (int64_t)p.n_vert + 1, 0, s);
        return e;
    }
    e = launch("mixed_map", mixed_map_kernel, dim3((unsigned)ceil_div(p.n_elem, MX_BLOCK)), dim3(MX_BLOCK), s,
               elem_off, etypes, p.n_elem, p.n_ids, map, err);
    const MixedElemPairSrc src{conn, map, elem_off, p.n_vert};
    const DigitPlan dp = digit_plan(p.ep.pp);
    if (e == hipSuccess && p.ep.pp.wide) {
        const int n_words = dp.n_pass * WRADIX;
        const int grid = (int)tmin<int64_t>(ceil_div(p.n_ids, MX_BLOCK), HIST_GRID_WIDE);
        uint32_t* part = (uint32_t*)(w + p.ep.off_part);
        e = launch("mixed_hist", mixed_hist_kernel<WRADIX>, dim3(grid), dim3(MX_BLOCK), s, src, p.n_ids, dp, part,
                   hdr + HDR_KEY_COUNT, err);
        if (e == hipSuccess)
            e = launch("hist_sum", hist_sum_kernel, dim3((unsigned)ceil_div(n_words, HSUM_BLOCK)), dim3(HSUM_BLOCK), s,
                       (const uint32_t*)part, grid, n_words, (uint32_t*)(w + p.ep.off_hist));
    } else if (e == hipSuccess) {
        e = launch("mixed_hist", mixed_hist_kernel<RADIX>,
                   dim3((unsigned)tmin<int64_t>(ceil_div(p.n_ids, MX_BLOCK), MX_GRID_MAX)), dim3(MX_BLOCK), s, src,
                   p.n_ids, dp, (uint32_t*)(w + p.ep.off_hist), hdr + HDR_KEY_COUNT, err);
    }
    if (e == hipSuccess) e = elem_passes(p.ep, src, elem_row_ptr, elem_cols, elem_cap, w, s);
    if (e != hipSuccess) return e;
    const ErowsBufs b = erows_bufs(p.er, w, err, hdr + HDR_TICKET0 + TK_EROWS);
    return launch_erows("mixed", MixedRows{conn, elem_off, etypes, p.n_elem, p.n_ids, p.n_vert}, elem_row_ptr,
                        elem_cols, elem_cap, p.n_vert, p.n_ids, node_row_ptr, node_cols, node_cap, b, s);
}

}  // namespace mnb
