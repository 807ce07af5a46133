// Kernels and the radix-pass driver of the element relation (Sec. 2.1.2,
// 2.2.2), shared by meshes of one element type (elem_path.hip) and meshes of
// several (mixed_path.hip).
#pragma once

#include "common.hpp"
#include "csr.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "radix.hpp"

namespace mnb {

constexpr int HIST_BLOCK = 512;
constexpr int HIST_GRID_MAX = 1024;
constexpr int HIST_UNROLL = 4;
constexpr int MAX_EPASS = 4;  // 31 vertex bits

// Ticket slots in the workspace header.
constexpr int TK_PASS0 = 0;  // passes 0..3

// The element holding slot s contains vertex v = conn[s] for the first time
// (set semantics for degenerate elements: a repeated id counts once).
template <int NPE>
__device__ __forceinline__ bool first_occurrence(const int32_t* __restrict__ conn, uint32_t e, int j, int32_t v) {
    bool first = true;
    const int32_t* el = conn + (size_t)e * NPE;
#pragma unroll
    for (int jj = 0; jj < NPE - 1; ++jj)
        if (jj < j) first &= el[jj] != v;
    return first;
}

// (vertex, element) pair of connectivity slot s as the key (u << 32) | e
// with u = v - v_lo, or KEY_NONE when the slot repeats an id of its element
// or v lies outside the window [v_lo, v_lo + n_vert) (the whole mesh unless a
// bounded-memory build sorts one vertex range at a time).
template <int ET>
struct ElemPairSrc {
    const int32_t* __restrict__ conn;
    int32_t n_vert;
    int32_t v_lo = 0;
    static constexpr bool kSkipNone = true;
    static constexpr bool kStaged = true;
    static constexpr int NPE = Elem<ET>::NPE;

    // ids of the tile's whole elements to s[0 ..): at most TILE + 2 * NPE words
    template <int BLOCK, int TILE>
    __device__ __forceinline__ void stage(int64_t tile_base, int64_t n, int32_t* s, int tid) const {
        constexpr int MAXC = TILE + 2 * NPE;
        constexpr int PER = (MAXC + BLOCK - 1) / BLOCK;
        static_assert(MAXC <= 2 * TILE, "staged ids fit the key staging area");
        const uint32_t e0 = (uint32_t)tile_base / NPE;
        const uint32_t e1 = ((uint32_t)tmin<int64_t>(tile_base + TILE, n) - 1u) / NPE;
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
    __device__ __forceinline__ uint64_t load_staged(Header, int64_t s, int64_t tile_base, const int32_t* st) const {
        const uint32_t ss = (uint32_t)s;
        const uint32_t e = ss / NPE;
        const int32_t* el = st + (e - (uint32_t)tile_base / NPE) * NPE;
        const int j = (int)(ss - e * NPE);
        const int32_t v = el[j];
        const uint32_t u = (uint32_t)(v - v_lo);
        if (u >= (uint32_t)n_vert) return KEY_NONE;
        bool first = true;
#pragma unroll
        for (int jj = 0; jj < NPE - 1; ++jj)
            if (jj < j) first &= el[jj] != v;
        return first ? ((uint64_t)u << 32) | (uint64_t)e : KEY_NONE;
    }

    __device__ __forceinline__ uint64_t load(int64_t s) const {
        const int32_t v = conn[s];
        const uint32_t u = (uint32_t)(v - v_lo);
        if (u >= (uint32_t)n_vert) return KEY_NONE;
        const uint32_t ss = (uint32_t)s;  // slot indices stay below 2^31
        const uint32_t e = ss / NPE;
        const int j = (int)(ss - e * NPE);
        if (!first_occurrence<NPE>(conn, e, j, v)) return KEY_NONE;
        return ((uint64_t)u << 32) | (uint64_t)e;
    }
};

// The digits of every pass of a sort over the vertex bits (shift and mask of
// the vertex id per pass), as the histogram kernels take them.
struct DigitPlan {
    int n_pass;
    uint32_t shift[MAX_EPASS];
    uint32_t mask[MAX_EPASS];
};
inline DigitPlan digit_plan(const PassPlan& pp) {
    DigitPlan d{};
    d.n_pass = pp.n_pass;
    for (int q = 0; q < pp.n_pass && q < MAX_EPASS; ++q) {
        d.shift[q] = pp.shift[q];
        d.mask[q] = (1u << pp.width[q]) - 1;
    }
    return d;
}
// Passes whose histograms one block keeps in LDS, per digit width.
constexpr int hist_passes(int radix) { return radix > RADIX ? 3 : MAX_EPASS; }

// Block histograms go to the global ones.  8-bit digits: added with global
// atomics.  Wider digits (HR = 2048 values per pass) would take eight times as
// many atomics, each a memory-side operation on this GPU, so every block
// stores its partial histograms whole at part + blockIdx.x * n_pass * HR and
// hist_sum_kernel adds them up.
template <int HR>
__device__ __forceinline__ void flush_hist(const uint32_t* s_hist, int n_words, uint32_t* __restrict__ hist,
                                           int tid, int nthreads) {
    if constexpr (HR > RADIX) {
        uint32_t* part = hist + (int64_t)blockIdx.x * n_words;
        for (int i = tid; i < n_words; i += nthreads) part[i] = s_hist[i];
    } else {
        for (int i = tid; i < n_words; i += nthreads)
            if (s_hist[i]) atomicAdd(&hist[i], s_hist[i]);
    }
}

// hist[i] = sum over the G blocks' partials part[b * n_words + i].
constexpr int HSUM_BLOCK = 256;
static __global__ __launch_bounds__(HSUM_BLOCK) void hist_sum_kernel(const uint32_t* __restrict__ part, int blocks,
                                                                    int n_words, uint32_t* __restrict__ hist) {
    const int i = blockIdx.x * HSUM_BLOCK + threadIdx.x;
    if (i >= n_words) return;
    uint32_t acc[4] = {0, 0, 0, 0};
    int b = 0;
    for (; b + 4 <= blocks; b += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += part[(int64_t)(b + u) * n_words + i];
    }
    for (; b < blocks; ++b) acc[0] += part[(int64_t)b * n_words + i];
    hist[i] = acc[0] + acc[1] + acc[2] + acc[3];
}

// Grid of a wide histogram kernel (one partial per block).
constexpr int HIST_GRID_WIDE = 256;

// Histograms of the digits of u = v - v_lo over the pairs whose vertex lies
// in the window [v_lo, v_lo + n_win) (pass q's digit values at hist[q * HR
// ..], or the block partials, see flush_hist), and their number.  A thread
// takes whole elements, HIST_UNROLL of them in flight; a repeated id inside
// an element counts once.  Raises ERR_INDEX_RANGE for an id outside
// [0, n_vert).
template <int ET, int HR>
__global__ __launch_bounds__(HIST_BLOCK) void elem_hist_kernel(const int32_t* __restrict__ conn, int64_t n_elem,
                                                              int32_t n_vert, int32_t v_lo, int32_t n_win,
                                                              DigitPlan dp, uint32_t* __restrict__ hist,
                                                              uint32_t* pair_count, uint32_t* err) {
    constexpr int NPE = Elem<ET>::NPE;
    __shared__ uint32_t s_hist[hist_passes(HR) * HR];
    __shared__ uint32_t s_pairs;
    const int tid = threadIdx.x;
    const int n_pass = dp.n_pass;
    if (tid == 0) s_pairs = 0;
    for (int i = tid; i < n_pass * HR; i += HIST_BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool bad = false;
    uint32_t pairs = 0;
    const int64_t stride = (int64_t)gridDim.x * HIST_BLOCK;
    for (int64_t e0 = (int64_t)blockIdx.x * HIST_BLOCK + tid; e0 < n_elem; e0 += stride * HIST_UNROLL) {
        int32_t id[HIST_UNROLL][NPE];
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; ++u) {  // all loads in flight first
            const int64_t e = e0 + u * stride;
            if (e < n_elem) load_elem_ids<ET>(conn, e, id[u]);
        }
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; ++u) {
            if (e0 + u * stride >= n_elem) continue;
#pragma unroll
            for (int j = 0; j < NPE; ++j) {
                const int32_t v = id[u][j];
                const uint32_t w = (uint32_t)(v - v_lo);
                bad |= (uint32_t)v >= (uint32_t)n_vert;
                bool take = w < (uint32_t)n_win;
#pragma unroll
                for (int jj = 0; jj < j; ++jj) take &= id[u][jj] != v;
                if (!take) continue;
                ++pairs;
                for (int p = 0; p < n_pass; ++p)
                    atomicAdd(&s_hist[p * HR + ((w >> dp.shift[p]) & dp.mask[p])], 1u);
            }
        }
    }
    if (bad) set_error(err, ERR_INDEX_RANGE);
    if (pairs) atomicAdd(&s_pairs, pairs);
    __syncthreads();
    if (tid == 0 && s_pairs) atomicAdd(pair_count, s_pairs);
    flush_hist<HR>(s_hist, n_pass * HR, hist, tid, HIST_BLOCK);
}

// The radix passes of the element relation over keys from `first` (the
// first pass's source); the last pass writes the CSR.  Shared by single
// meshes of one type and meshes of several types.
template <class First>
inline hipError_t elem_passes(const ElemPlan& p, First first, int32_t* row_ptr, int32_t* cols, int64_t cols_cap, char* w,
                       hipStream_t s) {
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    uint32_t* count = hdr + HDR_KEY_COUNT;
    uint32_t* hist = (uint32_t*)(w + p.off_hist);
    uint64_t* lb[2] = {(uint64_t*)(w + p.off_lb0), (uint64_t*)(w + p.off_lb1)};
    uint64_t* kb[2] = {(uint64_t*)(w + p.off_keys0), (uint64_t*)(w + p.off_keys1)};
    const int shape = p.opts.shape;
    const int n_pass = p.pp.n_pass;
    // the last pass (CsrOut) offers every row start: unset entries hold
    // INT32_MAX (set by the caller)
    const CsrOut csr{cols, row_ptr, cols ? cols_cap : 0, 32u, 0xffffffffull};
    hipError_t e = hipSuccess;
    const uint32_t hs = p.pp.hist_stride();
    auto pass = [&](const char* name, auto src, auto out, int q) {
        const uint32_t shift = 32 + p.pp.shift[q];
        const uint32_t bits = p.pp.width[q];
        uint64_t* lb_next = q + 1 == n_pass ? nullptr : lb[(q + 1) & 1];
        uint32_t* ticket = hdr + HDR_TICKET0 + TK_PASS0 + q;
        const uint32_t* hq = hist + q * hs;
        if (p.pp.wide)
            return launch_radix_wide(name, src, out, p.n_slots, shift, bits, hq, lb[q & 1], lb_next, ticket, err, s);
        return launch_radix_pass(name, shape, src, out, p.n_slots, shift, bits, hq, lb[q & 1], lb_next, ticket, err,
                                 s);
    };
    for (int q = 0; q < n_pass && e == hipSuccess; ++q) {
        const bool last = q + 1 == n_pass;
        const KeyOut out{kb[q & 1]};
        const CountedKeySrc later{kb[(q - 1) & 1], count};
        if (q == 0 && last) e = pass("elem_radix_first", first, csr, q);
        else if (q == 0) e = pass("elem_radix_first", first, out, q);
        else if (last) e = pass("elem_radix", later, csr, q);
        else e = pass("elem_radix", later, out, q);
    }
    if (e != hipSuccess) return e;
    return launch_rowptr_fill("elem_row_fill", row_ptr, p.n_vert, count, (int32_t*)(w + p.off_bmin), s);
}

}  // namespace mnb
