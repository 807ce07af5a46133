// One-ring neighboring elements (paper Sec. 2.1.2 and 2.2.2).
//
// The paper forms one (node, element) pair per node of every element and
// sorts the pairs by node.  Here the sort by node is a counting sort: the
// number of distinct elements per vertex is counted with atomics, scanned to
// row starts, element ids are scattered into their rows through per-vertex
// cursors, and each row is then sorted ascending, which makes the (otherwise
// arrival-ordered) result canonical.
//
//   elem_count     conn -> per-vertex counts            (atomics)
//   elem_scan      counts -> row_ptr, cursors           (single-pass look-back scan)
//   elem_scatter   conn -> cols in arrival order        (atomics on cursors)
//   elem_rowsort   rows <= 64 sorted per thread in LDS; longer rows listed
//   elem_longrows  listed rows: bitonic sort per block (LDS, or global memory)
#include <climits>

#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int EC_BLOCK = 256;
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
constexpr int RS_BLOCK = 256;    // rows per row-sort block (one per thread)
constexpr int RS_LDS = 8192;     // int32 slots staged per row-sort block
constexpr int RS_SHORT = 64;     // longest row sorted by a single thread
constexpr int LR_BLOCK = 256;
constexpr int LR_LDS = 8192;     // longest row sorted in LDS by one block
constexpr int LR_GRID = 256;

// The element holding slot s contains vertex v = conn[s] for the first time
// (set semantics for degenerate elements: a repeated id counts once).
template <int NPE>
__device__ __forceinline__ bool first_occurrence(const int32_t* __restrict__ conn, int64_t e, int j, int32_t v) {
    bool first = true;
#pragma unroll
    for (int jj = 0; jj < NPE - 1; ++jj)
        if (jj < j) first &= conn[e * NPE + jj] != v;
    return first;
}

template <int ET>
__global__ __launch_bounds__(EC_BLOCK) void elem_count_kernel(const int32_t* __restrict__ conn, int64_t n_slots,
                                                             int32_t n_vert, uint32_t* __restrict__ cnt,
                                                             uint32_t* err) {
    constexpr int NPE = Elem<ET>::NPE;
    const int64_t s = (int64_t)blockIdx.x * EC_BLOCK + threadIdx.x;
    if (s >= n_slots) return;
    const int32_t v = conn[s];
    if ((uint32_t)v >= (uint32_t)n_vert) {
        set_error(err, ERR_INDEX_RANGE);
        return;
    }
    const int64_t e = s / NPE;
    const int j = (int)(s - e * NPE);
    if (first_occurrence<NPE>(conn, e, j, v)) atomicAdd(&cnt[v], 1u);
}

// Exclusive scan of the counts: row_ptr[v] = sum of counts below v, and the
// cursor of v starts at its row start.  row_ptr[n_vert] = total.
__global__ __launch_bounds__(SCAN_BLOCK) void elem_scan_kernel(uint32_t* __restrict__ cnt, int32_t n_vert,
                                                              int32_t* __restrict__ row_ptr, uint64_t* lookback,
                                                              uint32_t* ticket, uint32_t* err) {
    constexpr int WAVES = SCAN_BLOCK / WAVE;
    static_assert(SCAN_ITEMS * WAVES <= WAVE, "one wave scans the item/wave sums");
    __shared__ uint32_t s_sum[SCAN_ITEMS * WAVES];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * SCAN_TILE;
    uint32_t c[SCAN_ITEMS], ex[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t v = base + j * SCAN_BLOCK + wid * WAVE + lane;
        c[j] = v < n_vert ? cnt[v] : 0u;
        const uint32_t incl = wave_inclusive_sum(c[j]);
        ex[j] = incl - c[j];
        if (lane == WAVE - 1) s_sum[j * WAVES + wid] = incl;
    }
    __syncthreads();
    if (wid == 0) {
        const uint32_t v = lane < SCAN_ITEMS * WAVES ? s_sum[lane] : 0u;
        const uint32_t incl = wave_inclusive_sum(v);
        if (lane < SCAN_ITEMS * WAVES) s_sum[lane] = incl - v;
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        if (lane == 0) {
            lb_store(lookback + tile, (tile == 0 ? LB_INC : LB_AGG) | total);
            s_prefix = lookback_prefix(lookback, 1, tile, total, err);
        }
    }
    __syncthreads();
    const uint64_t prefix = s_prefix;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t v = base + j * SCAN_BLOCK + wid * WAVE + lane;
        if (v < n_vert) {
            const uint32_t start = (uint32_t)(prefix + s_sum[j * WAVES + wid] + ex[j]);
            row_ptr[v] = (int32_t)start;
            cnt[v] = start;
            if (v == n_vert - 1) row_ptr[n_vert] = (int32_t)(start + c[j]);
        }
    }
}

template <int ET>
__global__ __launch_bounds__(EC_BLOCK) void elem_scatter_kernel(const int32_t* __restrict__ conn, int64_t n_slots,
                                                               int32_t n_vert, uint32_t* __restrict__ cursor,
                                                               int32_t* __restrict__ cols, int64_t cols_cap,
                                                               uint32_t* err) {
    constexpr int NPE = Elem<ET>::NPE;
    const int64_t s = (int64_t)blockIdx.x * EC_BLOCK + threadIdx.x;
    if (s >= n_slots) return;
    const int32_t v = conn[s];
    if ((uint32_t)v >= (uint32_t)n_vert) return;  // already flagged by elem_count
    const int64_t e = s / NPE;
    const int j = (int)(s - e * NPE);
    if (!first_occurrence<NPE>(conn, e, j, v)) return;
    const uint32_t pos = atomicAdd(&cursor[v], 1u);
    if ((int64_t)pos < cols_cap) cols[pos] = (int32_t)e;
    else set_error(err, ERR_CAPACITY);
}

__device__ __forceinline__ void insertion_sort(int32_t* a, int n) {
    for (int i = 1; i < n; ++i) {
        const int32_t x = a[i];
        int k = i - 1;
        while (k >= 0 && a[k] > x) {
            a[k + 1] = a[k];
            --k;
        }
        a[k + 1] = x;
    }
}

__device__ __forceinline__ int64_t clamp_cap(int64_t x, int64_t cap) { return x < cap ? x : cap; }

__global__ __launch_bounds__(RS_BLOCK) void elem_rowsort_kernel(const int32_t* __restrict__ row_ptr, int32_t n_vert,
                                                               int32_t* __restrict__ cols, int64_t cols_cap,
                                                               int32_t* __restrict__ long_list, int64_t long_cap,
                                                               uint32_t* long_count, uint32_t* err) {
    __shared__ int32_t s_cols[RS_LDS];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * RS_BLOCK;
    const int64_t r1 = tmin<int64_t>(r0 + RS_BLOCK, n_vert);
    const int64_t beg = clamp_cap(row_ptr[r0], cols_cap);
    const int64_t end = clamp_cap(row_ptr[r1], cols_cap);
    const bool staged = end - beg <= RS_LDS;
    const int64_t r = r0 + tid;
    const bool has = r < r1;
    const int64_t rb = has ? clamp_cap(row_ptr[r], cols_cap) : 0;
    const int64_t re = has ? clamp_cap(row_ptr[r + 1], cols_cap) : 0;
    const int len = (int)(re - rb);
    if (staged) {
        for (int64_t i = tid; i < end - beg; i += RS_BLOCK) s_cols[i] = cols[beg + i];
        __syncthreads();
    }
    if (has && len > 1) {
        if (len <= RS_SHORT) {
            insertion_sort(staged ? s_cols + (rb - beg) : cols + rb, len);
        } else {
            const uint32_t slot = atomicAdd(long_count, 1u);
            if ((int64_t)slot < long_cap) long_list[slot] = (int32_t)r;
            else set_error(err, ERR_INTERNAL);
        }
    }
    if (staged) {
        __syncthreads();
        for (int64_t i = tid; i < end - beg; i += RS_BLOCK) cols[beg + i] = s_cols[i];
    }
}

// Rows longer than RS_SHORT: one block per row.  Up to LR_LDS entries the row
// is padded with INT_MAX to a power of two and bitonic-sorted in LDS; longer
// rows run the same network in place in global memory, in its form where
// every comparator puts the smaller value at the lower index, so the virtual
// INT_MAX padding never moves and its comparators are skipped.
__global__ __launch_bounds__(LR_BLOCK) void elem_longrows_kernel(const int32_t* __restrict__ row_ptr,
                                                                int32_t* cols, int64_t cols_cap,
                                                                const int32_t* __restrict__ long_list,
                                                                int64_t long_cap, const uint32_t* long_count) {
    __shared__ int32_t s[LR_LDS];
    const int tid = threadIdx.x;
    const int64_t n_long = tmin<int64_t>(*long_count, long_cap);
    for (int64_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const int32_t r = long_list[li];
        const int64_t rb = clamp_cap(row_ptr[r], cols_cap);
        const int64_t len = clamp_cap(row_ptr[r + 1], cols_cap) - rb;
        int64_t n2 = 1;
        while (n2 < len) n2 <<= 1;
        if (len <= LR_LDS) {
            for (int64_t i = tid; i < n2; i += LR_BLOCK) s[i] = i < len ? cols[rb + i] : INT_MAX;
            __syncthreads();
            for (int64_t k = 2; k <= n2; k <<= 1) {
                for (int64_t j = k >> 1; j > 0; j >>= 1) {
                    for (int64_t i = tid; i < n2; i += LR_BLOCK) {
                        const int64_t p = i ^ j;
                        if (p > i) {
                            const int32_t a = s[i], c = s[p];
                            const bool up = (i & k) == 0;
                            if ((a > c) == up) {
                                s[i] = c;
                                s[p] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int64_t i = tid; i < len; i += LR_BLOCK) cols[rb + i] = s[i];
        } else {
            int32_t* x = cols + rb;
            for (int64_t k = 2; k <= n2; k <<= 1) {
                for (int64_t j = k >> 1; j > 0; j >>= 1) {
                    for (int64_t i = tid; i < len; i += LR_BLOCK) {
                        const int64_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
                        if (p > i && p < len) {
                            const int32_t a = x[i], c = x[p];
                            if (a > c) {
                                x[i] = c;
                                x[p] = a;
                            }
                        }
                    }
                    __threadfence_block();
                    __syncthreads();
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool plan_elem(int64_t n_elem, int32_t etype, int32_t n_vert, ElemPlan* p) {
    const int npe = nodes_per_elem(etype);
    if (npe == 0 || n_elem < 0 || n_vert < 0) return false;
    p->n_elem = n_elem;
    p->etype = etype;
    p->n_vert = n_vert;
    p->n_slots = (int64_t)npe * n_elem;
    p->n_stiles = ceil_div(n_vert, SCAN_TILE);
    p->long_cap = p->n_slots / (RS_SHORT + 1) + 1;
    size_t off = HEADER_BYTES;
    p->off_cursor = off;
    off += align_up((size_t)n_vert * sizeof(uint32_t));
    p->off_lb = off;
    off += align_up((size_t)p->n_stiles * sizeof(uint64_t));
    p->zero_bytes = off;  // header, cursors, look-back
    p->off_long = off;
    off += align_up((size_t)p->long_cap * sizeof(int32_t));
    p->total = off;
    return true;
}

template <int ET>
static hipError_t launch_count_scatter(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                                       int64_t cols_cap, uint32_t* cursor, uint64_t* lb, uint32_t* hdr,
                                       hipStream_t s) {
    uint32_t* err = hdr + HDR_ERR;
    const dim3 grid((unsigned)ceil_div(p.n_slots, EC_BLOCK));
    hipError_t e = launch("elem_count", elem_count_kernel<ET>, grid, dim3(EC_BLOCK), s, conn, p.n_slots, p.n_vert,
                          cursor, err);
    if (e != hipSuccess || p.n_vert == 0) return e;
    e = launch("elem_scan", elem_scan_kernel, dim3((unsigned)p.n_stiles), dim3(SCAN_BLOCK), s, cursor, p.n_vert,
               row_ptr, lb, hdr + HDR_TICKET0, err);
    if (e != hipSuccess) return e;
    return launch("elem_scatter", elem_scatter_kernel<ET>, grid, dim3(EC_BLOCK), s, conn, p.n_slots, p.n_vert,
                  cursor, cols, cols_cap, err);
}

hipError_t run_elem(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                    void* ws, hipStream_t s) {
    char* w = (char*)ws;
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* cursor = (uint32_t*)(w + p.off_cursor);
    uint64_t* lb = (uint64_t*)(w + p.off_lb);
    int32_t* long_list = (int32_t*)(w + p.off_long);

    hipError_t e = zero_words(ws, p.zero_bytes, s);
    if (e != hipSuccess) return e;
    if (p.n_slots == 0) return fill_i32(row_ptr, (int64_t)p.n_vert + 1, 0, s);
    switch (p.etype) {
        case TRI3: e = launch_count_scatter<TRI3>(p, conn, row_ptr, cols, cols_capacity, cursor, lb, hdr, s); break;
        case TET4: e = launch_count_scatter<TET4>(p, conn, row_ptr, cols, cols_capacity, cursor, lb, hdr, s); break;
        default: e = launch_count_scatter<HEX8>(p, conn, row_ptr, cols, cols_capacity, cursor, lb, hdr, s); break;
    }
    if (e != hipSuccess) return e;
    if (p.n_vert == 0) return fill_i32(row_ptr, 1, 0, s);  // every id was out of range
    e = launch("elem_rowsort", elem_rowsort_kernel, dim3((unsigned)ceil_div(p.n_vert, RS_BLOCK)), dim3(RS_BLOCK), s,
               row_ptr, p.n_vert, cols, cols_capacity, long_list, p.long_cap, hdr + HDR_LONG_COUNT, hdr + HDR_ERR);
    if (e != hipSuccess) return e;
    return launch("elem_longrows", elem_longrows_kernel, dim3(LR_GRID), dim3(LR_BLOCK), s, row_ptr, cols,
                  cols_capacity, long_list, p.long_cap, hdr + HDR_LONG_COUNT);
}

}  // namespace mnb
