// Per-row canonicalisation of pair keys that are sorted by their high part
// only: keys (hi << b) | lo arrive grouped by hi (one group = one row, i.e.
// one vertex), with the lo values of a row in any order and possibly
// repeated.  For every row the distinct lo values are written ascending to
// temp[start .. start + count) (start = index of the row's first key), with
// deg[hi] = count and src[hi] = start.  A scan of deg then gives row_ptr and
// a gather moves each row to cols.  This is the paper's sort by the first
// array (Sec. 2.2.1) followed by the duplicate-free, ascending rows of our
// reading of the serial solution (Sec. 3.2.2).
#pragma once

#include <climits>

#include "common.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int ROW_BLOCK = 256;
constexpr int ROW_TILE = 4096;   // keys whose rows a block owns
constexpr int ROW_HALO = 1024;   // keys read past the tile to finish its last row
constexpr int ROW_SHORT = 256;   // longest row ranked in LDS; longer rows are listed
constexpr int LONG_BLOCK = 256;
constexpr int LONG_LDS = 16384;  // longest row sorted in LDS by one block
constexpr int LONG_GRID = 256;
constexpr int GATHER_BLOCK = 256;

// A block owns the rows whose first key lies in its tile.  Each key of such a
// row finds its row's extent in LDS, decides whether it is the first copy of
// its lo value, and (after a barrier) counts the distinct values below it:
// that count is its place in the row.  Rows longer than ROW_SHORT, or not
// ending inside the halo, are listed (by first key index) for long_rows.
static __global__ __launch_bounds__(ROW_BLOCK) void row_unique_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                              uint32_t b, int32_t n_vert, int32_t* __restrict__ deg,
                                                              int64_t* __restrict__ src, int32_t* __restrict__ temp,
                                                              int64_t* __restrict__ long_list, int64_t long_cap,
                                                              uint32_t* long_count, uint32_t* err) {
    constexpr int SPAN = ROW_TILE + ROW_HALO;
    constexpr int PER = SPAN / ROW_BLOCK;
    __shared__ uint64_t s_k[SPAN + 1];    // s_k[0] = key before the tile, s_k[1 + p] = key base + p
    __shared__ uint8_t s_start[SPAN + 1];  // s_start[p]: position p starts a row (p = SPAN: sentinel)
    __shared__ uint8_t s_first[SPAN];      // position p holds the first copy of its lo value in its row
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * ROW_TILE;
    const int span = (int)tmin<int64_t>(SPAN, n - base);
    const uint64_t lo_mask = (1ull << b) - 1;
    {
        uint64_t k[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int p = q * ROW_BLOCK + tid;
            k[q] = p < span ? keys[base + p] : KEY_NONE;
        }
        const uint64_t before = (tid == 0 && base > 0) ? keys[base - 1] : KEY_NONE;
#pragma unroll
        for (int q = 0; q < PER; ++q) s_k[1 + q * ROW_BLOCK + tid] = k[q];
        if (tid == 0) s_k[0] = before;
    }
    __syncthreads();
    // row starts: a real key whose hi differs from its predecessor's (the
    // first real key of the array starts a row; KEY_NONE ends the data)
    for (int p = tid; p <= SPAN; p += ROW_BLOCK) {
        bool st;
        if (p == SPAN || p >= span) st = true;
        else {
            const uint64_t cur = s_k[1 + p];
            if (cur == KEY_NONE) st = true;
            else if (base + p == 0) st = true;
            else st = (cur >> b) != (s_k[p] >> b) || s_k[p] == KEY_NONE;
        }
        s_start[p] = st;
    }
    __syncthreads();
    // owned region: from the first row start in the tile to the first row start at or after ROW_TILE
    // (every thread finds the same bounds)
    int p0 = ROW_TILE, pe = SPAN;
    for (int p = 0; p < ROW_TILE; ++p)
        if (s_start[p]) {
            p0 = p;
            break;
        }
    for (int p = ROW_TILE; p <= SPAN; ++p)
        if (s_start[p]) {
            pe = p;
            break;
        }
    if (p0 >= ROW_TILE) return;  // the tile lies inside a row owned by an earlier tile
    // keep flags
    bool bad = false;
    for (int p = p0 + tid; p < pe; p += ROW_BLOCK) {
        const uint64_t cur = s_k[1 + p];
        if (cur == KEY_NONE) continue;
        int rs = p;
        while (!s_start[rs]) --rs;
        int re = p + 1;
        while (!s_start[re]) ++re;
        if (re - rs > ROW_SHORT || (re == SPAN && base + SPAN < n)) {
            if (p == rs) {
                const uint32_t slot = atomicAdd(long_count, 1u);
                if ((int64_t)slot < long_cap) long_list[slot] = base + rs;
                else bad = true;
            }
            s_first[p] = 0;
            continue;
        }
        const uint64_t lo = cur & lo_mask;
        bool first = true;
        for (int j = rs; j < p; ++j) first &= (s_k[1 + j] & lo_mask) != lo;
        s_first[p] = first;
    }
    __syncthreads();
    for (int p = p0 + tid; p < pe; p += ROW_BLOCK) {
        const uint64_t cur = s_k[1 + p];
        if (cur == KEY_NONE) continue;
        int rs = p;
        while (!s_start[rs]) --rs;
        int re = p + 1;
        while (!s_start[re]) ++re;
        if (re - rs > ROW_SHORT || (re == SPAN && base + SPAN < n)) continue;
        const uint64_t lo = cur & lo_mask;
        if (s_first[p]) {
            int below = 0;
            for (int j = rs; j < re; ++j) below += (s_first[j] && (s_k[1 + j] & lo_mask) < lo) ? 1 : 0;
            temp[base + rs + below] = (int32_t)lo;
        }
        if (p == rs) {
            int cnt = 0;
            for (int j = rs; j < re; ++j) cnt += s_first[j];
            const int64_t hi = (int64_t)(cur >> b);
            if (hi < n_vert) {
                deg[hi] = cnt;
                src[hi] = base + rs;
            } else {
                bad = true;
            }
        }
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// Rows longer than ROW_SHORT: one block per listed row.  The lo values are
// copied to the row's temp range, sorted (bitonic, in LDS up to LONG_LDS
// entries, else in place in global memory with every comparator putting the
// smaller value at the lower index, so virtual INT_MAX padding never moves),
// then compacted to their distinct values.
static __global__ __launch_bounds__(LONG_BLOCK) void long_rows_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                              uint32_t b, int32_t n_vert, int32_t* __restrict__ deg,
                                                              int64_t* __restrict__ src, int32_t* temp,
                                                              const int64_t* __restrict__ long_list,
                                                              int64_t long_cap, const uint32_t* long_count,
                                                              uint32_t* err) {
    __shared__ int32_t s[LONG_LDS];
    __shared__ uint32_t s_wcnt[LONG_BLOCK / WAVE];
    __shared__ int64_t s_len;
    const int tid = threadIdx.x;
    const uint64_t lo_mask = (1ull << b) - 1;
    const int64_t n_long = tmin<int64_t>(*long_count, long_cap);
    for (int64_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const int64_t rs = long_list[li];
        const uint64_t hi = keys[rs] >> b;
        if (tid == 0) {  // end of the row: first later key of another row (binary search)
            int64_t lo = rs + 1, up = n;
            while (lo < up) {
                const int64_t mid = lo + (up - lo) / 2;
                const uint64_t km = keys[mid];
                if (km != KEY_NONE && (km >> b) == hi) lo = mid + 1;
                else up = mid;
            }
            s_len = lo - rs;
        }
        __syncthreads();
        const int64_t len = s_len;
        int64_t n2 = 1;
        while (n2 < len) n2 <<= 1;
        int32_t* x = temp + rs;
        if (len <= LONG_LDS) {
            for (int64_t i = tid; i < n2; i += LONG_BLOCK) s[i] = i < len ? (int32_t)(keys[rs + i] & lo_mask) : INT_MAX;
            __syncthreads();
            for (int64_t k = 2; k <= n2; k <<= 1)
                for (int64_t j = k >> 1; j > 0; j >>= 1) {
                    for (int64_t i = tid; i < n2; i += LONG_BLOCK) {
                        const int64_t p = i ^ j;
                        if (p > i) {
                            const int32_t a = s[i], c = s[p];
                            if ((a > c) == ((i & k) == 0)) {
                                s[i] = c;
                                s[p] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            for (int64_t i = tid; i < len; i += LONG_BLOCK) x[i] = s[i];
        } else {
            for (int64_t i = tid; i < len; i += LONG_BLOCK) x[i] = (int32_t)(keys[rs + i] & lo_mask);
            __threadfence_block();
            __syncthreads();
            for (int64_t k = 2; k <= n2; k <<= 1)
                for (int64_t j = k >> 1; j > 0; j >>= 1) {
                    for (int64_t i = tid; i < len; i += LONG_BLOCK) {
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
        __threadfence_block();
        __syncthreads();
        // compact the sorted values to their distinct ones, chunk by chunk in order
        int64_t out = 0;
        for (int64_t c0 = 0; c0 < len; c0 += LONG_BLOCK) {
            const int64_t i = c0 + tid;
            const int32_t v = i < len ? x[i] : 0;
            const bool keep = i < len && (i == 0 || x[i - 1] != v);
            __syncthreads();  // every read of this chunk precedes any write to it
            uint32_t total;
            const uint32_t at = block_exclusive_sum<LONG_BLOCK>((uint32_t)keep, s_wcnt, &total);
            if (keep) x[out + at] = v;
            out += total;
            __threadfence_block();
            __syncthreads();
        }
        if (tid == 0) {
            if ((int64_t)hi < n_vert) {
                deg[hi] = (int32_t)out;
                src[hi] = rs;
            } else {
                set_error(err, ERR_INTERNAL);
            }
        }
        __syncthreads();
    }
}

// cols[row_ptr[v] + i] = temp[src[v] + i] for i < deg[v]: one thread per row.
static __global__ __launch_bounds__(GATHER_BLOCK) void row_gather_kernel(const int32_t* __restrict__ row_ptr,
                                                                 const int32_t* __restrict__ deg,
                                                                 const int64_t* __restrict__ src,
                                                                 const int32_t* __restrict__ temp, int32_t n_vert,
                                                                 int32_t* __restrict__ cols, int64_t cols_cap,
                                                                 uint32_t* err) {
    const int64_t v = (int64_t)blockIdx.x * GATHER_BLOCK + threadIdx.x;
    if (v >= n_vert) return;
    const int d = deg[v];
    if (d <= 0) return;
    const int64_t from = src[v];
    const int64_t to = row_ptr[v];
    if (to + d > cols_cap) {
        set_error(err, ERR_CAPACITY);
        return;
    }
    for (int i = 0; i < d; ++i) cols[to + i] = temp[from + i];
}

}  // namespace mnb
