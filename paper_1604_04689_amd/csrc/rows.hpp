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
constexpr int ROW_TILE = 2048;   // keys whose rows a block owns
constexpr int ROW_HALO = 512;    // keys read past the tile to finish its last row
constexpr int ROW_SHORT = 256;   // longest row handled in LDS; longer rows are listed
constexpr int LONG_BLOCK = 256;
constexpr int LONG_LDS = 16384;  // longest row sorted in LDS by one block
constexpr int LONG_GRID = 256;
constexpr int GATHER_BLOCK = 256;
constexpr uint32_t SLOT_EMPTY = 0xffffffffu;

static_assert(ROW_HALO >= ROW_SHORT, "a short row owned by a tile ends inside its halo");

// A block owns the rows whose first key lies in its tile (keys read past the
// tile finish its last row).  Per position: its row's first position by a
// max-scan of row starts, the row length from the row's last position.  Each
// key of a short row inserts its low part into an open-addressing table in
// LDS that spans the row's own positions (size L, linear probing); the
// insertion that fills an empty slot is the value's one kept copy.  A kept
// value's place in the row is the number of distinct values below it, counted
// over the row's table.  Rows longer than ROW_SHORT (or running past the halo)
// are listed, by first key index, for long_rows.
static __global__ __launch_bounds__(ROW_BLOCK) void row_unique_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                                     uint32_t b, int32_t n_vert,
                                                                     int32_t* __restrict__ deg,
                                                                     int64_t* __restrict__ src,
                                                                     int32_t* __restrict__ temp,
                                                                     int64_t* __restrict__ long_list,
                                                                     int64_t long_cap, uint32_t* long_count,
                                                                     uint32_t* err) {
    constexpr int SPAN = ROW_TILE + ROW_HALO;
    constexpr int PER = SPAN / ROW_BLOCK;
    constexpr int WAVES = ROW_BLOCK / WAVE;
    static_assert(SPAN % ROW_BLOCK == 0, "whole positions per thread");
    __shared__ uint64_t s_k[SPAN + 1];   // s_k[0] = key before the tile, s_k[1 + p] = key base + p
    __shared__ int16_t s_rs[SPAN];       // first position of p's row (-1: row starts before the tile)
    __shared__ int16_t s_len[SPAN];      // at a row's first position: its length (0 if it leaves the span)
    __shared__ uint32_t s_tab[SPAN];     // per-row open-addressing tables over the row's positions
    __shared__ int32_t s_tmp[WAVES];
    __shared__ int32_t s_bounds[2];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t base = (int64_t)blockIdx.x * ROW_TILE;
    const int span = (int)tmin<int64_t>(SPAN, n - base);
    const uint64_t lo_mask = (1ull << b) - 1;
    {
        uint64_t k[PER];  // striped, coalesced; all loads in flight before the stores
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int p = q * ROW_BLOCK + tid;
            k[q] = p < span ? keys[base + p] : KEY_NONE;
        }
        const uint64_t before = (tid == 0 && base > 0) ? keys[base - 1] : KEY_NONE;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int p = q * ROW_BLOCK + tid;
            s_k[1 + p] = k[q];
            s_tab[p] = SLOT_EMPTY;
            s_len[p] = 0;
        }
        if (tid == 0) {
            s_k[0] = before;
            s_bounds[0] = ROW_TILE;
            s_bounds[1] = SPAN;
        }
    }
    __syncthreads();
    // ---- row starts and the first position of every row (blocked: PER
    // consecutive positions per thread, then a max-scan over the threads)
    bool st[PER];
    int last = -1;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = tid * PER + q;
        const uint64_t cur = s_k[1 + p], prev = s_k[p];
        const bool s_ = p >= span || cur == KEY_NONE || base + p == 0 || prev == KEY_NONE || (cur >> b) != (prev >> b);
        st[q] = s_;
        if (s_) last = p;
    }
    {
        int incl = last;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int y = __shfl_up(incl, d, WAVE);
            if (lane >= d) incl = y > incl ? y : incl;
        }
        if (lane == WAVE - 1) s_tmp[wid] = incl;
        __syncthreads();
        int before_w = -1;
#pragma unroll
        for (int w = 0; w < WAVES; ++w)
            if (w < wid) before_w = s_tmp[w] > before_w ? s_tmp[w] : before_w;
        int prev = __shfl_up(incl, 1, WAVE);
        if (lane == 0) prev = -1;
        int cur_rs = prev > before_w ? prev : before_w;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int p = tid * PER + q;
            if (st[q]) cur_rs = p;
            s_rs[p] = (int16_t)cur_rs;
            if (st[q] && p < ROW_TILE) atomicMin(&s_bounds[0], p);
            if (st[q] && p >= ROW_TILE) atomicMin(&s_bounds[1], p);
        }
    }
    __syncthreads();
    const int p0 = s_bounds[0], pe = s_bounds[1];
    if (p0 >= ROW_TILE) return;  // the tile lies inside a row owned by an earlier tile
    // ---- row lengths, written at each row's first position by its last position
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = tid * PER + q;
        if (p < p0 || p >= pe || s_k[1 + p] == KEY_NONE) continue;
        bool next_start;
        if (q + 1 < PER) next_start = st[q + 1];
        else if (p + 1 >= SPAN) next_start = false;  // the row may go on past the span
        else next_start = s_rs[p + 1] == p + 1;
        if (next_start) s_len[s_rs[p]] = (int16_t)(p + 1 - s_rs[p]);
    }
    __syncthreads();
    // ---- insert every key of a short row into its row's table (striped:
    // consecutive positions on consecutive threads); a first probe for all,
    // then further probes for the few that collided
    bool bad = false;
    uint32_t kept = 0, pending = 0;
    uint32_t hslot[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        hslot[q] = 0;
        if (p < p0 || p >= pe) continue;
        const uint64_t cur = s_k[1 + p];
        if (cur == KEY_NONE) continue;
        const int rs = s_rs[p];
        const int len = s_len[rs];
        if (len == 0 || len > ROW_SHORT) {  // long, or running past the span
            if (p == rs) {
                const uint32_t slot = atomicAdd(long_count, 1u);
                if ((int64_t)slot < long_cap) long_list[slot] = base + rs;
                else bad = true;
            }
            continue;
        }
        const uint32_t lo = (uint32_t)(cur & lo_mask);
        const uint32_t h = (uint32_t)(((uint64_t)(lo * 2654435761u) * (uint32_t)len) >> 32);
        const uint32_t old = atomicCAS(&s_tab[rs + h], SLOT_EMPTY, lo);
        if (old == SLOT_EMPTY) kept |= 1u << q;
        else if (old != lo) {
            pending |= 1u << q;
            hslot[q] = h;
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (!((pending >> q) & 1u)) continue;
        const int p = q * ROW_BLOCK + tid;
        const int rs = s_rs[p];
        const uint32_t len = (uint32_t)s_len[rs];
        const uint32_t lo = (uint32_t)(s_k[1 + p] & lo_mask);
        uint32_t h = hslot[q];
        for (uint32_t probe = 1; probe < len; ++probe) {
            h = h + 1 == len ? 0 : h + 1;
            const uint32_t old = atomicCAS(&s_tab[rs + h], SLOT_EMPTY, lo);
            if (old == SLOT_EMPTY) {
                kept |= 1u << q;
                break;
            }
            if (old == lo) break;
        }
    }
    __syncthreads();
    // ---- place every kept value: the number of distinct values below it
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        if (p < p0 || p >= pe) continue;
        const uint64_t cur = s_k[1 + p];
        if (cur == KEY_NONE) continue;
        const int rs = s_rs[p];
        const int len = s_len[rs];
        if (len == 0 || len > ROW_SHORT) continue;
        if ((kept >> q) & 1u) {
            const uint32_t lo = (uint32_t)(cur & lo_mask);
            int below = 0;
            for (int j = 0; j < len; ++j) {
                const uint32_t t = s_tab[rs + j];
                below += (t < lo) ? 1 : 0;  // SLOT_EMPTY is above every value
            }
            temp[base + rs + below] = (int32_t)lo;
        }
        if (p == rs) {
            int cnt = 0;
            for (int j = 0; j < len; ++j) cnt += s_tab[rs + j] != SLOT_EMPTY ? 1 : 0;
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

// cols[row_ptr[v] + i] = temp[src[v] + i] for i < deg[v].  A block covers
// GATHER_BLOCK consecutive vertices; their output range is contiguous, so the
// block walks it with consecutive threads on consecutive outputs (coalesced
// writes), finding each output's row by binary search over the block's row
// starts in LDS.
static __global__ __launch_bounds__(GATHER_BLOCK) void row_gather_kernel(const int32_t* __restrict__ row_ptr,
                                                                        const int32_t* __restrict__ deg,
                                                                        const int64_t* __restrict__ src,
                                                                        const int32_t* __restrict__ temp,
                                                                        int32_t n_vert, int32_t* __restrict__ cols,
                                                                        int64_t cols_cap, uint32_t* err) {
    __shared__ int32_t s_start[GATHER_BLOCK + 1];
    __shared__ int64_t s_src[GATHER_BLOCK];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * GATHER_BLOCK;
    const int nv = (int)tmin<int64_t>(GATHER_BLOCK, (int64_t)n_vert - v0);
    if (tid < nv) {
        s_start[tid] = row_ptr[v0 + tid];
        s_src[tid] = deg[v0 + tid] > 0 ? src[v0 + tid] : 0;
    }
    if (tid == 0) s_start[nv] = row_ptr[v0 + nv];
    __syncthreads();
    const int64_t a = s_start[0], e = s_start[nv];
    if (e > cols_cap) {
        if (tid == 0) set_error(err, ERR_CAPACITY);
        return;
    }
    for (int64_t i = a + tid; i < e; i += GATHER_BLOCK) {
        int lo = 0, hi = nv - 1;  // last row whose start <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        cols[i] = temp[s_src[lo] + (i - s_start[lo])];
    }
}

}  // namespace mnb
