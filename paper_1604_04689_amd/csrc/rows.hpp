// Per-row canonicalisation of pair keys that are sorted by their high part
// only: keys (hi << b) | lo arrive grouped by hi (one group = one row, i.e.
// one vertex), with the lo values of a row in any order and possibly
// repeated.  For every row the distinct lo values are written ascending to
// temp[start .. start + count), with deg[hi] = count and src[hi] = start.  A
// tile's rows are packed one after another from the index of its first owned
// key (so its writes cover whole lines), within the tile's own key range;
// in a tile that owns a long row every row (long ones included) starts at the
// index of its own first key instead.  A scan of deg then gives row_ptr and
// a gather moves each row to cols.  This is the paper's sort by the first
// array (Sec. 2.2.1) followed by the duplicate-free, ascending rows of our
// reading of the serial solution (Sec. 3.2.2).
#pragma once

#include <climits>

#include "common.hpp"
#include "csr.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int ROW_BLOCK = 256;
constexpr int ROW_TILE = 2048;   // keys whose rows a block owns
constexpr int ROW_HALO = 256;    // keys read past the tile to finish its last row
constexpr int ROW_SHORT = 256;   // longest row handled in LDS; longer rows are listed
constexpr int LONG_BLOCK = 256;
constexpr int LONG_LDS = 16384;  // longest row sorted in LDS by one block
constexpr int LONG_GRID = 256;
constexpr int GATHER_BLOCK = 256;
constexpr uint32_t SLOT_EMPTY = 0xffffffffu;

static_assert(ROW_HALO >= ROW_SHORT, "a short row owned by a tile ends inside its halo");

// A block owns the rows whose first key lies in its tile (keys read past the
// tile finish its last row).  Positions are striped over the block: chunk
// c = q * WAVES + wave holds positions 64c .. 64c + 63, one per lane, so row
// starts, row ends and prefix counts come from wave ballots plus one short
// scan over the chunks.  Each key of a short row inserts its low part into an
// open-addressing table in LDS that spans the row's own positions (size L,
// linear probing); the insertion that fills an empty slot is the value's one
// kept copy.  Kept copies are compacted in position order into a dense list,
// where each row's distinct values are contiguous; a value's place in its row
// is the number of the row's distinct values below it.  Rows longer than
// ROW_SHORT (or running past the halo) are listed, by first key index, for
// long_rows.
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
    constexpr int CH = SPAN / WAVE;  // chunks of 64 positions
    static_assert(SPAN % ROW_BLOCK == 0 && ROW_TILE % WAVE == 0, "whole chunks per thread and per tile");
    static_assert(CH <= WAVE, "one wave scans the chunk summaries");
    __shared__ int16_t s_rs[SPAN];        // first position of p's row (-1: row starts before the tile)
    __shared__ int16_t s_len[SPAN];       // at a row's first position: its length (0 if it leaves the span)
    // per-row open-addressing tables over the row's positions; once every
    // insertion is done, the same words hold the kept values, dense, in
    // position order
    __shared__ uint32_t s_tab[SPAN];
    uint32_t* const s_dval = s_tab;
    __shared__ int16_t s_e[SPAN + 1];     // kept copies before position p
    __shared__ uint64_t s_lastkey[CH];    // key at the last position of each chunk
    __shared__ uint64_t s_startmask[CH];  // row-start flags of each chunk
    __shared__ int32_t s_csum[CH + 1];    // per chunk: last row start, then kept count; scanned
    __shared__ int32_t s_bounds[2];
    __shared__ int32_t s_haslong;
    __shared__ uint64_t s_before;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t base = (int64_t)blockIdx.x * ROW_TILE;
    const int span = (int)tmin<int64_t>(SPAN, n - base);
    const uint64_t lo_mask = (1ull << b) - 1;
    const uint64_t lt_mask = (1ull << lane) - 1;
    uint64_t k[PER];  // striped, coalesced; all loads in flight before the stores
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        k[q] = p < span ? keys[base + p] : KEY_NONE;
    }
    if (tid == 0) {
        s_before = base > 0 ? keys[base - 1] : KEY_NONE;
        s_bounds[0] = ROW_TILE;
        s_bounds[1] = SPAN;
        s_haslong = 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        if (lane == WAVE - 1) s_lastkey[q * WAVES + wid] = k[q];
        s_tab[p] = SLOT_EMPTY;
        s_len[p] = 0;
    }
    __syncthreads();
    // ---- row starts: ballots per chunk, the tile's first owned start and the halo's first start
    uint64_t smask[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid, c = q * WAVES + wid;
        uint64_t prev = __shfl_up(k[q], 1, WAVE);
        if (lane == 0) prev = c == 0 ? s_before : s_lastkey[c - 1];
        const uint64_t cur = k[q];
        const bool st = p >= span || cur == KEY_NONE || prev == KEY_NONE || (cur >> b) != (prev >> b);
        smask[q] = __ballot(st);
        if (lane == 0) {
            s_startmask[c] = smask[q];
            s_csum[c] = smask[q] ? c * WAVE + 63 - __clzll((long long)smask[q]) : -1;
            if (smask[q]) atomicMin(&s_bounds[c * WAVE < ROW_TILE ? 0 : 1], c * WAVE + __ffsll((unsigned long long)smask[q]) - 1);
        }
    }
    __syncthreads();
    if (wid == 0) {  // exclusive max-scan of the chunks' last starts
        int v = lane < CH ? s_csum[lane] : -1;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int y = __shfl_up(v, d, WAVE);
            if (lane >= d) v = y > v ? y : v;
        }
        int ex = __shfl_up(v, 1, WAVE);
        if (lane == 0) ex = -1;
        if (lane < CH) s_csum[lane] = ex;
    }
    __syncthreads();
    const int p0 = s_bounds[0], pe = s_bounds[1];
    if (p0 >= ROW_TILE) return;  // the tile lies inside a row owned by an earlier tile
    // ---- every position's row start; row lengths written at each row's
    // first position by its last position
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid, c = q * WAVES + wid;
        const uint64_t upto = smask[q] & (lt_mask | (1ull << lane));
        const int rs = upto ? c * WAVE + 63 - __clzll((long long)upto) : s_csum[c];
        s_rs[p] = (int16_t)rs;
        if (p < p0 || p >= pe || k[q] == KEY_NONE) continue;
        bool next_start;
        if (lane < WAVE - 1) next_start = (smask[q] >> (lane + 1)) & 1ull;
        else next_start = c + 1 < CH ? (s_startmask[c + 1] & 1ull) : false;  // past the span: unknown
        if (next_start) s_len[rs] = (int16_t)(p + 1 - rs);
    }
    __syncthreads();
    // ---- insert every key of a short row into its row's table; a first
    // probe for all, then further probes for the few that collided
    bool bad = false;
    uint32_t kept = 0, pending = 0;
    uint32_t hslot[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        hslot[q] = 0;
        if (p < p0 || p >= pe || k[q] == KEY_NONE) continue;
        const int rs = s_rs[p];
        const int len = s_len[rs];
        if (len == 0 || len > ROW_SHORT) {  // long, or running past the span
            if (p == rs) {
                const uint32_t slot = atomicAdd(long_count, 1u);
                if ((int64_t)slot < long_cap) long_list[slot] = base + rs;
                else bad = true;
                s_haslong = 1;
            }
            continue;
        }
        const uint32_t lo = (uint32_t)(k[q] & lo_mask);
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
        const uint32_t lo = (uint32_t)(k[q] & lo_mask);
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
    // ---- dense list of the kept values in position order
    uint64_t kmask[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        kmask[q] = __ballot((kept >> q) & 1u);
        if (lane == 0) s_csum[q * WAVES + wid] = __popcll(kmask[q]);
    }
    __syncthreads();
    if (wid == 0) {  // exclusive sum-scan of the chunks' kept counts
        const int x = lane < CH ? s_csum[lane] : 0;
        int v = x;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int y = __shfl_up(v, d, WAVE);
            if (lane >= d) v += y;
        }
        if (lane < CH) s_csum[lane] = v - x;
        if (lane == CH - 1) s_csum[CH] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid, c = q * WAVES + wid;
        const int e = s_csum[c] + __popcll(kmask[q] & lt_mask);
        s_e[p] = (int16_t)e;
        if ((kept >> q) & 1u) s_dval[e] = (uint32_t)(k[q] & lo_mask);
    }
    if (tid == 0) s_e[SPAN] = (int16_t)s_csum[CH];
    __syncthreads();
    // ---- place every kept value; the row's first position records the row.
    // Rows are packed from the tile's first owned key on, unless the tile
    // owns a long row (whose output fills its own key range): then every row
    // writes into its own key range.
    const bool packed = s_haslong == 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int p = q * ROW_BLOCK + tid;
        if (p < p0 || p >= pe || k[q] == KEY_NONE) continue;
        const int rs = s_rs[p];
        const int len = s_len[rs];
        if (len == 0 || len > ROW_SHORT) continue;
        const int ds = s_e[rs], u = s_e[rs + len] - ds;
        if ((kept >> q) & 1u) {
            const uint32_t lo = (uint32_t)(k[q] & lo_mask);
            int below = 0;
            for (int j = 0; j < u; ++j) below += s_dval[ds + j] < lo ? 1 : 0;
            temp[base + (packed ? p0 + ds : rs) + below] = (int32_t)lo;
        }
        if (p == rs) {
            const int64_t hi = (int64_t)(k[q] >> b);
            if (hi < n_vert) {
                deg[hi] = u;
                src[hi] = base + (packed ? p0 + ds : rs);
            } else {
                bad = true;
            }
        }
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// Sorts x[0 .. len) ascending in place (bitonic: in LDS through s when
// len <= LONG_LDS, else in global memory with every comparator putting the
// smaller value at the lower index, so virtual INT_MAX padding never moves),
// then compacts it to its distinct values other than INT_MAX (the marker of
// an absent value).  Returns the distinct count (the same on every thread).
// Every thread of the block calls it; s_wcnt needs LONG_BLOCK / 64 words.
__device__ inline int64_t block_sort_unique(int32_t* x, int64_t len, int32_t* s, uint32_t* s_wcnt) {
    const int tid = threadIdx.x;
    int64_t n2 = 1;
    while (n2 < len) n2 <<= 1;
    if (len <= LONG_LDS) {
        for (int64_t i = tid; i < n2; i += LONG_BLOCK) s[i] = i < len ? x[i] : INT_MAX;
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
        const bool keep = i < len && v != INT_MAX && (i == 0 || x[i - 1] != v);
        __syncthreads();  // every read of this chunk precedes any write to it
        uint32_t total;
        const uint32_t at = block_exclusive_sum<LONG_BLOCK>((uint32_t)keep, s_wcnt, &total);
        if (keep) x[out + at] = v;
        out += total;
        __threadfence_block();
        __syncthreads();
    }
    return out;
}

// Rows longer than ROW_SHORT: one block per listed row.  The lo values are
// copied to the row's temp range, then sorted and compacted to their
// distinct values there (block_sort_unique).
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
        int32_t* x = temp + rs;
        for (int64_t i = tid; i < len; i += LONG_BLOCK) x[i] = (int32_t)(keys[rs + i] & lo_mask);
        __threadfence_block();
        __syncthreads();
        const int64_t out = block_sort_unique(x, len, s, s_wcnt);
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

// The vertex-rows stage after the radix passes over the high key bits:
// row dedup, long rows, scan of the distinct counts into row_ptr, gather into
// cols.  `deg` must be zero on entry and `*long_count` zero; `temp` needs n
// words; `scan_lb` room for ceil((n_vert + 1) / SCAN_TILE) zeroed look-back
// slots.  Kernel names carry `tag` ("node" or "batch_node").
struct RowsStage {
    const uint64_t* sorted;
    int64_t n;
    uint32_t b;  // low bits of a key (the neighbor id)
    int32_t n_vert;
    int32_t* deg;
    int64_t* src;
    int32_t* temp;
    int64_t* long_list;
    int64_t long_cap;
    uint32_t* long_count;
    uint64_t* scan_lb;
    uint32_t* scan_ticket;
    uint32_t* err;
};

// Row dedup, long rows, and the scan of the distinct counts into row_ptr
// (n_vert + 1 entries).
static inline hipError_t launch_rows_dedup(const RowsStage& r, int32_t* row_ptr, hipStream_t s, bool batch = false) {
    hipError_t e = launch(batch ? "batch_node_row_unique" : "node_row_unique", row_unique_kernel,
                          dim3((unsigned)ceil_div(r.n, ROW_TILE)), dim3(ROW_BLOCK), s, r.sorted, r.n, r.b, r.n_vert,
                          r.deg, r.src, r.temp, r.long_list, r.long_cap, r.long_count, r.err);
    if (e == hipSuccess)
        e = launch(batch ? "batch_node_long_rows" : "node_long_rows", long_rows_kernel, dim3(LONG_GRID),
                   dim3(LONG_BLOCK), s, r.sorted, r.n, r.b, r.n_vert, r.deg, r.src, r.temp,
                   (const int64_t*)r.long_list, r.long_cap, (const uint32_t*)r.long_count, r.err);
    if (e == hipSuccess)
        e = launch(batch ? "batch_node_row_scan" : "node_row_scan", scan_i32_kernel,
                   dim3((unsigned)ceil_div((int64_t)r.n_vert, SCAN_TILE)), dim3(SCAN_BLOCK), s, (const int32_t*)r.deg,
                   (int64_t)r.n_vert, row_ptr, r.scan_lb, r.scan_ticket, r.err, (const int32_t*)nullptr);
    return e;
}

static inline hipError_t launch_rows_stage(bool batch, const RowsStage& r, int32_t* row_ptr, int32_t* cols,
                                           int64_t cols_cap, hipStream_t s) {
    hipError_t e = launch_rows_dedup(r, row_ptr, s, batch);
    if (e == hipSuccess)
        e = launch(batch ? "batch_node_row_gather" : "node_row_gather", row_gather_kernel,
                   dim3((unsigned)ceil_div((int64_t)r.n_vert, GATHER_BLOCK)), dim3(GATHER_BLOCK), s,
                   (const int32_t*)row_ptr, (const int32_t*)r.deg, (const int64_t*)r.src, (const int32_t*)r.temp,
                   r.n_vert, cols, cols_cap, r.err);
    return e;
}

}  // namespace mnb
