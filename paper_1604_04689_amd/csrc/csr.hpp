// Sorted keys -> CSR: the segmented reduction and scan of the paper
// (Sec. 2.2.1: counts per vertex by segmented reduction, first indices by
// segmented scan), done in one pass over the keys sorted ascending.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int UNIQ_BLOCK = 256;
constexpr int UNIQ_ITEMS = 16;
constexpr int UNIQ_TILE = UNIQ_BLOCK * UNIQ_ITEMS;

// ---------------------------------------------------------------------------
// unique_csr over keys (hi << b) | lo sorted ascending, KEY_NONE last.  A key
// is kept when it is not KEY_NONE and differs from its predecessor; kept keys
// are compacted into cols (cols[i] = lo).  Where the high part (the vertex)
// changes between neighbors in sorted order, the row starts of the vertices
// in between are written, so empty rows get their offsets; the last real key
// writes the tail up to row_ptr[n_vert] = nnz; with no real key at all the
// first tile writes row_ptr = 0.  The key count is n, or *n_dev when given.
// Wave w of a tile owns positions [w*64*ITEMS, (w+1)*64*ITEMS); compaction
// offsets come from ballots, a scan over the waves and a look-back across
// tiles (one wave walks 64 earlier tiles per step).
// ---------------------------------------------------------------------------
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void unique_csr_kernel(const uint64_t* __restrict__ keys, int64_t n_host,
                                                          const uint32_t* __restrict__ n_dev, uint32_t b,
                                                          int32_t n_vert, int32_t* __restrict__ cols,
                                                          int64_t cols_cap, int32_t* __restrict__ row_ptr,
                                                          uint64_t* lookback, uint32_t* ticket, uint32_t* err) {
    constexpr int WAVES = BLOCK / WAVE;
    constexpr int TILE = BLOCK * ITEMS;
    static_assert(ITEMS <= 32, "keep flags in one word");
    __shared__ uint64_t s_keys[TILE + 2];  // [0] predecessor, [1..tile_n] tile, [tile_n+1] successor
    __shared__ uint32_t s_wtot[WAVES];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_prefix;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * TILE;
    const int wpos = wid * WAVE * ITEMS + lane;
    // keys are read up to the array length n_host, so the loads need not wait
    // for the device count; only positions below the count take part
    const int load_n = (int)tmin<int64_t>(TILE, n_host - base);
    const int64_t n = n_dev ? tmin<int64_t>(n_host, (int64_t)*n_dev) : n_host;
    const int tile_n = (int)tmin<int64_t>(TILE, n - base);  // may be <= 0 when n is a device count
    {
        uint64_t k[ITEMS];  // all loads in flight before the LDS stores
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int pos = wpos + j * WAVE;
            k[j] = pos < load_n ? keys[base + pos] : KEY_NONE;
        }
        if (tile_n <= 0) {
            // past the device key count: no later tile has keys either
            if (tile == 0)
                for (int64_t v = tid; v <= n_vert; v += BLOCK) row_ptr[v] = 0;
            return;
        }
        uint64_t halo = KEY_NONE;
        if (tid == 0 && base > 0) halo = keys[base - 1];
        if (tid == 1 && base + tile_n < n) halo = keys[base + tile_n];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int pos = wpos + j * WAVE;
            if (pos < tile_n) s_keys[1 + pos] = k[j];
        }
        if (tid == 0) s_keys[0] = halo;
        if (tid == 1) s_keys[tile_n + 1] = halo;
    }
    __syncthreads();

    uint32_t keep_bits = 0, wsum = 0;
    uint32_t jcnt[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int pos = wpos + j * WAVE;
        bool keep = false;
        if (pos < tile_n) {
            const uint64_t cur = s_keys[1 + pos];
            keep = cur != KEY_NONE && (base + pos == 0 || cur != s_keys[pos]);
        }
        keep_bits |= (uint32_t)keep << j;
        jcnt[j] = wsum;  // kept keys of this wave before item j
        wsum += (uint32_t)__popcll(__ballot(keep));
    }
    if (lane == 0) s_wtot[wid] = wsum;
    __syncthreads();
    uint32_t woff = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t t = s_wtot[w];
        woff += w < wid ? t : 0u;
        total += t;
    }
    if (wid == 0) {
        if (lane == 0) lb_store(lookback + tile, (tile == 0 ? LB_INC : LB_AGG) | total);
        const uint64_t before = wave_lookback_prefix(lookback, tile, total, err);
        if (lane == 0) s_prefix = before;
    }
    __syncthreads();
    const int64_t prefix = (int64_t)s_prefix + woff;
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint64_t lo_mask = b >= 64 ? ~0ull : (1ull << b) - 1;
    bool cap_hit = false, bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int pos = wpos + j * WAVE;
        const bool keep = (keep_bits >> j) & 1u;
        const int64_t idx = prefix + jcnt[j] + __popcll(__ballot(keep) & lt_mask);
        if (pos >= tile_n) continue;
        const uint64_t cur = s_keys[1 + pos];
        const int64_t gi = base + pos;
        if (keep) {
            if (idx < cols_cap) cols[idx] = (int32_t)(cur & lo_mask);
            else cap_hit = true;
        }
        if (cur != KEY_NONE) {
            const int64_t hi = (int64_t)(cur >> b);
            if (hi >= n_vert) {  // only after a failed look-back left stale keys
                bad = true;
                continue;
            }
            const int64_t prev_hi = gi == 0 ? -1 : tmin<int64_t>((int64_t)(s_keys[pos] >> b), n_vert);
            for (int64_t v = prev_hi + 1; v <= hi; ++v) row_ptr[v] = (int32_t)idx;
            const uint64_t next = s_keys[pos + 2];
            if (gi == n - 1 || next == KEY_NONE) {
                const int32_t nnz = (int32_t)(idx + (keep ? 1 : 0));
                for (int64_t v = hi + 1; v <= n_vert; ++v) row_ptr[v] = nnz;
            }
        } else if (gi == 0) {
            for (int64_t v = 0; v <= n_vert; ++v) row_ptr[v] = 0;  // no real key at all
        }
    }
    if (cap_hit) set_error(err, ERR_CAPACITY);
    if (bad) set_error(err, ERR_INTERNAL);
}

// Tiles: ceil(n_host / UNIQ_TILE); the look-back array needs that many words.
inline hipError_t launch_unique_csr(const char* name, const uint64_t* keys, int64_t n_host, const uint32_t* n_dev, uint32_t b,
                                    int32_t n_vert, int32_t* cols, int64_t cols_cap, int32_t* row_ptr,
                                    uint64_t* lookback, uint32_t* ticket, uint32_t* err, hipStream_t s) {
    return launch(name, unique_csr_kernel<UNIQ_BLOCK, UNIQ_ITEMS>, dim3((unsigned)ceil_div(n_host, UNIQ_TILE)),
                  dim3(UNIQ_BLOCK), s, keys, n_host, n_dev, b, n_vert, cols, cols_cap, row_ptr, lookback, ticket, err);
}

// Exclusive scan of n int32 counts: out[i] = B + sum of in[0..i), out[n] =
// B + total, where B = *base read on the device (0 for a null base).  base
// may point at out[0]: the value written there is the one read.  Tiles by
// ticket, one wave-wide look-back per tile.
constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

static __global__ __launch_bounds__(SCAN_BLOCK) void scan_i32_kernel(const int32_t* __restrict__ in, int64_t n,
                                                             int32_t* out, uint64_t* lookback,
                                                             uint32_t* ticket, uint32_t* err,
                                                             const int32_t* base) {
    constexpr int WAVES = SCAN_BLOCK / WAVE;
    constexpr int PARTS = SCAN_ITEMS * WAVES;  // one sum per (item, wave), in element order
    static_assert(PARTS % WAVE == 0, "the partial sums fill whole waves");
    __shared__ uint32_t s_sum[PARTS];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t first = (int64_t)tile * SCAN_TILE;
    uint32_t c[SCAN_ITEMS], ex[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t i = first + j * SCAN_BLOCK + wid * WAVE + lane;
        c[j] = i < n ? (uint32_t)in[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const uint32_t incl = wave_inclusive_sum(c[j]);
        ex[j] = incl - c[j];
        if (lane == WAVE - 1) s_sum[j * WAVES + wid] = incl;
    }
    __syncthreads();
    if (wid == 0) {
        // exclusive scan of the partial sums, 64 at a time with a carry (a
        // large tile keeps the look-back walks short: they are latency-bound)
        uint32_t total = 0;
#pragma unroll
        for (int c = 0; c < PARTS / WAVE; ++c) {
            const uint32_t v = s_sum[c * WAVE + lane];
            const uint32_t incl = wave_inclusive_sum(v);
            s_sum[c * WAVE + lane] = total + incl - v;
            total += __shfl(incl, WAVE - 1, WAVE);
        }
        if (lane == 0) lb_store(lookback + tile, (tile == 0 ? LB_INC : LB_AGG) | (uint64_t)total);
        const uint64_t before = wave_lookback_prefix(lookback, tile, total, err);
        if (lane == 0) s_prefix = before;
    }
    __syncthreads();
    const uint64_t prefix = s_prefix + (base ? (uint64_t)(uint32_t)*base : 0u);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t i = first + j * SCAN_BLOCK + wid * WAVE + lane;
        if (i < n) {
            const uint64_t start = prefix + s_sum[j * WAVES + wid] + ex[j];
            out[i] = (int32_t)start;
            if (i == n - 1) out[n] = (int32_t)(start + c[j]);
        }
    }
}

}  // namespace mnb

namespace mnb {

// Row starts after a CsrOut pass: row_ptr[v] holds the first slot of vertex
// v's row, or INT32_MAX for a vertex without keys.  Such a vertex's row is
// empty and starts where the next non-empty row starts, so row_ptr becomes
// its suffix minimum, with row_ptr[n] = *count.  Two launches: block minima,
// then the fill (a block takes the minimum of the later blocks' minima, then
// the suffix minimum of its own entries).
constexpr int RF_BLOCK = 256;
constexpr int RF_ITEMS = 16;
constexpr int RF_TILE = RF_BLOCK * RF_ITEMS;

static __global__ __launch_bounds__(RF_BLOCK) void rowptr_blockmin_kernel(int32_t* __restrict__ row_ptr, int64_t n,
                                                                         const uint32_t* __restrict__ count,
                                                                         int32_t* __restrict__ block_min) {
    __shared__ int32_t s_min[RF_BLOCK / WAVE];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const int64_t base = (int64_t)blockIdx.x * RF_TILE;
    int32_t m = INT32_MAX;
#pragma unroll
    for (int j = 0; j < RF_ITEMS; ++j) {
        const int64_t i = base + j * RF_BLOCK + tid;
        if (i < n) m = min(m, row_ptr[i]);
        else if (i == n) {
            const int32_t c = (int32_t)*count;
            row_ptr[n] = c;  // only this block reads entry n
            m = min(m, c);
        }
    }
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) m = min(m, __shfl_xor(m, d, WAVE));
    if (lane == 0) s_min[wid] = m;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < RF_BLOCK / WAVE; ++w) m = min(m, s_min[w]);
        block_min[blockIdx.x] = m;
    }
}

static __global__ __launch_bounds__(RF_BLOCK) void rowptr_fill_kernel(int32_t* __restrict__ row_ptr, int64_t n,
                                                                      const int32_t* __restrict__ block_min,
                                                                      int64_t n_blocks) {
    __shared__ int32_t s_red[RF_BLOCK / WAVE];
    __shared__ int32_t s_after[RF_BLOCK / WAVE];  // minimum over each wave's entries
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    // minimum over the later blocks (entry n lives in the last block)
    int32_t later = INT32_MAX;
    for (int64_t b = (int64_t)blockIdx.x + 1 + tid; b < n_blocks; b += RF_BLOCK) later = min(later, block_min[b]);
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) later = min(later, __shfl_xor(later, d, WAVE));
    if (lane == 0) s_red[wid] = later;
    // this thread's entries, RF_ITEMS consecutive ones
    const int64_t first = (int64_t)blockIdx.x * RF_TILE + (int64_t)tid * RF_ITEMS;
    int32_t v[RF_ITEMS];
    int32_t mine = INT32_MAX;
#pragma unroll
    for (int j = 0; j < RF_ITEMS; ++j) {
        const int64_t i = first + j;
        v[j] = i <= n ? row_ptr[i] : INT32_MAX;
        mine = min(mine, v[j]);
    }
    // suffix minimum over the later lanes of the wave, then the later waves
    int32_t suf = mine;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int32_t y = __shfl_down(suf, d, WAVE);
        if (lane + d < WAVE) suf = min(suf, y);
    }
    int32_t after = __shfl_down(suf, 1, WAVE);  // exclusive
    if (lane == WAVE - 1) after = INT32_MAX;
    if (lane == 0) s_after[wid] = suf;  // the whole wave's minimum
    __syncthreads();
    for (int w = 0; w < RF_BLOCK / WAVE; ++w) later = min(later, s_red[w]);
    int32_t carry = min(later, after);
    for (int w = wid + 1; w < RF_BLOCK / WAVE; ++w) carry = min(carry, s_after[w]);
#pragma unroll
    for (int j = RF_ITEMS - 1; j >= 0; --j) {
        const int64_t i = first + j;
        const int32_t r = min(v[j], carry);
        if (i < n && r != v[j]) row_ptr[i] = r;
        carry = r;
    }
}

// Launches the two fix-up kernels; block_min needs ceil((n + 1) / RF_TILE) ints.
static inline hipError_t launch_rowptr_fill(const char* tag, int32_t* row_ptr, int64_t n, const uint32_t* count,
                                            int32_t* block_min, hipStream_t s) {
    const int64_t blocks = ceil_div(n + 1, (int64_t)RF_TILE);
    hipError_t e = launch(tag, rowptr_blockmin_kernel, dim3((unsigned)blocks), dim3(RF_BLOCK), s, row_ptr, n, count,
                          block_min);
    if (e == hipSuccess)
        e = launch(tag, rowptr_fill_kernel, dim3((unsigned)blocks), dim3(RF_BLOCK), s, row_ptr, n,
                   (const int32_t*)block_min, blocks);
    return e;
}

}  // namespace mnb
