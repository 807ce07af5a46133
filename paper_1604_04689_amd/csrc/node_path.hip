// One-ring neighboring nodes (paper Sec. 2.1.1 and 2.2.1).
//
// The paper forms two integer pairs per triangle edge (both directions), sorts
// the pairs by their first entry, and derives per vertex the count and first
// index of its neighbors by segmented reduction and scan.  Here each directed
// pair (u, w) is packed into one 64-bit key (u << b) | w, b = bits of a vertex
// id, and the whole key is sorted, so rows come out ascending and a repeated
// edge (shared by several elements) lands next to its copy; one pass then
// drops repeats, writes cols and the row starts.
//
//   node_emit      conn -> keys, plus the digit histograms of every radix pass
//   radix_pass x p keys -> keys (stable, one 8-bit digit per pass, onesweep:
//                  ranks within a tile, decoupled look-back across tiles)
//   unique_csr     keys -> cols, row_ptr
#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int RBITS = 8;
constexpr int RADIX = 1 << RBITS;
constexpr int MAX_PASS = 8;  // 2b <= 62 key bits

constexpr int EMIT_BLOCK = 256;   // elements per emit tile (one per thread)
constexpr int EMIT_GRID_MAX = 2048;
constexpr int SORT_BLOCK = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_BLOCK * SORT_ITEMS;
constexpr int UNIQ_BLOCK = 256;
constexpr int UNIQ_ITEMS = 16;
constexpr int UNIQ_TILE = UNIQ_BLOCK * UNIQ_ITEMS;

// ---------------------------------------------------------------------------
// node_emit: both directions of every element edge as packed keys.
// A self pair (repeated id in a degenerate element) or a pair touching an id
// outside [0, n_vert) becomes KEY_NONE; a bad id also raises ERR_INDEX_RANGE.
// Each block accumulates the digit histograms of all passes in LDS over the
// element tiles it visits and flushes them once with global atomics.
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(EMIT_BLOCK) void node_emit_kernel(const int32_t* __restrict__ conn, int64_t n_elem,
                                                              int32_t n_vert, uint32_t b, int n_pass,
                                                              uint32_t last_bits, uint64_t* __restrict__ keys,
                                                              uint32_t* __restrict__ hist, uint32_t* err) {
    using E = Elem<ET>;
    constexpr int NPE = E::NPE;
    constexpr int KPE = 2 * E::NE;
    __shared__ int32_t s_conn[EMIT_BLOCK * NPE];
    __shared__ uint64_t s_keys[EMIT_BLOCK * KPE];
    __shared__ uint32_t s_hist[MAX_PASS * RADIX];

    const int tid = threadIdx.x;
    for (int i = tid; i < n_pass * RADIX; i += EMIT_BLOCK) s_hist[i] = 0;
    bool bad_seen = false;

    for (int64_t tile = blockIdx.x; tile * EMIT_BLOCK < n_elem; tile += gridDim.x) {
        const int64_t e0 = tile * EMIT_BLOCK;
        const int ne = (int)tmin<int64_t>(EMIT_BLOCK, n_elem - e0);
        __syncthreads();  // previous tile's LDS fully consumed (and s_hist zeroed)
        const int32_t* src = conn + e0 * NPE;
        for (int i = tid; i < ne * NPE; i += EMIT_BLOCK) s_conn[i] = src[i];
        __syncthreads();
        if (tid < ne) {
            int32_t id[NPE];
            bool ok[NPE];
#pragma unroll
            for (int j = 0; j < NPE; ++j) {
                id[j] = s_conn[tid * NPE + j];
                ok[j] = (uint32_t)id[j] < (uint32_t)n_vert;
                bad_seen |= !ok[j];
            }
#pragma unroll
            for (int k = 0; k < E::NE; ++k) {
                const int32_t u = id[E::A[k]], w = id[E::B[k]];
                const bool edge = ok[E::A[k]] && ok[E::B[k]] && u != w;
                const uint64_t k0 = edge ? ((uint64_t)u << b) | (uint64_t)w : KEY_NONE;
                const uint64_t k1 = edge ? ((uint64_t)w << b) | (uint64_t)u : KEY_NONE;
                s_keys[tid * KPE + 2 * k] = k0;
                s_keys[tid * KPE + 2 * k + 1] = k1;
                for (int p = 0; p < n_pass; ++p) {
                    const uint32_t mask = (p == n_pass - 1) ? ((1u << last_bits) - 1) : (RADIX - 1);
                    atomicAdd(&s_hist[p * RADIX + ((uint32_t)(k0 >> (p * RBITS)) & mask)], 1u);
                    atomicAdd(&s_hist[p * RADIX + ((uint32_t)(k1 >> (p * RBITS)) & mask)], 1u);
                }
            }
        }
        __syncthreads();
        uint64_t* dst = keys + e0 * KPE;
        for (int i = tid; i < ne * KPE; i += EMIT_BLOCK) dst[i] = s_keys[i];
    }
    if (bad_seen) set_error(err, ERR_INDEX_RANGE);
    __syncthreads();
    for (int i = tid; i < n_pass * RADIX; i += EMIT_BLOCK) {
        const uint32_t v = s_hist[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

// ---------------------------------------------------------------------------
// radix_pass: stable scatter of keys by the digit (key >> shift) & mask.
//
// Tile t (taken by atomic ticket, so earlier tiles are always resident) holds
// SORT_TILE keys.  Wave w of the block owns a contiguous run of 64*ITEMS keys,
// item j of lane l at offset j*64 + l, so (j, lane) order is input order.
// Ranking: for each item, the lanes holding the same digit are found with one
// ballot per digit bit; the lowest such lane bumps the wave's private digit
// counter in LDS and the others take their rank from it.  Per digit, wave
// counts are scanned in wave order (stability), the tile count is published
// for look-back, and the tile's keys are staged in LDS in digit order before
// a coalesced write to their global slots.
// ---------------------------------------------------------------------------
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void radix_pass_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                          int64_t n, uint32_t shift, uint32_t bits,
                                                          const uint32_t* __restrict__ hist, uint64_t* lookback,
                                                          uint64_t* lookback_next, uint32_t* ticket, uint32_t* err) {
    static_assert(BLOCK >= RADIX, "one thread per digit");
    constexpr int WAVES = BLOCK / WAVE;
    constexpr int TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_whist[WAVES][RADIX];
    __shared__ uint32_t s_tile_off[RADIX];
    __shared__ int64_t s_glob[RADIX];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = tid; i < WAVES * RADIX; i += BLOCK) (&s_whist[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t tile_base = (int64_t)tile * TILE;
    const uint32_t dmask = (1u << bits) - 1;

    // ---- load (coalesced: lanes of a wave read 64 consecutive keys) --------
    const int64_t wbase = tile_base + (int64_t)wid * WAVE * ITEMS + lane;
    uint64_t key[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = wbase + j * WAVE;
        key[j] = idx < n ? in[idx] : KEY_NONE;
    }

    // ---- rank within the wave --------------------------------------------
    const uint64_t lt_mask = (1ull << lane) - 1;
    uint32_t rank[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = wbase + j * WAVE < n;
        const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < RBITS; ++bit) {
            const bool on = (dg >> bit) & 1u;
            const uint64_t vote = __ballot(on);
            peers &= on ? vote : ~vote;
        }
        const uint32_t below = __popcll(peers & lt_mask);
        const int leader = __ffsll((unsigned long long)peers) - 1;
        uint32_t base = 0;
        if (valid && below == 0) {
            base = s_whist[wid][dg];
            s_whist[wid][dg] = base + (uint32_t)__popcll(peers);
        }
        base = __shfl(base, leader & (WAVE - 1), WAVE);
        rank[j] = base + below;
    }
    __syncthreads();

    // ---- per digit: wave offsets, tile count, publish ----------------------
    uint32_t tile_cnt = 0;
    if (tid < RADIX) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_whist[w][tid];
            s_whist[w][tid] = run;
            run += c;
        }
        tile_cnt = run;
        lb_store(lookback + (int64_t)tile * RADIX + tid, (tile == 0 ? LB_INC : LB_AGG) | tile_cnt);
    }
    uint32_t tile_total;
    const uint32_t toff = block_exclusive_sum<BLOCK>(tile_cnt, s_tmp, &tile_total);
    uint32_t hist_total;
    const uint32_t gstart = block_exclusive_sum<BLOCK>(tid < RADIX ? hist[tid] : 0u, s_tmp, &hist_total);
    if (tid < RADIX) {
        s_tile_off[tid] = toff;
        const uint64_t before = lookback_prefix(lookback + tid, RADIX, tile, tile_cnt, err);
        s_glob[tid] = (int64_t)gstart + (int64_t)before - (int64_t)toff;
        lookback_next[(int64_t)tile * RADIX + tid] = 0;  // slot of the next pass
    }
    __syncthreads();

    // ---- stage in digit order, then write out -------------------------------
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (wbase + j * WAVE < n) {
            const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
            s_keys[s_tile_off[dg] + s_whist[wid][dg] + rank[j]] = key[j];
        }
    }
    __syncthreads();
    const int tile_n = (int)tmin<int64_t>(TILE, n - tile_base);
    bool bad = false;
    for (int i = tid; i < tile_n; i += BLOCK) {
        const uint64_t k = s_keys[i];
        const uint32_t dg = (uint32_t)(k >> shift) & dmask;
        const int64_t dst = s_glob[dg] + i;
        if ((uint64_t)dst < (uint64_t)n) out[dst] = k;
        else bad = true;
    }
    if (bad) set_error(err, ERR_INTERNAL);
}

// ---------------------------------------------------------------------------
// unique_csr: the segmented reduction and scan of Sec. 2.2.1 over the sorted
// keys.  A key is kept when it differs from its predecessor and is an edge;
// kept keys are compacted into cols (low b bits = neighbor id).  Where the
// high part (the vertex) changes between neighbors in sorted order, the row
// starts of the vertices in between are written, so empty rows get the right
// offsets; the last real key writes the tail up to row_ptr[n_vert] = nnz.
// Positions are ordered (item j, wave, lane) inside a tile; compaction
// offsets come from ballots, a scan over the ITEMS x WAVES counts, and a
// look-back across tiles.
// ---------------------------------------------------------------------------
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void unique_csr_kernel(const uint64_t* __restrict__ keys, int64_t n, uint32_t b,
                                                          int32_t n_vert, int32_t* __restrict__ cols,
                                                          int64_t cols_cap, int32_t* __restrict__ row_ptr,
                                                          uint64_t* lookback, uint32_t* ticket, uint32_t* err) {
    constexpr int WAVES = BLOCK / WAVE;
    constexpr int TILE = BLOCK * ITEMS;
    static_assert(ITEMS * WAVES <= WAVE, "one wave scans the item/wave counts");
    __shared__ uint64_t s_keys[TILE + 2];  // [0] predecessor, [1..n] tile, [n+1] successor
    __shared__ uint32_t s_cnt[ITEMS * WAVES];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_prefix;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * TILE;
    const int tile_n = (int)tmin<int64_t>(TILE, n - base);
    if (tid == 0) s_keys[0] = base > 0 ? keys[base - 1] : KEY_NONE;
    if (tid == 1) s_keys[tile_n + 1] = base + tile_n < n ? keys[base + tile_n] : KEY_NONE;
    for (int i = tid; i < tile_n; i += BLOCK) s_keys[1 + i] = keys[base + i];
    __syncthreads();

    uint32_t keep_bits = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int pos = j * BLOCK + wid * WAVE + lane;
        bool keep = false;
        if (pos < tile_n) {
            const uint64_t cur = s_keys[1 + pos];
            keep = cur != KEY_NONE && (base + pos == 0 || cur != s_keys[pos]);
        }
        const uint64_t m = __ballot(keep);
        if (lane == 0) s_cnt[j * WAVES + wid] = (uint32_t)__popcll(m);
        keep_bits |= (uint32_t)keep << j;
    }
    __syncthreads();
    if (wid == 0) {
        const uint32_t v = lane < ITEMS * WAVES ? s_cnt[lane] : 0u;
        const uint32_t incl = wave_inclusive_sum(v);
        if (lane < ITEMS * WAVES) s_cnt[lane] = incl - v;
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        if (lane == 0) {
            lb_store(lookback + tile, (tile == 0 ? LB_INC : LB_AGG) | total);
            s_prefix = lookback_prefix(lookback, 1, tile, total, err);
        }
    }
    __syncthreads();
    const int64_t prefix = (int64_t)s_prefix;
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint64_t wmask = (1ull << b) - 1;
    bool cap_hit = false;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int pos = j * BLOCK + wid * WAVE + lane;
        const bool keep = (keep_bits >> j) & 1u;
        const uint64_t m = __ballot(keep);
        const int64_t idx = prefix + s_cnt[j * WAVES + wid] + __popcll(m & lt_mask);
        if (pos >= tile_n) continue;
        const uint64_t cur = s_keys[1 + pos];
        const int64_t gi = base + pos;
        if (keep) {
            if (idx < cols_cap) cols[idx] = (int32_t)(cur & wmask);
            else cap_hit = true;
        }
        if (cur != KEY_NONE) {
            const int64_t hi = (int64_t)(cur >> b);
            if (hi >= n_vert) {  // only after a failed look-back left stale keys
                set_error(err, ERR_INTERNAL);
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
            for (int64_t v = 0; v <= n_vert; ++v) row_ptr[v] = 0;  // no edge at all
        }
    }
    if (cap_hit) set_error(err, ERR_CAPACITY);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static uint32_t id_bits_for(int32_t n_vert) {
    uint32_t b = 1;
    while (b < 31 && ((int64_t)1 << b) < (int64_t)n_vert) ++b;
    return b;
}

bool plan_node(int64_t n_elem, int32_t etype, int32_t n_vert, NodePlan* p) {
    const int ne = edges_per_elem(etype);
    if (ne == 0 || n_elem < 0 || n_vert < 0) return false;
    p->n_elem = n_elem;
    p->etype = etype;
    p->n_vert = n_vert;
    p->n_pairs = 2 * (int64_t)ne * n_elem;
    p->id_bits = id_bits_for(n_vert);
    p->n_pass = (int)ceil_div(2 * p->id_bits, RBITS);
    p->n_tiles = ceil_div(p->n_pairs, SORT_TILE);
    p->n_utiles = ceil_div(p->n_pairs, UNIQ_TILE);
    size_t off = HEADER_BYTES;
    p->off_hist = off;
    off += align_up(MAX_PASS * RADIX * sizeof(uint32_t));
    p->off_ulb = off;
    off += align_up((size_t)p->n_utiles * sizeof(uint64_t));
    p->off_lb0 = off;
    off += align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t));
    p->zero_bytes = off;  // header, histograms, unique look-back, pass-0 look-back
    p->off_lb1 = off;
    off += align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t));
    p->off_keys0 = off;
    off += align_up((size_t)p->n_pairs * sizeof(uint64_t));
    p->off_keys1 = off;
    off += align_up((size_t)p->n_pairs * sizeof(uint64_t));
    p->total = off;
    return true;
}

template <int ET>
static hipError_t launch_emit(const NodePlan& p, const int32_t* conn, uint64_t* keys, uint32_t* hist, uint32_t* err,
                              hipStream_t s) {
    const int64_t tiles = ceil_div(p.n_elem, EMIT_BLOCK);
    const int grid = (int)tmin<int64_t>(tiles, EMIT_GRID_MAX);
    const uint32_t last_bits = 2 * p.id_bits - (uint32_t)(p.n_pass - 1) * RBITS;
    return launch("node_emit", node_emit_kernel<ET>, dim3(grid), dim3(EMIT_BLOCK), s, conn, p.n_elem, p.n_vert,
                  p.id_bits, p.n_pass, last_bits, keys, hist, err);
}

hipError_t run_node(const NodePlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                    void* ws, hipStream_t s) {
    char* w = (char*)ws;
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    uint32_t* tickets = hdr + HDR_TICKET0;
    uint32_t* hist = (uint32_t*)(w + p.off_hist);
    uint64_t* ulb = (uint64_t*)(w + p.off_ulb);
    uint64_t* lb[2] = {(uint64_t*)(w + p.off_lb0), (uint64_t*)(w + p.off_lb1)};
    uint64_t* kb[2] = {(uint64_t*)(w + p.off_keys0), (uint64_t*)(w + p.off_keys1)};

    hipError_t e = zero_words(ws, p.zero_bytes, s);
    if (e != hipSuccess) return e;
    if (p.n_pairs == 0) return fill_i32(row_ptr, (int64_t)p.n_vert + 1, 0, s);

    switch (p.etype) {
        case TRI3: e = launch_emit<TRI3>(p, conn, kb[0], hist, err, s); break;
        case TET4: e = launch_emit<TET4>(p, conn, kb[0], hist, err, s); break;
        default: e = launch_emit<HEX8>(p, conn, kb[0], hist, err, s); break;
    }
    if (e != hipSuccess) return e;
    const uint32_t total_bits = 2 * p.id_bits;
    for (int pass = 0; pass < p.n_pass; ++pass) {
        const uint32_t shift = (uint32_t)pass * RBITS;
        const uint32_t bits = tmin<uint32_t>(RBITS, total_bits - shift);
        e = launch("radix_pass", radix_pass_kernel<SORT_BLOCK, SORT_ITEMS>, dim3((unsigned)p.n_tiles),
                   dim3(SORT_BLOCK), s, kb[pass & 1], kb[(pass + 1) & 1], p.n_pairs, shift, bits,
                   hist + pass * RADIX, lb[pass & 1], lb[(pass + 1) & 1], tickets + pass, err);
        if (e != hipSuccess) return e;
    }
    const uint64_t* sorted = kb[p.n_pass & 1];
    return launch("unique_csr", unique_csr_kernel<UNIQ_BLOCK, UNIQ_ITEMS>, dim3((unsigned)p.n_utiles),
                  dim3(UNIQ_BLOCK), s, sorted, p.n_pairs, p.id_bits, p.n_vert, cols, cols_capacity, row_ptr, ulb,
                  tickets + (N_TICKETS - 1), err);
}

}  // namespace mnb
