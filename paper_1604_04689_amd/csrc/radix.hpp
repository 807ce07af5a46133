// One stable LSD radix pass over 64-bit keys (8-bit digit, or up to 11 bits in
// the wide pass below), onesweep style:
// tiles ranked in LDS, decoupled look-back across tiles, keys staged in digit
// order in LDS and written out in coalesced runs.  The key source is a
// template parameter, so the first pass of a pipeline can generate its keys
// straight from the connectivity instead of reading an emitted key array.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace mnb {

constexpr int RBITS = 8;
constexpr int RADIX = 1 << RBITS;

// Keys read from an array.  Every position holds a participating key.
struct KeyArraySrc {
    const uint64_t* __restrict__ keys;
    static constexpr bool kSkipNone = false;
    __device__ __forceinline__ uint64_t load(int64_t i) const { return keys[i]; }
};

// Keys in an array whose participating length is only known on the device:
// positions at or past *count are not read (the kernel reads the count once
// per tile, alongside the key loads).
struct CountedKeySrc {
    const uint64_t* __restrict__ keys;
    const uint32_t* __restrict__ count;
    static constexpr bool kSkipNone = true;
    __device__ __forceinline__ uint64_t load(int64_t i) const { return keys[i]; }
};

// Sources that define kStaged = true copy their tile's inputs into LDS first
// (stage); if staged(s) says the tile was staged (the same for the whole
// block), its keys are built from there with the tile's header read once
// (header, load_staged), else with load(); see NodePairSrc.
template <class S, class = void>
struct is_staged : std::false_type {};
template <class S>
struct is_staged<S, std::void_t<decltype(S::kStaged)>> : std::bool_constant<S::kStaged> {};

// Output of a pass.  KeyOut writes every key to its slot.  CsrOut, for the
// last pass of a sort by the bits above vshift (stable, so each row comes out
// in input order), writes the low part of each key to cols and the start of
// every row to row_ptr with atomicMin: a key starts a row where the high part
// changes inside a tile's run of one digit, and the first key of a run may
// start one (its predecessor lies in another tile), so it offers its slot and
// the smallest offer wins.  Every row-start write is the atomic: plain stores
// mixed with atomics on the same lines cost several times more than either.
// row_ptr must hold INT32_MAX beforehand; rows with no keys are filled in by
// rowptr_fill afterwards.
struct KeyOut {
    uint64_t* __restrict__ out;
    __device__ __forceinline__ bool put(uint64_t k, int64_t dst, int, int, const uint64_t*) const {
        out[dst] = k;
        return true;
    }
};

struct CsrOut {
    int32_t* __restrict__ cols;
    int32_t* row_ptr;
    int64_t cols_cap;
    uint32_t vshift;
    uint64_t lo_mask;
    // false: no room in cols (capacity error)
    __device__ __forceinline__ bool put(uint64_t k, int64_t dst, int i, int run_first, const uint64_t* s_keys) const {
        if (dst >= cols_cap) return false;
        cols[dst] = (int32_t)(k & lo_mask);
        const uint64_t v = k >> vshift;
        if (i == run_first || v != (s_keys[i - 1] >> vshift)) atomicMin(&row_ptr[v], (int32_t)dst);
        return true;
    }
};

template <class Src>
__device__ __forceinline__ int64_t source_limit(const Src&, int64_t n) {
    return n;
}
template <>
__device__ __forceinline__ int64_t source_limit<CountedKeySrc>(const CountedKeySrc& s, int64_t n) {
    return tmin<int64_t>(n, (int64_t)*s.count);
}

// Tile shapes the library is built with: threads per block x keys per thread.
// The LDS staging area is 8 * BLOCK * ITEMS bytes.
struct RadixShape {
    int block, items;
};
constexpr int N_RADIX_SHAPES = 7;
constexpr RadixShape RADIX_SHAPES[N_RADIX_SHAPES] = {{512, 16}, {256, 32}, {512, 12}, {512, 24},
                                                     {1024, 8}, {512, 8},  {256, 16}};
constexpr int DEFAULT_RADIX_SHAPE = 0;

// ---------------------------------------------------------------------------
// radix_pass: stable scatter of the keys by digit (key >> shift) & mask.
//
// Tile t (taken by atomic ticket, so every earlier tile is already resident)
// holds BLOCK*ITEMS source positions.  Wave w owns a contiguous run of
// 64*ITEMS positions, item j of lane l at offset j*64 + l, so (j, lane) order
// is input order.
//
// Order of work inside a tile, chosen so that the serial chain through the
// tiles (each tile's global offsets depend on all earlier tiles) is short:
//  1. load the keys and count the tile's digits with LDS atomics;
//  2. publish the tile's digit counts at once, then threads 0..255 walk back
//     over earlier tiles (decoupled look-back) for their digit's offset while
//     the other waves already rank their keys;
//  3. rank: for each item, the lanes holding the same digit are found with one
//     ballot per digit bit; the lowest such lane bumps the wave's private
//     digit counter in LDS and the others take their rank from it; wave
//     counts are then scanned in wave order (stability);
//  4. stage the keys in LDS in digit order and write them to their global
//     slots in coalesced runs.
// Each tile also clears its status slots in `lookback_next` (null for the
// last pass), the array the following pass uses.  `hist` is the global count
// of every digit value over the participating keys of the whole pass.  When
// Src::kSkipNone is set, KEY_NONE marks a position without a key.
// ---------------------------------------------------------------------------
// Waves per SIMD when as many blocks share a CU as its 160 KB of LDS allow:
// the register budget the kernel is compiled for (more registers than that
// would leave a block's worth of LDS idle).
constexpr int radix_waves_per_eu(int block, int items) {
    const int lds = 8 * block * items + (block / WAVE) * RADIX * 4 + 4 * RADIX * 4 + 256;
    int blocks = (160 * 1024) / lds;
    if (blocks < 1) blocks = 1;
    const int w = blocks * (block / WAVE) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int BLOCK, int ITEMS, class Src, class Out, class W>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(radix_waves_per_eu(BLOCK, ITEMS))))
void radix_pass_kernel(Src src, Out out, int64_t n, uint32_t shift, uint32_t bits, const uint32_t* __restrict__ hist,
                       W* lookback, W* lookback_next, uint32_t* ticket, uint32_t* err) {
    static_assert(BLOCK >= RADIX, "one thread per digit");
    constexpr int WAVES = BLOCK / WAVE;
    constexpr int TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_whist[WAVES][RADIX];
    __shared__ uint32_t s_cnt[RADIX];
    __shared__ uint32_t s_tile_off[RADIX];
    __shared__ int64_t s_glob[RADIX];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    // With a device-side count below n, only the first ceil(count / TILE)
    // blocks take tickets, so those tickets are exactly the tiles that hold
    // keys; the other blocks leave before touching the ticket counter (a
    // single-address atomic that every block would otherwise queue on).
    const int64_t limit_n = source_limit(src, n);
    if ((int64_t)blockIdx.x * TILE >= limit_n) return;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = tid; i < WAVES * RADIX; i += BLOCK) (&s_whist[0][0])[i] = 0;
    for (int i = tid; i < RADIX; i += BLOCK) s_cnt[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t tile_base = (int64_t)tile * TILE;
    const uint32_t dmask = (1u << bits) - 1;

    // ---- 1. load (lanes of a wave read 64 consecutive positions), count ------
    const int64_t wbase = tile_base + (int64_t)wid * WAVE * ITEMS + lane;
    // (No ticket reaches past the participating keys: see above.  A tile past
    // them would have nothing to place, and no tile would ever look back at it.)
    if (tile_base >= limit_n) return;
    uint64_t key[ITEMS];
    uint32_t valid_bits = 0;
    bool direct = true;
    if constexpr (is_staged<Src>::value) {
        // the staging area is free until step 4
        int32_t* s_stage = reinterpret_cast<int32_t*>(s_keys);
        src.template stage<BLOCK, TILE>(tile_base, n, s_stage, tid);
        __syncthreads();
        if (src.staged(s_stage)) {
            direct = false;
            const auto hdr = src.header(s_stage);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const int64_t idx = wbase + j * WAVE;
                key[j] = idx < n ? src.load_staged(hdr, idx, tile_base, s_stage) : KEY_NONE;
                const bool valid = idx < limit_n && !(Src::kSkipNone && key[j] == KEY_NONE);
                valid_bits |= (uint32_t)valid << j;
            }
        }
    }
    if (direct) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t idx = wbase + j * WAVE;
            // positions in [limit_n, n) lie inside the source array; they are read
            // but never take part, so the loads need not wait for the count
            key[j] = idx < n ? src.load(idx) : KEY_NONE;
            const bool valid = idx < limit_n && !(Src::kSkipNone && key[j] == KEY_NONE);
            valid_bits |= (uint32_t)valid << j;
        }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        if ((valid_bits >> j) & 1u) atomicAdd(&s_cnt[(uint32_t)(key[j] >> shift) & dmask], 1u);
    __syncthreads();

    // ---- 2. publish, tile offsets, look-back ---------------------------------
    const uint32_t tile_cnt = tid < RADIX ? s_cnt[tid] : 0u;
    if (tid < RADIX)
        lb_store(lookback + (int64_t)tile * RADIX + tid, (W)((tile == 0 ? LbWord<W>::INC : LbWord<W>::AGG) | tile_cnt));
    uint32_t tile_total;
    const uint32_t toff = block_exclusive_sum<BLOCK>(tile_cnt, s_tmp, &tile_total);
    uint32_t hist_total;
    const uint32_t gstart = block_exclusive_sum<BLOCK>(tid < RADIX ? hist[tid] : 0u, s_tmp, &hist_total);
    if (tid < RADIX) {
        s_tile_off[tid] = toff;
        const uint64_t before = lookback_prefix(lookback + tid, RADIX, tile, tile_cnt, err);
        s_glob[tid] = (int64_t)gstart + (int64_t)before - (int64_t)toff;
        if (lookback_next) lookback_next[(int64_t)tile * RADIX + tid] = 0;  // slot of the next pass (same width)
    }

    // ---- 3. rank within the wave ---------------------------------------------
    // peers = valid lanes whose digit equals this lane's, kept as two 32-bit
    // halves: per digit bit, m is all ones where the bit is set, and a lane
    // keeps the voters that agree with it, peers &= ~(vote ^ m), one
    // three-input bitwise instruction per half.  The lowest lane of each
    // digit group (the leader) reads and bumps the wave's counter for that
    // digit; the others take the old count from it by a shuffle and add their
    // rank among the group.
    const uint64_t lt_mask = (1ull << lane) - 1;
    // ranks are below TILE <= 2^16: two per register
    static_assert(TILE <= 65536, "16-bit ranks");
    uint32_t rank2[(ITEMS + 1) / 2] = {};
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = (valid_bits >> j) & 1u;
        const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
        const uint64_t vv = __ballot(valid);
        uint32_t plo = (uint32_t)vv, phi = (uint32_t)(vv >> 32);
#pragma unroll
        for (int bit = 0; bit < RBITS; ++bit) {
            uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)dg, bit, 1);
            asm("" : "+v"(m));  // keeps the vote a compare of m itself
            const uint64_t vote = __ballot(m != 0);
            plo &= ~((uint32_t)vote ^ m);
            phi &= ~((uint32_t)(vote >> 32) ^ m);
            asm("" : "+v"(plo), "+v"(phi));  // one three-input op per half
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t below = __popcll(peers & lt_mask);
        const int leader = __ffsll((unsigned long long)peers) - 1;
        uint32_t base = 0;
        if (valid && below == 0) {
            base = s_whist[wid][dg];
            s_whist[wid][dg] = base + (uint32_t)__popcll(peers);
        }
        base = __shfl(base, leader & (WAVE - 1), WAVE);
        rank2[j / 2] |= (base + below) << (16 * (j & 1));
    }
    __syncthreads();
    if (tid < RADIX) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_whist[w][tid];
            s_whist[w][tid] = run;
            run += c;
        }
    }
    __syncthreads();

    // ---- 4. stage in digit order, then write out -------------------------------
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if ((valid_bits >> j) & 1u) {
            const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
            const uint32_t rank = (rank2[j / 2] >> (16 * (j & 1))) & 0xffffu;
            s_keys[s_tile_off[dg] + s_whist[wid][dg] + rank] = key[j];
        }
    }
    __syncthreads();
    const int64_t limit = hist_total;  // participating keys of the pass = output size
    bool bad = false, full = false;
    for (int i = tid; i < (int)tile_total; i += BLOCK) {
        const uint64_t k = s_keys[i];
        const uint32_t dg = (uint32_t)(k >> shift) & dmask;
        const int64_t dst = s_glob[dg] + i;
        if ((uint64_t)dst < (uint64_t)limit) full |= !out.put(k, dst, i, (int)s_tile_off[dg], s_keys);
        else bad = true;
    }
    if (bad) set_error(err, ERR_INTERNAL);
    if (full) set_error(err, ERR_CAPACITY);
}

template <int BLOCK, int ITEMS, class Src, class Out, class W = uint32_t>
hipError_t launch_radix_shape(const char* name, Src src, Out out, int64_t n, uint32_t shift, uint32_t bits, const uint32_t* hist,
                              uint64_t* lb, uint64_t* lb_next, uint32_t* ticket, uint32_t* err, hipStream_t s) {
    const int64_t tiles = ceil_div(n, (int64_t)BLOCK * ITEMS);
    return launch(name, radix_pass_kernel<BLOCK, ITEMS, Src, Out, W>, dim3((unsigned)tiles), dim3(BLOCK), s, src,
                  out, n, shift, bits, hist, reinterpret_cast<W*>(lb), reinterpret_cast<W*>(lb_next), ticket, err);
}

// The tile shape a pass over n keys launches with when `shape` is asked
// for: passes over LB32_MAX_KEYS keys or more use 64-bit look-back words and
// only the default shape; an unknown shape is the default.  Every table sized
// by the tiles of a pass (batch tile records, histogram tiling, staged ids)
// takes its tile size from here.
inline int radix_effective_shape(int shape, int64_t n) {
    if (n >= LB32_MAX_KEYS || shape < 0 || shape >= N_RADIX_SHAPES) return DEFAULT_RADIX_SHAPE;
    return shape;
}
inline int64_t radix_tile_keys(int shape, int64_t n) {
    const RadixShape sh = RADIX_SHAPES[radix_effective_shape(shape, n)];
    return (int64_t)sh.block * sh.items;
}

// Launches one radix pass with tile shape RADIX_SHAPES[radix_effective_shape(
// shape, n)].  The look-back arrays need room for ceil(n / min_radix_tile())
// tiles.
template <class Src, class Out>
hipError_t launch_radix_pass(const char* name, int shape, Src src, Out out, int64_t n, uint32_t shift, uint32_t bits,
                             const uint32_t* hist, uint64_t* lb, uint64_t* lb_next, uint32_t* ticket, uint32_t* err,
                             hipStream_t s) {
    // The status arrays hold 64-bit words; passes over fewer than
    // LB32_MAX_KEYS keys use them as 32-bit words (every pass of one
    // pipeline has the same n, so a pass and the next agree on the width of
    // the slots they hand over).
    if (n >= LB32_MAX_KEYS)
        return launch_radix_shape<512, 16, Src, Out, uint64_t>(name, src, out, n, shift, bits, hist, lb, lb_next,
                                                               ticket, err, s);
    switch (radix_effective_shape(shape, n)) {
        case 1: return launch_radix_shape<256, 32>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        case 2: return launch_radix_shape<512, 12>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        case 3: return launch_radix_shape<512, 24>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        case 4: return launch_radix_shape<1024, 8>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        case 5: return launch_radix_shape<512, 8>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        case 6: return launch_radix_shape<256, 16>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
        default: return launch_radix_shape<512, 16>(name, src, out, n, shift, bits, hist, lb, lb_next, ticket, err, s);
    }
}

template <class Src>
hipError_t launch_radix_pass(const char* name, int shape, Src src, uint64_t* out, int64_t n, uint32_t shift,
                             uint32_t bits, const uint32_t* hist, uint64_t* lb, uint64_t* lb_next, uint32_t* ticket,
                             uint32_t* err, hipStream_t s) {
    return launch_radix_pass(name, shape, src, KeyOut{out}, n, shift, bits, hist, lb, lb_next, ticket, err, s);
}

constexpr int min_radix_tile() {
    int m = RADIX_SHAPES[0].block * RADIX_SHAPES[0].items;
    for (int i = 1; i < N_RADIX_SHAPES; ++i)
        if (RADIX_SHAPES[i].block * RADIX_SHAPES[i].items < m) m = RADIX_SHAPES[i].block * RADIX_SHAPES[i].items;
    return m;
}

// ---------------------------------------------------------------------------
// radix_wide_pass: the same stable pass with digits of up to WBITS = 11 bits
// (2048 digit values), so that the vertex bits of the largest meshes here
// (20 to 22 bits) are sorted in two passes instead of three.
//
// The tile keeps the 8-bit pass's order of work; what changes is where the
// digit counters live.  Per-wave counters for 2048 digits would not fit beside
// the key staging area, so they are 16-bit and sit INSIDE the staging area,
// which is idle until the keys are staged: after ranking, every key's place in
// the tile is computed into registers, and only then are the keys written
// over the counters.  The tile's digit counts (later its digit offsets) are
// 16-bit pairs in one word, counted with 32-bit LDS atomics (a count never
// carries into its neighbour: a tile holds at most 2^16 - 1 keys); global
// offsets are 32-bit (passes of this width cover fewer than 2^30 keys).  Each
// thread owns DPT = 2048 / BLOCK consecutive digits for the look-back, walked
// together.
// ---------------------------------------------------------------------------
constexpr int WBITS = 11;
constexpr int WRADIX = 1 << WBITS;

// Exclusive prefix of the running counts of ND consecutive digits (status
// words of digit j of tile t at status[t * WRADIX + j]), walked together by
// one thread: every round requests LB_BATCH predecessors of every unfinished
// digit at once.  Publishes LB_INC | (prefix + agg) for each.
template <int ND, class W>
__device__ __forceinline__ void lookback_prefix_n(W* status, uint32_t tile, const uint32_t (&agg)[ND],
                                                  uint32_t (&prefix)[ND], uint32_t* err) {
    using L = LbWord<W>;
    constexpr int B = 2;  // predecessors per digit per round (registers are the limit here)
    int32_t t[ND];        // next tile to read; -1 once the walk is done
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        prefix[d] = 0;
        t[d] = (int32_t)tile - 1;
    }
    uint32_t spins = 0;
    while (true) {
        W s[ND][B];
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int k = 0; k < B; ++k)
                s[d][k] = t[d] - k >= 0 ? lb_load(status + (int64_t)(t[d] - k) * WRADIX + d) : L::INC;
        bool stalled = false, all = true;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            bool stop = t[d] < 0;
#pragma unroll
            for (int k = 0; k < B; ++k) {
                if (stop) continue;
                const W f = s[d][k] & L::FLAG;
                if (f == 0) {  // resume this digit's walk at this tile
                    stop = true;
                    stalled = true;
                    continue;
                }
                prefix[d] += (uint32_t)(s[d][k] & L::VAL);
                t[d] = f == L::INC ? -1 : t[d] - 1;
                stop = t[d] < 0;
            }
            all &= t[d] < 0;
        }
        if (all) break;
        if (stalled) {
            if (lookback_give_up(++spins, err)) {
                set_error(err, ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) lb_store(status + (int64_t)tile * WRADIX + d, (W)(L::INC | (W)(prefix[d] + agg[d])));
}

template <int BLOCK, int ITEMS, class Src, class Out>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(radix_waves_per_eu(BLOCK, ITEMS))))
void radix_wide_kernel(Src src, Out out, int64_t n, uint32_t shift, uint32_t bits, const uint32_t* __restrict__ hist,
                       uint32_t* lookback, uint32_t* lookback_next, uint32_t* ticket, uint32_t* err) {
    constexpr int WAVES = BLOCK / WAVE;
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int DPT = WRADIX / BLOCK;  // digits per thread
    static_assert(WRADIX % BLOCK == 0 && DPT % 2 == 0, "whole digit pairs per thread");
    static_assert(WAVES * WRADIX * 2 <= TILE * 8, "16-bit wave counters fit the staging area");
    static_assert(TILE < 65536, "16-bit counts and places");
    using L = LbWord<uint32_t>;
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_cnt2[WRADIX / 2];  // 16-bit digit counts, then digit offsets, two per word
    __shared__ int32_t s_glob[WRADIX];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile;
    uint16_t* s_wc = reinterpret_cast<uint16_t*>(s_keys);  // [WAVES][WRADIX] while ranking

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wid = tid / WAVE;
    const int64_t limit_n = source_limit(src, n);
    if ((int64_t)blockIdx.x * TILE >= limit_n) return;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = tid; i < WRADIX / 2; i += BLOCK) s_cnt2[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t tile_base = (int64_t)tile * TILE;
    const uint32_t dmask = (1u << bits) - 1;

    // ---- 1. load, count ---------------------------------------------------------
    const int64_t wbase = tile_base + (int64_t)wid * WAVE * ITEMS + lane;
    if (tile_base >= limit_n) return;
    uint64_t key[ITEMS];
    uint32_t valid_bits = 0;
    bool direct = true;
    if constexpr (is_staged<Src>::value) {
        int32_t* s_stage = reinterpret_cast<int32_t*>(s_keys);
        src.template stage<BLOCK, TILE>(tile_base, n, s_stage, tid);
        __syncthreads();
        if (src.staged(s_stage)) {
            direct = false;
            const auto hdr = src.header(s_stage);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const int64_t idx = wbase + j * WAVE;
                key[j] = idx < n ? src.load_staged(hdr, idx, tile_base, s_stage) : KEY_NONE;
                const bool valid = idx < limit_n && !(Src::kSkipNone && key[j] == KEY_NONE);
                valid_bits |= (uint32_t)valid << j;
            }
        }
        __syncthreads();  // the staged ids are read: the area takes the wave counters
    }
    if (direct) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t idx = wbase + j * WAVE;
            key[j] = idx < n ? src.load(idx) : KEY_NONE;
            const bool valid = idx < limit_n && !(Src::kSkipNone && key[j] == KEY_NONE);
            valid_bits |= (uint32_t)valid << j;
        }
    }
    {
        uint32_t* w32 = reinterpret_cast<uint32_t*>(s_wc);
        for (int i = tid; i < WAVES * WRADIX / 2; i += BLOCK) w32[i] = 0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if ((valid_bits >> j) & 1u) {
            const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
            atomicAdd(&s_cnt2[dg >> 1], 1u << (16 * (dg & 1)));
        }
    }
    __syncthreads();

    // ---- 2. publish, tile offsets, look-back -----------------------------------
    // thread tid owns digits d0 .. d0 + DPT - 1
    const int d0 = tid * DPT;
    uint32_t cnt[DPT], hq[DPT];
    uint32_t mine = 0, gmine = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        cnt[j] = (s_cnt2[(d0 + j) >> 1] >> (16 * ((d0 + j) & 1))) & 0xffffu;
        lb_store(lookback + (int64_t)tile * WRADIX + d0 + j, (uint32_t)((tile == 0 ? L::INC : L::AGG) | cnt[j]));
        hq[j] = hist[d0 + j];
        mine += cnt[j];
        gmine += hq[j];
    }
    uint32_t tile_total, hist_total;
    uint32_t toff = block_exclusive_sum<BLOCK>(mine, s_tmp, &tile_total);
    uint32_t gstart = block_exclusive_sum<BLOCK>(gmine, s_tmp, &hist_total);
    uint32_t before[DPT];
    lookback_prefix_n<DPT>(lookback + d0, tile, cnt, before, err);
#pragma unroll
    for (int j = 0; j < DPT; j += 2) {  // this thread's own words of s_cnt2: no other thread reads them yet
        s_cnt2[(d0 + j) >> 1] = toff | ((toff + cnt[j]) << 16);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s_glob[d0 + j + h] = (int32_t)(gstart + before[j + h]) - (int32_t)toff;
            toff += cnt[j + h];
            gstart += hq[j + h];
        }
        if (lookback_next) {
            lookback_next[(int64_t)tile * WRADIX + d0 + j] = 0;
            lookback_next[(int64_t)tile * WRADIX + d0 + j + 1] = 0;
        }
    }

    // ---- 3. rank within the wave (as in radix_pass, over WBITS digit bits),
    // the wave counters 16-bit in the staging area --------------------------------
    const uint64_t lt_mask = (1ull << lane) - 1;
    uint32_t rank2[(ITEMS + 1) / 2] = {};
    uint16_t* wc = s_wc + wid * WRADIX;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = (valid_bits >> j) & 1u;
        const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
        const uint64_t vv = __ballot(valid);
        uint32_t plo = (uint32_t)vv, phi = (uint32_t)(vv >> 32);
#pragma unroll
        for (int bit = 0; bit < WBITS; ++bit) {
            uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)dg, bit, 1);
            asm("" : "+v"(m));
            const uint64_t vote = __ballot(m != 0);
            plo &= ~((uint32_t)vote ^ m);
            phi &= ~((uint32_t)(vote >> 32) ^ m);
            asm("" : "+v"(plo), "+v"(phi));
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t below = __popcll(peers & lt_mask);
        const int leader = __ffsll((unsigned long long)peers) - 1;
        uint32_t base = 0;
        if (valid && below == 0) {
            base = wc[dg];
            wc[dg] = (uint16_t)(base + (uint32_t)__popcll(peers));
        }
        base = __shfl(base, leader & (WAVE - 1), WAVE);
        rank2[j / 2] |= (base + below) << (16 * (j & 1));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DPT; ++j) {  // wave counts of each digit scanned in wave order (stability)
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_wc[w * WRADIX + d0 + j];
            s_wc[w * WRADIX + d0 + j] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();

    // ---- 4. places in the tile, then the keys staged in digit order over the
    // counters, then written out ------------------------------------------------
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {  // rank -> place, in the same 16 bits
        if ((valid_bits >> j) & 1u) {
            const uint32_t dg = (uint32_t)(key[j] >> shift) & dmask;
            const uint32_t off = (s_cnt2[dg >> 1] >> (16 * (dg & 1))) & 0xffffu;
            rank2[j / 2] += (off + (uint32_t)wc[dg]) << (16 * (j & 1));
        }
    }
    __syncthreads();  // every counter is read: the area takes the keys
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        if ((valid_bits >> j) & 1u) s_keys[(rank2[j / 2] >> (16 * (j & 1))) & 0xffffu] = key[j];
    __syncthreads();
    const int64_t limit = hist_total;  // participating keys of the pass = output size
    bool bad = false, full = false;
    for (int i = tid; i < (int)tile_total; i += BLOCK) {
        const uint64_t k = s_keys[i];
        const uint32_t dg = (uint32_t)(k >> shift) & dmask;
        const int64_t dst = (int64_t)s_glob[dg] + i;
        const int run_first = (int)((s_cnt2[dg >> 1] >> (16 * (dg & 1))) & 0xffffu);
        if ((uint64_t)dst < (uint64_t)limit) full |= !out.put(k, dst, i, run_first, s_keys);
        else bad = true;
    }
    if (bad) set_error(err, ERR_INTERNAL);
    if (full) set_error(err, ERR_CAPACITY);
}

constexpr int WIDE_BLOCK = 512, WIDE_ITEMS = 16;
constexpr int WIDE_TILE = WIDE_BLOCK * WIDE_ITEMS;

// Launches one wide pass (bits <= WBITS) over n < LB32_MAX_KEYS keys.  The
// look-back arrays need room for ceil(n / WIDE_TILE) * WRADIX 32-bit words;
// the histogram holds WRADIX words.
template <class Src, class Out>
hipError_t launch_radix_wide(const char* name, Src src, Out out, int64_t n, uint32_t shift, uint32_t bits,
                             const uint32_t* hist, uint64_t* lb, uint64_t* lb_next, uint32_t* ticket, uint32_t* err,
                             hipStream_t s) {
    if (n >= LB32_MAX_KEYS || bits > (uint32_t)WBITS) return hipErrorInvalidValue;
    return launch(name, radix_wide_kernel<WIDE_BLOCK, WIDE_ITEMS, Src, Out>, dim3((unsigned)ceil_div(n, WIDE_TILE)),
                  dim3(WIDE_BLOCK), s, src, out, n, shift, bits, hist, reinterpret_cast<uint32_t*>(lb),
                  reinterpret_cast<uint32_t*>(lb_next), ticket, err);
}

// Look-back bytes per array of a sort over n keys with either pass width.
inline size_t radix_lookback_bytes(int64_t n, bool wide) {
    const size_t narrow = (size_t)ceil_div(n, (int64_t)min_radix_tile()) * RADIX * sizeof(uint64_t);
    if (!wide) return narrow;
    const size_t w = (size_t)ceil_div(n, (int64_t)WIDE_TILE) * WRADIX * sizeof(uint32_t);
    return w > narrow ? w : narrow;
}

}  // namespace mnb
