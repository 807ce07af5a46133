// Device building blocks shared by the node and element pipelines: error
// word, decoupled look-back status words, wave64 and block prefix sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mnb {

constexpr int WAVE = 64;

// Bits of the device error word (first word of every workspace).
constexpr uint32_t ERR_INDEX_RANGE = 1u;  // a connectivity id outside [0, n_vert)
constexpr uint32_t ERR_CAPACITY = 2u;     // more nnz than the cols capacity
constexpr uint32_t ERR_INTERNAL = 4u;     // a look-back wait gave up / bad offset

// Key value of a pair that is not an edge (self pair, bad id): all ones, so it
// sorts after every real key on any digit split, and is dropped at the end.
constexpr uint64_t KEY_NONE = ~0ull;

// Workspace header: error word, tile tickets, counters (bytes).
constexpr size_t HEADER_BYTES = 256;
constexpr int HDR_ERR = 0;          // u32 index of the error word
constexpr int HDR_TICKET0 = 4;      // u32 index of the first tile ticket
constexpr int N_TICKETS = 16;
constexpr int HDR_LONG_COUNT = 32;  // u32 index of the long-row counter
constexpr int HDR_KEY_COUNT = 33;   // u32 index of a device-side key count
constexpr int HDR_TILE_LISTS = 40;  // u32 index of the batch stage's tile-list counts (7 words)

// Decoupled look-back status word: 2 flag bits over a 62-bit value.
constexpr uint64_t LB_AGG = 1ull << 62;  // value = this tile's own count
constexpr uint64_t LB_INC = 2ull << 62;  // value = count of this and all earlier tiles
constexpr uint64_t LB_FLAG = 3ull << 62;
constexpr uint64_t LB_VAL = ~LB_FLAG;

// The radix passes' status words come in two widths: 32 bits (2 flag bits
// over a 30-bit count) for passes over fewer than LB32_MAX_KEYS keys, which
// halves the look-back traffic, and 64 bits beyond.
template <class W>
struct LbWord;
template <>
struct LbWord<uint64_t> {
    static constexpr uint64_t AGG = LB_AGG, INC = LB_INC, FLAG = LB_FLAG, VAL = LB_VAL;
};
template <>
struct LbWord<uint32_t> {
    static constexpr uint32_t AGG = 1u << 30, INC = 2u << 30, FLAG = 3u << 30, VAL = ~(3u << 30);
};
constexpr int64_t LB32_MAX_KEYS = (int64_t)1 << 30;

// A look-back wait polls at most this many times (about a second with the
// sleep below) before it records ERR_INTERNAL and moves on, so every wave of
// every kernel always terminates.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

template <class W>
__device__ __forceinline__ W lb_load(const W* p) {
    return __hip_atomic_load(const_cast<W*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class W>
__device__ __forceinline__ void lb_store(W* p, W v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_error(uint32_t* err, uint32_t bit) {
    atomicOr(err, bit);
}

__device__ __forceinline__ bool lookback_give_up(uint32_t spins, uint32_t* err) {
    // give up after SPIN_LIMIT polls, or at once when another wait already
    // gave up (so a failure cannot chain into long waits)
    return spins > SPIN_LIMIT ||
           ((spins & 1023u) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_INTERNAL));
}

// Exclusive prefix over the tiles before `tile` of one running count whose
// status words sit `stride` apart (status[t * stride]), walked by one thread.
// The statuses of LB_BATCH predecessors are requested together, so one memory
// round trip covers LB_BATCH steps of the walk.  The caller has already
// published LB_AGG | agg for this tile (or LB_INC for tile 0).  Tiles are
// handed out in launch order by an atomic ticket, so every earlier tile is
// resident and the walk finishes.  Publishes LB_INC | (prefix + agg).
constexpr int LB_BATCH = 4;

template <class W>
__device__ __forceinline__ uint64_t lookback_prefix(W* status, int64_t stride, uint32_t tile, uint64_t agg,
                                                    uint32_t* err) {
    using L = LbWord<W>;
    if (tile == 0) return 0;
    uint64_t prefix = 0;
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (t >= 0) {
        W s[LB_BATCH];
#pragma unroll
        for (int k = 0; k < LB_BATCH; ++k) s[k] = t - k >= 0 ? lb_load(status + (t - k) * stride) : L::INC;
        bool stalled = false, done = false;
#pragma unroll
        for (int k = 0; k < LB_BATCH; ++k) {
            if (done || stalled) continue;
            const W f = s[k] & L::FLAG;
            if (f == 0) {
                stalled = true;  // resume the walk at this tile
                continue;
            }
            prefix += s[k] & L::VAL;
            --t;
            done = f == L::INC || t < 0;
        }
        if (done) break;
        if (stalled) {
            if (lookback_give_up(++spins, err)) {
                set_error(err, ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    lb_store(status + (int64_t)tile * stride, (W)(L::INC | (W)(prefix + agg)));
    return prefix;
}

// The same for a single running count, walked by a whole wave: lane l reads
// the status of tile (t - l), the wave finds the nearest inclusive value with
// a ballot and sums the window with a wave reduction.  Every lane of the wave
// must call it; all lanes return the prefix, lane 0 publishes.
__device__ __forceinline__ uint64_t wave_lookback_prefix(uint64_t* status, uint32_t tile, uint64_t agg,
                                                         uint32_t* err) {
    const int lane = __lane_id();
    if (tile == 0) return 0;
    uint64_t prefix = 0;
    int64_t t = (int64_t)tile - 1;  // newest tile of the window
    uint32_t spins = 0;
    while (true) {
        const int64_t mine = t - lane;
        const uint64_t s = mine >= 0 ? lb_load(status + mine) : LB_INC;
        const uint64_t f = s & LB_FLAG;
        const uint64_t inc = __ballot(f == LB_INC);
        const uint64_t none = __ballot(f == 0);
        // lanes up to and including the first inclusive one must be ready
        const uint64_t upto = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;  // lanes 0..first INC
        if (none & upto) {
            if (lookback_give_up(++spins, err)) {
                if (lane == 0) set_error(err, ERR_INTERNAL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = ((upto >> lane) & 1) ? (s & LB_VAL) : 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
        prefix += v;
        if (inc) break;
        t -= WAVE;
    }
    if (lane == 0) lb_store(status + tile, LB_INC | (prefix + agg));
    return prefix;
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive prefix sum of one value per thread across the block, in thread
// order; *total receives the block sum.  s_tmp needs BLOCK/64 entries.
// Contains __syncthreads: every thread of the block must call it.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* s_tmp, T* total) {
    constexpr int WAVES = BLOCK / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    T x = wave_inclusive_sum(v);
    if (lane == WAVE - 1) s_tmp[wid] = x;
    __syncthreads();
    T before = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        T t = s_tmp[w];
        before += (w < wid) ? t : T(0);
        sum += t;
    }
    __syncthreads();
    *total = sum;
    return before + x - v;
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T>
__host__ __device__ constexpr T tmin(T a, T b) {
    return a < b ? a : b;
}

template <typename T>
__host__ __device__ constexpr T tmax(T a, T b) {
    return a < b ? b : a;
}

}  // namespace mnb
