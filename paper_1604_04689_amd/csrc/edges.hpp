// Edge-rows node algorithm, after the rows stage has run over the canonical
// edge keys (min << b) | max sorted by min: for every vertex v the distinct
// higher neighbours are in temp[src[v] .. src[v] + deg[v]) (ascending) and
// up_ptr is their exclusive scan, up_ptr[V] = E unique edges.
//   edge_transpose  each unique edge (v, w), v < w, as the key (w << b) | v in
//                   v-then-w order, and w alone into up_cols;
//   key_hist        digit histograms of those keys over the bits of w;
//   (radix passes over the bits of w: stable, so the v of one w stay ascending)
//   low_ptr         start of every vertex's group of lower neighbours;
//   edge_merge      row u = its lower neighbours, then its higher ones, both
//                   ascending and every lower one below u, every higher one
//                   above it; row_ptr[u] = low_ptr[u] + up_ptr[u].
// This is the paper's pair sort (Sec. 2.2.1) with each undirected edge sorted
// once instead of twice.
#pragma once

#include "common.hpp"
#include "launch.hpp"
#include "radix.hpp"

namespace mnb {

constexpr int EDGE_BLOCK = 256;  // vertices per block in transpose and merge
constexpr int KH_BLOCK = 512;
constexpr int KH_GRID_MAX = 1024;
constexpr int LOWPTR_BLOCK = 256;
constexpr int MAX_KH_PASS = 4;  // 31 vertex bits

static __global__ __launch_bounds__(EDGE_BLOCK) void edge_transpose_kernel(const int32_t* __restrict__ up_ptr,
                                                                         const int32_t* __restrict__ deg,
                                                                         const int64_t* __restrict__ src,
                                                                         const int32_t* __restrict__ temp,
                                                                         int32_t n_vert, uint32_t b,
                                                                         uint64_t* __restrict__ tkeys,
                                                                         int32_t* __restrict__ up_cols) {
    __shared__ int32_t s_start[EDGE_BLOCK + 1];
    __shared__ int64_t s_src[EDGE_BLOCK];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * EDGE_BLOCK;
    const int nv = (int)tmin<int64_t>(EDGE_BLOCK, (int64_t)n_vert - v0);
    if (tid < nv) {
        s_start[tid] = up_ptr[v0 + tid];
        s_src[tid] = deg[v0 + tid] > 0 ? src[v0 + tid] : 0;
    }
    if (tid == 0) s_start[nv] = up_ptr[v0 + nv];
    __syncthreads();
    const int64_t a = s_start[0], e = s_start[nv];
    for (int64_t i = a + tid; i < e; i += EDGE_BLOCK) {  // consecutive outputs on consecutive threads
        int lo = 0, hi = nv - 1;  // last row whose start <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const int32_t w = temp[s_src[lo] + (i - s_start[lo])];
        tkeys[i] = ((uint64_t)(uint32_t)w << b) | (uint64_t)(v0 + lo);
        up_cols[i] = w;
    }
}

// Digit histograms (from bit shift0) of keys[0 .. *count).
static __global__ __launch_bounds__(KH_BLOCK) void key_hist_kernel(const uint64_t* __restrict__ keys,
                                                                   const int32_t* __restrict__ count,
                                                                   uint32_t shift0, int n_pass, uint32_t last_bits,
                                                                   uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_hist[MAX_KH_PASS * RADIX];
    const int tid = threadIdx.x;
    for (int i = tid; i < n_pass * RADIX; i += KH_BLOCK) s_hist[i] = 0;
    __syncthreads();
    const int64_t n = *count;
    const int64_t stride = (int64_t)gridDim.x * KH_BLOCK;
    for (int64_t i0 = (int64_t)blockIdx.x * KH_BLOCK + tid; i0 < n; i0 += 4 * stride) {
        uint64_t k[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) k[u] = i0 + u * stride < n ? keys[i0 + u * stride] : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i0 + u * stride >= n) continue;
            for (int p = 0; p < n_pass; ++p) {
                const uint32_t mask = p == n_pass - 1 ? (1u << last_bits) - 1 : RADIX - 1;
                atomicAdd(&s_hist[p * RADIX + ((uint32_t)(k[u] >> (shift0 + p * RBITS)) & mask)], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < n_pass * RADIX; i += KH_BLOCK)
        if (s_hist[i]) atomicAdd(&hist[i], s_hist[i]);
}

// low_ptr[v] = first index of the keys (sorted by hi = key >> b) whose hi is
// at least v, for v in [0, n_vert]; the keys are keys[0 .. *count).  A
// position where hi changes writes the entries of the vertices it passes.
static __global__ __launch_bounds__(LOWPTR_BLOCK) void low_ptr_kernel(const uint64_t* __restrict__ keys,
                                                                     int64_t n_cap, const int32_t* __restrict__ count,
                                                                     uint32_t b, int32_t n_vert,
                                                                     int32_t* __restrict__ low_ptr) {
    const int64_t n = *count;
    const int64_t stride = (int64_t)gridDim.x * LOWPTR_BLOCK;
    const int64_t gid = (int64_t)blockIdx.x * LOWPTR_BLOCK + threadIdx.x;
    if (n == 0) {  // no edges: every group is empty
        for (int64_t v = gid; v <= n_vert; v += stride) low_ptr[v] = 0;
        return;
    }
    for (int64_t i = gid; i < n && i < n_cap; i += stride) {
        const int64_t w = (int64_t)(keys[i] >> b);
        const int64_t prev = i > 0 ? (int64_t)(keys[i - 1] >> b) : -1;
        if (w != prev)
            for (int64_t v = prev + 1; v <= w && v <= n_vert; ++v) low_ptr[v] = (int32_t)i;
        if (i == n - 1)
            for (int64_t v = w + 1; v <= n_vert; ++v) low_ptr[v] = (int32_t)n;
    }
}

// row_ptr and cols of the node relation from the lower groups (sorted
// transposed keys) and the higher rows (up_cols).
static __global__ __launch_bounds__(EDGE_BLOCK) void edge_merge_kernel(const int32_t* __restrict__ low_ptr,
                                                                     const int32_t* __restrict__ up_ptr,
                                                                     const uint64_t* __restrict__ tsorted,
                                                                     const int32_t* __restrict__ up_cols,
                                                                     int32_t n_vert, uint32_t b,
                                                                     int32_t* __restrict__ row_ptr,
                                                                     int32_t* __restrict__ cols, int64_t cols_cap,
                                                                     uint32_t* err) {
    __shared__ int32_t s_start[EDGE_BLOCK + 1];
    __shared__ int32_t s_low[EDGE_BLOCK];
    __shared__ int32_t s_nlow[EDGE_BLOCK];
    __shared__ int32_t s_up[EDGE_BLOCK];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * EDGE_BLOCK;
    const int nv = (int)tmin<int64_t>(EDGE_BLOCK, (int64_t)n_vert - v0);
    if (tid < nv) {
        const int64_t v = v0 + tid;
        const int32_t lo = low_ptr[v], lo1 = low_ptr[v + 1], up = up_ptr[v];
        s_start[tid] = lo + up;
        s_low[tid] = lo;
        s_nlow[tid] = lo1 - lo;
        s_up[tid] = up;
        row_ptr[v] = lo + up;
    }
    if (tid == 0) {
        s_start[nv] = low_ptr[v0 + nv] + up_ptr[v0 + nv];
        if (v0 + nv == n_vert) row_ptr[n_vert] = s_start[nv];
    }
    __syncthreads();
    const int64_t a = s_start[0], e = s_start[nv];
    if (e > cols_cap) {
        if (tid == 0) set_error(err, ERR_CAPACITY);
        return;
    }
    const uint64_t lo_mask = (1ull << b) - 1;
    for (int64_t i = a + tid; i < e; i += EDGE_BLOCK) {
        int lo = 0, hi = nv - 1;  // last row whose start <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const int o = (int)(i - s_start[lo]);
        cols[i] = o < s_nlow[lo] ? (int32_t)(tsorted[s_low[lo] + o] & lo_mask) : up_cols[s_up[lo] + (o - s_nlow[lo])];
    }
}

}  // namespace mnb
