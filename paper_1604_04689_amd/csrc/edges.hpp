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

#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "launch.hpp"
#include "csr.hpp"
#include "internal.hpp"
#include "radix.hpp"

namespace mnb {

constexpr int EDGE_BLOCK = 256;  // vertices per block in transpose and merge
constexpr int KH_BLOCK = 512;
constexpr int KH_GRID_MAX = 1024;
constexpr int MAX_KH_PASS = 4;  // 31 vertex bits

// With BATCH, row vertices are global (vert_off[m] + local) and neighbour
// ids local to the mesh: the transposed key is then
// ((vert_off + w) << b) | (v - vert_off), the mesh of v found among the
// segment records (vert_off non-decreasing; a vertex with rows belongs to a
// mesh with vertices).
template <bool BATCH>
static __global__ __launch_bounds__(EDGE_BLOCK) void edge_transpose_kernel(const int32_t* __restrict__ up_ptr,
                                                                         const int32_t* __restrict__ deg,
                                                                         const int64_t* __restrict__ src,
                                                                         const int32_t* __restrict__ temp,
                                                                         int32_t n_vert, uint32_t b,
                                                                         const mesh_segment* __restrict__ segs,
                                                                         int32_t n_mesh,
                                                                         uint64_t* __restrict__ tkeys,
                                                                         int32_t* __restrict__ up_cols) {
    __shared__ int32_t s_start[EDGE_BLOCK + 1];
    __shared__ int64_t s_src[EDGE_BLOCK];
    __shared__ int32_t s_voff[EDGE_BLOCK];
    const int tid = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * EDGE_BLOCK;
    const int nv = (int)tmin<int64_t>(EDGE_BLOCK, (int64_t)n_vert - v0);
    if (tid < nv) {
        s_start[tid] = up_ptr[v0 + tid];
        s_src[tid] = deg[v0 + tid] > 0 ? src[v0 + tid] : 0;
        int32_t voff = 0;
        if (BATCH) {  // largest m with vert_off[m] <= v
            const int64_t v = v0 + tid;
            int lo = 0, hi = n_mesh - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (segs[mid].vert_off <= v) lo = mid;
                else hi = mid - 1;
            }
            voff = segs[lo].vert_off;
        }
        s_voff[tid] = voff;
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
        const int32_t voff = s_voff[lo];
        tkeys[i] = ((uint64_t)(uint32_t)(voff + w) << b) | (uint64_t)(v0 + lo - voff);
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

// row_ptr and cols of the node relation from the lower groups (low_cols,
// each vertex's lower neighbours from low_ptr[v]) and the higher rows (up_cols
// from up_ptr[v]).
static __global__ __launch_bounds__(EDGE_BLOCK) void edge_merge_kernel(const int32_t* __restrict__ low_ptr,
                                                                     const int32_t* __restrict__ up_ptr,
                                                                     const int32_t* __restrict__ low_cols,
                                                                     const int32_t* __restrict__ up_cols,
                                                                     int32_t n_vert,
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
    for (int64_t i = a + tid; i < e; i += EDGE_BLOCK) {
        int lo = 0, hi = nv - 1;  // last row whose start <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const int o = (int)(i - s_start[lo]);
        cols[i] = o < s_nlow[lo] ? low_cols[s_low[lo] + o] : up_cols[s_up[lo] + (o - s_nlow[lo])];
    }
}

// Everything after the rows stage of the edge-rows algorithm.  up_ptr holds
// the scan of the higher-neighbour counts (up_ptr[n_vert] = E); keys[2] are
// two buffers of n_edges keys each (the transposed edges ping-pong between
// them), up_cols n_edges ints, hist2 zeroed, lb[l0] cleared for n_edges keys
// and lb[l0 ^ 1] for later clearing; tickets[0 .. n_pass) zero.  temp (the
// row values, dead once transposed) takes the lower neighbours, written by
// the last pass with their group starts in low_ptr (n_vert + 1 ints, set to
// INT32_MAX by the caller); block_min holds ceil((n_vert + 1) / RF_TILE) ints.
struct EdgeStage {
    const int32_t* up_ptr;
    const int32_t* deg;
    const int64_t* src;
    int32_t* temp;
    int32_t n_vert;
    uint32_t b;
    const mesh_segment* segs;  // batches (null for one mesh)
    int32_t n_mesh;
    int64_t n_edges;
    uint64_t* keys[2];
    int32_t* up_cols;
    uint32_t* hist2;
    uint64_t* lb[2];
    int l0;
    uint32_t* tickets;
    int shape;
    PassPlan pp;  // passes over the vertex bits of the transposed keys
    int32_t* low_ptr;
    int32_t* block_min;
    uint32_t* err;
};

static inline hipError_t launch_edge_stage(const EdgeStage& g, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                                           hipStream_t s) {
    const bool batch = g.segs != nullptr;
    const int32_t* E = g.up_ptr + g.n_vert;
    const unsigned vgrid = (unsigned)ceil_div((int64_t)g.n_vert, EDGE_BLOCK);
    const int n_pass = g.pp.n_pass;
    const uint32_t last_bits = g.pp.width[n_pass - 1];
    hipError_t e =
        batch ? launch("batch_node_edge_transpose", edge_transpose_kernel<true>, dim3(vgrid), dim3(EDGE_BLOCK), s,
                       g.up_ptr, g.deg, g.src, g.temp, g.n_vert, g.b, g.segs, g.n_mesh, g.keys[0], g.up_cols)
              : launch("node_edge_transpose", edge_transpose_kernel<false>, dim3(vgrid), dim3(EDGE_BLOCK), s,
                       g.up_ptr, g.deg, g.src, g.temp, g.n_vert, g.b, g.segs, g.n_mesh, g.keys[0], g.up_cols);
    if (e == hipSuccess)
        e = launch(batch ? "batch_node_edge_hist" : "node_edge_hist", key_hist_kernel,
                   dim3((unsigned)tmin<int64_t>(ceil_div(g.n_edges, KH_BLOCK), KH_GRID_MAX)), dim3(KH_BLOCK), s,
                   (const uint64_t*)g.keys[0], E, g.b, n_pass, last_bits, g.hist2);
    // the last pass writes the lower neighbours (low bits) and offers the
    // start of each vertex's group
    const CsrOut low{g.temp, g.low_ptr, g.n_edges, g.b, (1ull << g.b) - 1};
    const char* rname = batch ? "batch_node_edge_radix" : "node_edge_radix";
    for (int q = 0; q < n_pass && e == hipSuccess; ++q) {
        const uint32_t shift = g.b + g.pp.shift[q];
        const uint32_t bits = g.pp.width[q];
        const int l = g.l0 ^ (q & 1);  // look-back array, cleared by the previous pass
        const CountedKeySrc src{g.keys[q & 1], (const uint32_t*)E};
        if (q + 1 < n_pass)
            e = launch_radix_pass(rname, g.shape, src, g.keys[(q + 1) & 1], g.n_edges, shift, bits,
                                  g.hist2 + q * RADIX, g.lb[l], g.lb[l ^ 1], g.tickets + q, g.err, s);
        else
            e = launch_radix_pass(rname, g.shape, src, low, g.n_edges, shift, bits, g.hist2 + q * RADIX, g.lb[l],
                                  nullptr, g.tickets + q, g.err, s);
    }
    if (e == hipSuccess)
        e = launch_rowptr_fill(batch ? "batch_node_edge_low_fill" : "node_edge_low_fill", g.low_ptr, g.n_vert,
                               (const uint32_t*)E, g.block_min, s);
    if (e == hipSuccess)
        e = launch(batch ? "batch_node_edge_merge" : "node_edge_merge", edge_merge_kernel, dim3(vgrid),
                   dim3(EDGE_BLOCK), s, (const int32_t*)g.low_ptr, g.up_ptr, (const int32_t*)g.temp,
                   (const int32_t*)g.up_cols, g.n_vert, row_ptr, cols, cols_cap, g.err);
    return e;
}

}  // namespace mnb
